"""Synthetic crater meshes and sun directions (seeded, deterministic).

Recipes
-------
Spherical-cap crater (paper section 7 geometry, with the depth/diameter
ratio and rim radius of the workloads used here):
  * rim radius ``rc``, depth ``d = depth_ratio * 2 rc``; the bowl is a piece
    of the sphere of radius ``r = (rc^2 + d^2) / (2 d)`` centred at
    ``(0, 0, r - d)``, so the surface is ``z = (r - d) - sqrt(r^2 - rho^2)``.
  * points: a square grid of spacing ``h`` jittered by ``U(-0.3h, 0.3h)``
    (seeded), kept where ``rho < rc - h/2``, plus a ring of rim points at
    arc spacing ``h``; every point is lifted onto the sphere.
  * faces: the lower convex hull of the lifted points (faces whose outward
    hull normal points down), wound so that facet normals point into the
    crater.  The bowl is therefore convex from inside.

Synthetic polar terrain (stand-in for a lunar DEM):
  * ``(n+1) x (n+1)`` vertices at spacing ``dx``;
  * spectral fractional Brownian surface, power ``|k|^-(2H+2)``, DC removed,
    rescaled to the requested RMS height (seeded);
  * a spherical-cap bowl of diameter ``D`` and depth ratio 0.2 added at the
    centre;
  * two triangles per pixel with the fixed diagonal (i,j)-(i+1,j+1), normals
    up.

Closed bilobed body (stand-in for a comet shape model):
  * an icosahedron subdivided ``level`` times (each triangle into four, new
    vertices projected onto the unit sphere), faces wound so that normals
    point outward;
  * every vertex ``u`` moved to radius ``radius (1 + neck cos 2 theta)`` with
    ``cos theta = u_z``: two lobes joined by a concave waist at the equator
    (``neck`` = 0 gives the sphere).

Sun directions: unit vectors ``(cos e cos phi, cos e sin phi, sin e)`` with
``phi`` counter-clockwise from +x and ``e`` the elevation above the
horizontal plane.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.spatial import ConvexHull


@dataclass(frozen=True)
class CapSpec:
    h: float                 # grid spacing (m)
    rc: float = 1000.0       # rim radius (m)
    depth_ratio: float = 0.2  # d / D
    seed: int = 0

    @property
    def depth(self) -> float:
        return self.depth_ratio * 2.0 * self.rc

    @property
    def sphere_radius(self) -> float:
        d = self.depth
        return (self.rc * self.rc + d * d) / (2.0 * d)


# ~1,600 facets and ~40,000 facets (grid spacings chosen for those counts)
CAP_SMALL = CapSpec(h=63.0, seed=0)
CAP_LARGE = CapSpec(h=12.53, seed=0)


def _cap_points(spec: CapSpec) -> np.ndarray:
    rng = np.random.default_rng(spec.seed)
    h, rc = spec.h, spec.rc
    n = int(np.ceil(rc / h)) + 1
    g = np.arange(-n, n + 1) * h
    gx, gy = np.meshgrid(g, g, indexing="ij")
    p = np.stack([gx.ravel(), gy.ravel()], axis=1)
    p = p + rng.uniform(-0.3 * h, 0.3 * h, size=p.shape)
    p = p[np.hypot(p[:, 0], p[:, 1]) < rc - 0.5 * h]
    m = int(np.round(2.0 * np.pi * rc / h))
    th = np.arange(m) * (2.0 * np.pi / m)
    ring = np.stack([rc * np.cos(th), rc * np.sin(th)], axis=1)
    return np.concatenate([p, ring], axis=0)


def cap_mesh(spec: CapSpec = CAP_SMALL):
    """Return ``(verts f64[nv,3], faces i32[nf,3])`` of the bowl crater."""
    p = _cap_points(spec)
    r, d = spec.sphere_radius, spec.depth
    rho2 = p[:, 0] ** 2 + p[:, 1] ** 2
    z = (r - d) - np.sqrt(np.maximum(r * r - rho2, 0.0))
    verts = np.column_stack([p, z]).astype(np.float64)
    hull = ConvexHull(verts)
    lower = hull.equations[:, 2] < -1e-12
    faces = hull.simplices[lower].astype(np.int64)
    # orient every face so that its normal points up (into the bowl)
    a, b, c = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    nz = np.cross(b - a, c - a)[:, 2]
    flip = nz < 0
    faces[flip] = faces[flip][:, [0, 2, 1]]
    # deterministic face order: by centroid x then y
    cen = verts[faces].mean(axis=1)
    order = np.lexsort((cen[:, 1], cen[:, 0]))
    faces = faces[order]
    return verts, np.ascontiguousarray(faces.astype(np.int32))


@dataclass(frozen=True)
class DemSpec:
    n: int = 256              # pixels per side (vertices: n+1)
    extent: float = 2560.0    # side length (m)
    hurst: float = 0.8
    rms: float = 30.0         # RMS of the fBm part (m)
    crater_diameter: float = 1500.0
    crater_depth_ratio: float = 0.2
    seed: int = 2

    @property
    def dx(self) -> float:
        return self.extent / self.n


DEM_256 = DemSpec(n=256, seed=2)
DEM_512 = DemSpec(n=512, extent=5120.0, seed=7)


def _fbm(m: int, hurst: float, rms: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(m)[:, None]
    ky = np.fft.rfftfreq(m)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** (-(hurst + 1.0))
    spec = amp * (rng.standard_normal(k.shape) + 1j * rng.standard_normal(k.shape))
    spec[0, 0] = 0.0
    z = np.fft.irfft2(spec, s=(m, m))
    z -= z.mean()
    z *= rms / np.sqrt(np.mean(z * z))
    return z


def dem_heights(spec: DemSpec) -> np.ndarray:
    """Vertex heights ``z[i, j]`` at ``(x, y) = (i dx, j dx)``."""
    m = spec.n + 1
    z = _fbm(m, spec.hurst, spec.rms, spec.seed)
    dx = spec.dx
    c = 0.5 * spec.extent
    g = np.arange(m) * dx - c
    gx, gy = np.meshgrid(g, g, indexing="ij")
    rho = np.hypot(gx, gy)
    rcr = 0.5 * spec.crater_diameter
    d = spec.crater_depth_ratio * spec.crater_diameter
    rs = (rcr * rcr + d * d) / (2.0 * d)
    inside = rho < rcr
    bowl = np.zeros_like(z)
    bowl[inside] = (rs - d) - np.sqrt(rs * rs - rho[inside] ** 2)
    return z + bowl


def dem_mesh(spec: DemSpec = DEM_256):
    """Return ``(verts f64[nv,3], faces i32[nf,3])`` of the terrain."""
    m = spec.n + 1
    z = dem_heights(spec)
    dx = spec.dx
    ii, jj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    verts = np.column_stack([ii.ravel() * dx, jj.ravel() * dx, z.ravel()])
    i, j = np.meshgrid(np.arange(spec.n), np.arange(spec.n), indexing="ij")
    a = (i * m + j).ravel()
    b = ((i + 1) * m + j).ravel()
    c = ((i + 1) * m + j + 1).ravel()
    d = (i * m + j + 1).ravel()
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    faces = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return verts.astype(np.float64), np.ascontiguousarray(faces.astype(np.int32))


def instance_sizes(count: int = 64, lo: int = 5000, hi: int = 60000, seed: int = 4):
    """Log-uniform facet counts for a batch of independent terrains."""
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def dem_instance(k: int, n_facets: int, extent: float = 2560.0) -> DemSpec:
    """Terrain ``k`` of the uneven batch: ~n_facets triangles on one domain."""
    cells = max(2, int(np.round(np.sqrt(n_facets / 2.0))))
    return DemSpec(n=cells, extent=extent, seed=k)


def sun_directions(count: int, elev_deg=(5.0, 30.0), seed: int = 1):
    """Random sun unit vectors, elevation ``U[elev]`` and azimuth ``U[0, 360)``."""
    rng = np.random.default_rng(seed)
    e = np.deg2rad(rng.uniform(elev_deg[0], elev_deg[1], size=count))
    phi = np.deg2rad(rng.uniform(0.0, 360.0, size=count))
    return np.column_stack([np.cos(e) * np.cos(phi), np.cos(e) * np.sin(phi), np.sin(e)])


def sun_grid_azimuth(elev_deg: float, count: int, step_deg: float):
    """Sun at a fixed elevation stepping in azimuth: ``phi_k = k * step``."""
    e = np.deg2rad(elev_deg)
    phi = np.deg2rad(np.arange(count) * step_deg)
    return np.column_stack([np.cos(e) * np.cos(phi), np.cos(e) * np.sin(phi),
                            np.full(count, np.sin(e))])


def mlp_init(sizes, seed: int = 0) -> np.ndarray:
    """Packed initial parameters of a perceptron with layer widths ``sizes``:
    per layer W (out x in, row-major) drawn U(-1/sqrt(in), 1/sqrt(in)), then a
    zero bias.  FP32 values."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        a = 1.0 / np.sqrt(fi)
        parts.append(rng.uniform(-a, a, size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


@dataclass(frozen=True)
class BodySpec:
    level: int = 3            # subdivisions of the icosahedron: 20 * 4^level faces
    radius: float = 1000.0    # mean radius (m)
    neck: float = 0.5         # waist depth, r = radius (1 + neck cos 2 theta)


def _icosphere(level: int):
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
             (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts)
    Fc = np.array(faces, dtype=np.int32)
    # wind every face outward: normal . centroid > 0 on the unit sphere
    n = np.cross(V[Fc[:, 1]] - V[Fc[:, 0]], V[Fc[:, 2]] - V[Fc[:, 0]])
    flip = np.einsum("ij,ij->i", n, V[Fc].mean(axis=1)) < 0
    Fc[flip] = Fc[flip][:, [0, 2, 1]]
    return V, Fc


def body_mesh(spec: BodySpec = BodySpec()):
    """Closed bilobed body: (verts (nv, 3) FP64, faces (nf, 3) int32), normals outward."""
    V, Fc = _icosphere(spec.level)
    r = spec.radius * (1.0 + spec.neck * (2.0 * V[:, 2] ** 2 - 1.0))
    return V * r[:, None], Fc
