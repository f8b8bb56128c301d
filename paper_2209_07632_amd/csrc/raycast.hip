// Ray casting against the mesh on the GPU: sun visibility for the insolation
// (eq. insolation) and centroid-to-centroid visibility V_ij (section 3.2).
//
// Acceleration: a uniform grid over the xy bounding box of the mesh.  Every
// triangle is listed in each cell its xy bounding box touches; each cell
// keeps the largest vertex height of its triangles.  A ray walks the cells it
// crosses in xy (Amanatides-Woo traversal), skips a cell when it passes above
// that height, and otherwise tests the cell's triangles.  A hit point lies in
// its triangle's xy box, so the walk never misses a triangle the ray hits.
//
// The ray/triangle test is Moeller-Trumbore with edges counted as hits, and is
// written without contraction so that hit decisions equal those of a plain
// FP64 evaluation of the same expressions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rad_internal.h"

namespace rad {

namespace {

__device__ __forceinline__ double mul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double add(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ double sub(double a, double b) { return __dsub_rn(a, b); }
__device__ __forceinline__ double dot3(const double *a, const double *b) {
    return add(add(mul(a[0], b[0]), mul(a[1], b[1])), mul(a[2], b[2]));
}
__device__ __forceinline__ void cross3(const double *a, const double *b, double *o) {
    o[0] = sub(mul(a[1], b[2]), mul(a[2], b[1]));
    o[1] = sub(mul(a[2], b[0]), mul(a[0], b[2]));
    o[2] = sub(mul(a[0], b[1]), mul(a[1], b[0]));
}

__device__ bool ray_tri(const double *o, const double *d, double tlo, double thi, const double *tri) {
    double e1[3] = {sub(tri[3], tri[0]), sub(tri[4], tri[1]), sub(tri[5], tri[2])};
    double e2[3] = {sub(tri[6], tri[0]), sub(tri[7], tri[1]), sub(tri[8], tri[2])};
    double pv[3];
    cross3(d, e2, pv);
    double det = dot3(e1, pv);
    if (det == 0.0) return false;
    double inv = 1.0 / det;
    double tv[3] = {sub(o[0], tri[0]), sub(o[1], tri[1]), sub(o[2], tri[2])};
    double u = mul(dot3(tv, pv), inv);
    if (u < 0.0 || u > 1.0) return false;
    double qv[3];
    cross3(tv, e1, qv);
    double v = mul(dot3(d, qv), inv);
    if (v < 0.0 || add(u, v) > 1.0) return false;
    double t = mul(dot3(e2, qv), inv);
    return t > tlo && t < thi;
}

struct GridView {
    const double *tri;        // N x 9, tree order
    const int32_t *cell_start;
    const int32_t *cell_tris;
    const double *cell_zmax;
    double x0, y0, h;         // origin and cell size
    double ztop;              // highest vertex of the mesh
    int32_t gx, gy;
};

// Does the ray o + t d, t in (tlo, thi), hit a triangle other than skip1/skip2?
__device__ bool occluded(const GridView &G, const double *o, const double *d, double tlo, double thi,
                         int64_t skip1, int64_t skip2) {
    int cx = (int)floor((o[0] - G.x0) / G.h);
    int cy = (int)floor((o[1] - G.y0) / G.h);
    cx = min(max(cx, 0), G.gx - 1);
    cy = min(max(cy, 0), G.gy - 1);
    const double inf = __builtin_huge_val();
    int sx = d[0] > 0 ? 1 : (d[0] < 0 ? -1 : 0);
    int sy = d[1] > 0 ? 1 : (d[1] < 0 ? -1 : 0);
    double tdx = sx ? G.h / fabs(d[0]) : inf;
    double tdy = sy ? G.h / fabs(d[1]) : inf;
    double bx = G.x0 + (cx + (sx > 0 ? 1 : 0)) * G.h;
    double by = G.y0 + (cy + (sy > 0 ? 1 : 0)) * G.h;
    double tmx = sx ? (bx - o[0]) / d[0] : inf;
    double tmy = sy ? (by - o[1]) / d[1] : inf;
    if (tmx < 0) tmx = 0;
    if (tmy < 0) tmy = 0;
    double tin = 0.0;
    for (int guard = 0; guard < 4 * (G.gx + G.gy) + 8; ++guard) {
        double tout = fmin(tmx, tmy);
        double a = fmax(tin, 0.0), b = fmin(tout, thi);
        if (a > thi) break;
        int cell = cy * G.gx + cx;
        // ray height over [a, b]; b may be infinite when the ray leaves upward
        double za = o[2] + a * d[2];
        if (d[2] >= 0 && za > G.ztop + 1e-9 * (fabs(G.ztop) + 1.0)) break;  // above everything
        double zb = (b == inf) ? (d[2] >= 0 ? inf : -inf) : o[2] + b * d[2];
        double zlow = fmin(za, zb);
        double zmax = G.cell_zmax[cell];
        double margin = 1e-9 * (fabs(zmax) + fabs(zlow) + 1.0);
        if (!(zlow > zmax + margin)) {
            for (int k = G.cell_start[cell]; k < G.cell_start[cell + 1]; ++k) {
                int64_t t = G.cell_tris[k];
                if (t == skip1 || t == skip2) continue;
                if (ray_tri(o, d, tlo, thi, G.tri + 9 * t)) return true;
            }
        }
        // step to the next cell
        if (tmx < tmy) {
            cx += sx;
            tin = tmx;
            tmx += tdx;
        } else {
            cy += sy;
            tin = tmy;
            tmy += tdy;
        }
        if (cx < 0 || cx >= G.gx || cy < 0 || cy >= G.gy) break;
        if (tin > thi) break;
        if (sx == 0 && sy == 0) break;
    }
    return false;
}

template <class T>
__global__ void k_insolation(GridView G, const double *x, const double *n, const double *suns, int64_t N,
                             double flux, const int32_t *perm, int rmajor, T *Q, int64_t ldq) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t r = blockIdx.y;
    if (t >= N) return;
    const double *s = suns + 3 * r;
    const double *nt = n + 3 * t;
    double c = dot3(nt, s);
    double q = 0.0;
    if (c > 0.0 && !occluded(G, x + 3 * t, s, 1e-9, __builtin_huge_val(), t, t)) q = flux * c;
    if (rmajor) {
        Q[t * ldq + r] = (T)q;
    } else {
        int64_t row = perm ? (int64_t)perm[t] : t;
        Q[row + r * ldq] = (T)q;
    }
}

// V_ij bitmap (row i, 32 columns per word); the segment is cast from the facet
// with the smaller original index so that V is symmetric.
__global__ void k_vis_grid(GridView G, const double *x, const double *n, int64_t N, const int32_t *perm,
                           int64_t wpr, int64_t row0, int64_t rows, uint32_t *bits) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= rows * wpr) return;
    int64_t i = row0 + id / wpr, w = id % wpr;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
        int64_t j = w * 32 + b;
        if (j >= N || j == i) continue;
        const double *xi = x + 3 * i, *xj = x + 3 * j;
        double r[3] = {sub(xj[0], xi[0]), sub(xj[1], xi[1]), sub(xj[2], xi[2])};
        double ci = dot3(n + 3 * i, r);
        double cj = -dot3(n + 3 * j, r);
        if (!(ci > 0.0) || !(cj > 0.0)) continue;
        int64_t a = i, c = j;
        if (perm[j] < perm[i]) { a = j; c = i; }
        const double *xa = x + 3 * a, *xc = x + 3 * c;
        double d[3] = {sub(xc[0], xa[0]), sub(xc[1], xa[1]), sub(xc[2], xa[2])};
        if (!occluded(G, xa, d, 1e-9, 1.0 - 1e-9, a, c)) word |= 1u << b;
    }
    bits[id] = word;
}

GridView view_of(const rad_hmat *H) {
    GridView G;
    G.tri = H->d_tri.p;
    G.cell_start = H->d_cell_start.p;
    G.cell_tris = H->d_cell_tris.p;
    G.cell_zmax = H->d_cell_zmax.p;
    G.x0 = H->grid_x0;
    G.y0 = H->grid_y0;
    G.h = H->grid_h;
    G.gx = H->grid_gx;
    G.gy = H->grid_gy;
    G.ztop = H->grid_ztop;
    return G;
}

}  // namespace

// Host: bin triangles (tree order, 9 values each: one per facet, or none)
// into a uniform xy grid of about two triangles per cell.
void build_grid(rad_hmat *H, const std::vector<double> &tri) {
    const int64_t N = (int64_t)(tri.size() / 9);
    if (N == 0) {
        // no occluders: one empty cell below every ray
        H->d_tri.alloc(0);
        H->d_cell_start.upload(std::vector<int32_t>{0, 0});
        H->d_cell_tris.alloc(0);
        H->d_cell_zmax.upload(std::vector<double>{-1e300});
        H->grid_x0 = 0.0;
        H->grid_y0 = 0.0;
        H->grid_h = 1.0;
        H->grid_gx = 1;
        H->grid_gy = 1;
        H->grid_ztop = -1e300;
        return;
    }
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (int64_t t = 0; t < N; ++t)
        for (int v = 0; v < 3; ++v) {
            xmin = std::min(xmin, tri[9 * t + 3 * v]);
            xmax = std::max(xmax, tri[9 * t + 3 * v]);
            ymin = std::min(ymin, tri[9 * t + 3 * v + 1]);
            ymax = std::max(ymax, tri[9 * t + 3 * v + 1]);
        }
    double ext = std::max(xmax - xmin, ymax - ymin);
    if (!(ext > 0)) ext = 1.0;
    int64_t target = std::max<int64_t>(1, (int64_t)std::sqrt((double)N / 2.0));
    double h = ext / (double)target;
    // widen the box slightly so that every vertex falls strictly inside
    double pad = 1e-6 * ext;
    xmin -= pad;
    ymin -= pad;
    int32_t gx = (int32_t)std::max<int64_t>(1, (int64_t)std::ceil((xmax + pad - xmin) / h));
    int32_t gy = (int32_t)std::max<int64_t>(1, (int64_t)std::ceil((ymax + pad - ymin) / h));
    std::vector<int32_t> cnt((size_t)gx * gy + 1, 0);
    std::vector<double> zmax((size_t)gx * gy, -INFINITY);
    auto cell_range = [&](int64_t t, int &c0, int &c1, int &r0, int &r1) {
        double bx0 = INFINITY, bx1 = -INFINITY, by0 = INFINITY, by1 = -INFINITY;
        for (int v = 0; v < 3; ++v) {
            bx0 = std::min(bx0, tri[9 * t + 3 * v]);
            bx1 = std::max(bx1, tri[9 * t + 3 * v]);
            by0 = std::min(by0, tri[9 * t + 3 * v + 1]);
            by1 = std::max(by1, tri[9 * t + 3 * v + 1]);
        }
        double m = 1e-9 * ext;  // include neighbours touched within rounding
        c0 = std::max(0, (int)std::floor((bx0 - m - xmin) / h));
        c1 = std::min(gx - 1, (int)std::floor((bx1 + m - xmin) / h));
        r0 = std::max(0, (int)std::floor((by0 - m - ymin) / h));
        r1 = std::min(gy - 1, (int)std::floor((by1 + m - ymin) / h));
    };
    for (int64_t t = 0; t < N; ++t) {
        int c0, c1, r0, r1;
        cell_range(t, c0, c1, r0, r1);
        double tz = std::max({tri[9 * t + 2], tri[9 * t + 5], tri[9 * t + 8]});
        for (int r = r0; r <= r1; ++r)
            for (int c = c0; c <= c1; ++c) {
                cnt[(size_t)r * gx + c + 1]++;
                zmax[(size_t)r * gx + c] = std::max(zmax[(size_t)r * gx + c], tz);
            }
    }
    for (size_t k = 1; k < cnt.size(); ++k) cnt[k] += cnt[k - 1];
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1), items(cnt.back());
    for (int64_t t = 0; t < N; ++t) {
        int c0, c1, r0, r1;
        cell_range(t, c0, c1, r0, r1);
        for (int r = r0; r <= r1; ++r)
            for (int c = c0; c <= c1; ++c) items[fill[(size_t)r * gx + c]++] = (int32_t)t;
    }
    H->d_tri.upload(tri);
    H->d_cell_start.upload(cnt);
    H->d_cell_tris.upload(items);
    H->d_cell_zmax.upload(zmax);
    H->grid_x0 = xmin;
    H->grid_y0 = ymin;
    H->grid_h = h;
    H->grid_gx = gx;
    H->grid_gy = gy;
    double ztop = -INFINITY;
    for (double z : zmax) ztop = std::max(ztop, z);
    H->grid_ztop = ztop;
}

void launch_vis_grid(const rad_hmat *H, uint32_t *bits, int64_t wpr, int64_t row0, int64_t rows, hipStream_t s) {
    const int64_t tot = rows * wpr;
    if (tot <= 0) return;
    hipLaunchKernelGGL(k_vis_grid, dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, s, view_of(H), H->d_x.p,
                       H->d_n.p, H->N, H->d_perm.p, wpr, row0, rows, bits);
    RAD_HIP(hipGetLastError());
}

void launch_insolation(const rad_hmat *H, const double *suns_dev, int64_t R, double flux, int32_t dtype, void *Q,
                       int64_t ldq, int32_t order, hipStream_t s) {
    const int rmajor = order == RAD_ORDER_TREE_RMAJOR;
    const int32_t *perm = order == RAD_ORDER_ORIGINAL ? H->d_perm.p : nullptr;
    for (int64_t r0 = 0; r0 < R; r0 += 32768) {
        int64_t rn = std::min<int64_t>(32768, R - r0);
        dim3 grid((unsigned)((H->N + 127) / 128), (unsigned)rn);
        int64_t shift = rmajor ? r0 : r0 * ldq;
        if (dtype == RAD_F64)
            hipLaunchKernelGGL(k_insolation<double>, grid, dim3(128), 0, s, view_of(H), H->d_x.p, H->d_n.p,
                               suns_dev + 3 * r0, H->N, flux, perm, rmajor, (double *)Q + shift, ldq);
        else
            hipLaunchKernelGGL(k_insolation<float>, grid, dim3(128), 0, s, view_of(H), H->d_x.p, H->d_n.p,
                               suns_dev + 3 * r0, H->N, flux, perm, rmajor, (float *)Q + shift, ldq);
        RAD_HIP(hipGetLastError());
    }
}

}  // namespace rad
