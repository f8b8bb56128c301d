"""MI355X-native hierarchical low-rank view-factor matrices and radiosity solves.

The computation lives in librad.so (HIP for gfx950 behind the C-ABI of
include/rad.h, rad_warmstart.h and rad_timestep.h); this package is its thin
Python binding.

Typical use (device tensors from torch on the matrix's GPU)::

    from paper_2209_07632_amd import HMatrix, TimeStepper
    H = HMatrix(verts, faces, tol=1e-3, storage="f32", max_rhs=1024)   # Algorithms 2-4
    Q = H.insolation(suns, flux=1365.0, order="tree_rmajor")            # direct insolation
    B, info = H.solve(0.3 * Q, rho=0.3, rtol=1e-3, order="tree_rmajor") # (I - 0.3 F) B = E
    Y = H.matvec(X)                                                       # Algorithm 5

    # closed bodies: HMatrix(..., tree="oct") builds an octree instead of a quadtree

    S = TimeStepper(H, z, conductivity, heat_capacity, dt, albedo, emissivity, R=8)
    S.init(T0, Qdir0)          # Algorithm 6, level 0
    S.step(Qdir_levels)        # one product of 2R columns and one column step per level
    T_surface = S.read("T")[0]
"""
from .rad import HMatrix, RadError, load  # noqa: F401
from .timestep import TimeStepper  # noqa: F401
