"""MI355X-native differentiable volume rendering of sparse voxel grids.

The hot path of RGB-D mapping and tracking in a Plenoxel radiance field
(Teigen et al., WACV 2024): rays marched through a link-table voxel grid,
density and degree-2 SH colour trilinearly interpolated, colour and expected
depth alpha-composited (Eq. 1-3), and analytic gradients of the photometric
plus depth loss with respect to the grid (Eq. 6-10, mapping) and to the se(3)
camera pose (Eq. 12-14 with Appendix A, tracking); around it, the optimiser
steps (sparse RMSProp for the map, Adam or Gauss-Newton for the poses), the
dynamic grid's coarse-to-fine growth and pruning, and the batched loops that
drive them.

Modules
    pxm        ctypes binding of the C ABI (include/pxm.h) of libpxm.so
    autograd   torch.autograd.Function wrappers (recomputing backward)
    batch      ray packer, autotuner, captured tracking loop (Adam or
               Gauss-Newton), mapping loop (with growth and pruning) and
               image metrics
    synth      seeded synthetic workloads (inputs only)
    build      hipcc build of libpxm.so for gfx950
"""

__version__ = "0.1.0"
