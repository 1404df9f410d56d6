"""Method constants used by the oracle.

The paper fixes the 16x16 tile and the 64-bit (tile, depth) key (Appendix A,
"Details of the Rasterizer").  It inherits everything else from the 3D Gaussian
Splatting rasterizer it builds on and does not restate it; the values below are
the readings taken for those silences: 3DGS's published rules, except the
binning box, which is the tightest axis-aligned box that provably holds every
pixel where alpha can reach 1/255.
"""
import numpy as np

TILE = 16                 # tile side in pixels (Appendix A)
Z_NEAR = 0.2              # near-plane cull on camera-space depth
LOWPASS = 0.3             # screen-space low-pass added to the 2D covariance diagonal (px^2)
ALPHA_MAX = 0.99          # alpha clamp
ALPHA_MIN = 1.0 / 255.0   # blends with alpha below this are skipped
T_MIN = 1e-4              # a pixel stops before the blend that would take T below this
KAPPA = 11.1              # binning box half-extent = sqrt(KAPPA * Sigma2_diag); > 2 ln 255

# float32 images of the constants, as the float32 binning arithmetic uses them
Z_NEAR_F32 = np.float32(Z_NEAR)
LOWPASS_F32 = np.float32(LOWPASS)
KAPPA_F32 = np.float32(KAPPA)

# relative distance to a threshold below which a float32-vs-FP64 decision is
# called ambiguous (alpha >= ALPHA_MIN, T' < T_MIN, the ALPHA_MAX clamp)
AMBIG_REL = 1e-4

# density-rounding allowance of the surfel primitive, per unit of its
# first-order sensitivity (oracle/raster.c's header): an FP32 implementation
# rounds each record entry once and each product and sum of k0, k1, k2 once
# more (at most 3 roundings of each term's magnitude), and the quotient
# u = k0 / k2 adds the relative errors of both, so 6 units of FP32 roundoff
# bound u's error by 6 u32 um to first order
DEN_ROUND = 6.0 * 2.0 ** -24
