"""CPU oracle for the tile-based Gaussian-splatting rasterizer with feature fusion.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import, call or link anything in this package.  The
product path (the HIP library and its Python binding) never uses it, and this
package never imports the product package: the two share no code.

Everything here is plain, slow and written to be checked by eye against the
paper (FHGS, arXiv 2505.19154): compositing (Section 3.1, the colour equation
and the definition w_i = alpha_i T_i), the adjoint through w (Appendix A.2, the
derivative of the loss with respect to alpha_k), and the 3DGS-style tile
binning the paper builds on (Appendix A, "Details of the Rasterizer";
Algorithm 2).  Floating-point work is FP64 from the exact upcast of the float32
(or bfloat16) inputs, except the binning quantities, which the method decides
in float32 with a fixed operation order (binspec.py).

Modules
  consts    method constants and the readings of the paper's silences
  sh        real spherical harmonics from Legendre polynomials (FP64)
  project   per-Gaussian projection and its adjoint chain (FP64, numpy)
  binspec   float32 binning: depth keys, tile rects, keys and ranges (numpy)
  raster    per-pixel front-to-back compositing, its adjoint and the fusion
            sums, in plain C (raster.c) called through ctypes
  brute     per-pixel brute force without tiles (numpy FP64, and a torch
            float64 autograd version) for tiny scenes
  pipeline  the whole path for one scene, as used by the tests
"""
