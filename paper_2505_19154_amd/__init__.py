"""MI355X (gfx950) tile-based Gaussian-splatting rasterizer with w-weighted
feature fusion (FHGS, arXiv 2505.19154), behind the C ABI of include/fhgs.h.

    from paper_2505_19154_amd import raster, autograd
    r = raster.Rasterizer(cams, n, sh_degree, d)
    img = r.forward(gaussians)            # project + bin_sort + render_fwd
    grads = r.render_bwd(gaussians, img, dC, dF)

Importing the package loads nothing; the HIP library (libfhgs.so, built by
`python -m paper_2505_19154_amd.build`) is loaded on first use and its absence
is an error.
"""
__all__ = ["raster", "autograd", "build"]
