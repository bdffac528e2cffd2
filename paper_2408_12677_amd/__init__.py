"""MI355X-native differentiable tile-based Gaussian-splatting rasterizer (HIP, gfx950).

The hot path of GSFusion's online optimisation (arXiv 2408.12677, Sec. III-B-3): render
a Gaussian map through one or more cameras and back-propagate an L1 loss to every
Gaussian parameter.  The kernels live in ``libgsr.so`` behind the C ABI of
``include/gsr.h``; ``paper_2408_12677_amd.rasterize`` is the PyTorch binding.  Importing
this package does not load the library; the first call does, and fails loudly when it
has not been built (``python -m paper_2408_12677_amd.build``).
"""
