"""MI355X-native H-LU preconditioned GMRES for the time-harmonic Maxwell
equations (lowest-order Nedelec edge elements), after Parvizi, Khodadadian,
Beuchler, Wick, "Hierarchical LU preconditioning for the time-harmonic
Maxwell equations" (arXiv 2211.11303).

The compute path is the C-ABI library libhlu.so (HIP kernels for gfx950);
``hlu`` is its Python binding.  ``inputs`` draws the seeded synthetic inputs.
"""
