"""FP64 CPU oracle of the ratio-filter hot path (Murakami, Ghosh, Morisaki,
arXiv 2511.12894).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package.  The product path
(the HIP library and its Python binding) never imports, links or executes
anything here, and this package imports nothing from the product path: the
two share no kernels, headers, helpers, tables or constant generators.  The
only shared module is the seeded input generator, which holds no filtering
arithmetic.

Everything is float64 / complex128 NumPy, written for readability, not speed.

Modules
-------
taylorf2   TaylorF2 phase, amplitude, time-frequency map t(f) and t'(f)
mf         matched-filter SNR series and template norm (section II.A)
ratio      window, ratio spectrum, ratio kernel, truncation, reconstruction
           (sections II.B-II.D, appendix A)
peaks      peak / threshold read-out of an SNR series
mlp        reference forward/backward of the kernel-surrogate MLP
"""
