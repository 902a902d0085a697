"""FP64 CPU oracle for the SDMM imaging hot path (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the HIP path
is checked against.  It is test infrastructure: only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  The product
path (the HIP library and its Python binding) never imports or calls it, and it
shares no code, table or constant generator with that path.

Modules
  kaiser_bessel  Kaiser-Bessel interpolation kernel, its Fourier transform, I0
  nufft          measurement operator Phi = G F D Z (B = I) and its adjoint,
                 plus the exact direct Fourier sum it approximates (Sec. 5)
  wavelets       Daubechies filters by spectral factorisation, periodised
                 orthonormal 2-D DWT, SARA dictionary Psi (Sec. 3.3, Sec. 5)
  prox           proximity operators of f1, f2, f3 (Sec. 4.4, eqs. prox1-3)
  sdmm           conjugate gradient on Q, SDMM (Algorithm 1), penalty gamma,
                 noise bound epsilon, SNR (Sec. 4.3, 4.4, 6)

Every function cites the passage of the paper it follows.  Readings of passages
that are silent or garbled are listed in the module docstrings.
"""
