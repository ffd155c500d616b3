"""CPU oracle for the GaNi Fourier-Galerkin cell problem -- TEST INFRASTRUCTURE.

Plain, slow, FP64 NumPy/SciPy code written directly from the paper
(Vondrejc, Liu, Ladecky, Matthies, "FFT-based homogenisation accelerated by
low-rank tensor approximations", arXiv:1902.07455).  It exists to check the
HIP library; it shares no code with it and the library never calls it.
Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import it.

Modules
-------
fg        full-grid GaNi solve in Fourier space: PCG on eq. (ls_GaNi_fourier)
          preconditioned by eq. (Pls_GaNi_fourier); A_H from eq. (homog).
brute     dense real-space assembly of the same discrete minimisation
          (explicit DFT matrices, no FFT, direct solve) for tiny grids.
lowrank   CP / Tucker / TT operations of Sec. 3.1 and Appendix A written
          on small NumPy arrays (to_full, Hadamard, addition, 1-D DFTs on
          factors, SVD-based truncation) plus the truncated minimal-residual
          iteration of Sec. 3.3.
expsum    exponential-sum (sinc quadrature) approximation of 1/x used as
          the separable preconditioner of the low-rank path.
"""
