"""FP64 / exact-integer CPU oracle for the lattice FFT and the fast lattice
wavelet decomposition (Bergmann, "The fast Fourier Transform and fast Wavelet
Transform for Patterns on the Torus", arXiv:1107.5415).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, calls or links anything in
here, and nothing in here imports the product package: the two implementations
share no code.  The only module both sides read is the seeded input generator
``workloads``, which holds no arithmetic of the method.

Every function is written from the paper's definitions, in plain and slow
form (Python integers for all integer work, float64 / complex128 for all
floating-point work), so that it can be checked against the paper by eye.

Modules
  lattice  exact integer algebra: det, adjugate, Hermite and Smith invariants,
           natural residue boxes, symmetric representatives (Section 2.2)
  dft      the Fourier matrix F(M) as a direct O(m^2) sum (eq. Fouriermatrix)
           and an independent Hermite-form row/column FFT for large m
  wavelet  Dirichlet scaling mask (Section 6.2), one-level split and its
           inverse (Section 5.3, steps 1-5), multi-level pyramid, and the
           time-domain inner-product definition it must equal
  wavelet_q  the split for q = |det J| > 2 channels (Section 5.3 step 4 for
           general q) with the Dirichlet mask of any q and a Householder
           completion of the wavelet channels, its pyramid, and the
           time-domain definition it must equal
  interp   the change of basis between point values on P(M) and
           coefficients in the orthonormal translates of the Dirichlet
           kernel (Section 6.2), from the bracket sums of its coefficients
  scaling  the per-level scaling report of Theorem 3 (pattern dimensions,
           the step's direction) with brute-force pins
  grad     float64 torch autograd re-implementation for gradient checks

Parity status of every function is stated in its docstring; functions without
an independent pin say "parity unpinned".
"""
