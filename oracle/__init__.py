"""CPU oracle for the Walsh-to-boundary-wavelet change-of-basis operator.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, fp64 reference
implementation written from the paper (Antun, "Recovering wavelet
coefficients from binary samples using fast transforms").  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The GPU library never imports, links or calls
anything in here, and nothing in here imports the GPU library.

What it computes is the plain definition of the matrix: entry (n, c) is the
inner product of the sequency-ordered Walsh function w_n (Def. 3.1) with the
c-th function of the multiscale basis C_{psi,j} on [0, 1] built from
Daubechies wavelets with vanishing-moment-preserving boundary functions
(Sec. 3.2).  Because w_n with n < 2^J is constant on every cell
[i 2^-J, (i+1) 2^-J), that inner product is exactly the Walsh matrix times
the vector of cell integrals of the basis function; no quadrature error and
no fast transform is involved.

Modules
  walsh     Def. 3.1 digit by digit; Lemma 3.2 helpers.
  filters   Daubechies filters by spectral factorisation (mpmath).
  cascade   cell integrals and point values of phi and psi (cascade).
  halfline  half-line Gram matrix and boundary functions (mpmath).
  basis     cell integrals of the interval bases B_{phi,k}, B_{psi,k}.
  operator  dense 1D matrix, 2D separable and dense products, samples.

Parity status of every function is stated in its module header.
"""
