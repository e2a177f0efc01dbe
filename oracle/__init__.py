"""Plain FP64 CPU oracle for the PolyCLEAN measurement operator and solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product path
(the HIP library and its Python binding) never calls into it, and the two
share no code: no kernels, headers, tables, constants or helpers.

What it computes, and from which passage of the paper (Jarret et al. 2024,
"PolyCLEAN: Atomic Optimization for Super-Resolution Imaging and Uncertainty
Estimation in Radio Interferometry"):

  geometry  pixel grid and direction cosines (Sect. 2.2), nominal resolution
            1/(3 B0) (Sect. 6.1, "Resolution of the images").
  operator  the discrete forward operator Phi (Sect. 2.2, Eq. phi-discrete) and
            its adjoint Phi* (Eq. adjoint-phi), evaluated exactly as direct
            exponential sums in complex128 (no gridding, no FFT).
  solver    LASSO objective (Eq. lasso), lambda_max and lambda = alpha
            lambda_max (Eqs. lmax, lambda), dual certificate (Eq. dual_certif),
            the Polyatomic Frank-Wolfe iteration (Alg. 2) with an APGD/FISTA
            restricted solve on the active set (Sect. 4.4 and Sect. 5.1), and
            a standard LASSO duality gap.
  brute     cyclic coordinate descent on the explicit real measurement matrix,
            for tiny problems (an independent route to the LASSO minimiser).

Every floating-point quantity is float64/complex128.  Inputs that the GPU
receives in complex64 are passed here upcast, so input rounding is not charged
to the GPU.

Parity status: every function is pinned by the not-gpu tests (closed forms,
the adjoint dot test, the shifted-PSF identity, the orthogonal-design closed
form of the whole solver, KKT conditions, brute force and the printed numbers
of Tables 1, 2 and A.1); see tests/test_oracle_*.py.
"""
from . import geometry, operator, solver, brute  # noqa: F401
