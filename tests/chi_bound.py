"""Forward-error bound for chi from the same Lanczos coefficients.

chi_l(w) = n_1 z_l . x(w) with A(w) x = e_1, A = (w + i eta) I - T.  A
backward-stable tridiagonal solve (Gaussian elimination with partial
pivoting: growth at most 2, a few flops per eliminated row) returns x + dx
with ||dx|| <= c u kappa(A) ||x||, so two such solvers (the oracle's zgtsv,
the library's kernel) give chi values that differ by at most

    |d chi_l(w)| <= 2 c u kappa(A(w)) |n_1| ||z_l|| ||x(w)||.

For a pseudo-Hermitian chain T is real symmetric, A is normal and
kappa(A) = max_j |w + i eta - t_j| / min_j |w + i eta - t_j| over the
eigenvalues t_j of T.  c = 8 here; the test pins the bound on the CPU with
two different solvers (dense LU against zgtsv), which stay below a tenth of it.
"""
import numpy as np
import scipy.linalg as sla

U64 = 2.0 ** -53
C = 8.0


def chi_difference_bound(coeffs, m, omega, eta):
    """Bound [l][w] on |chi_a - chi_b| between two backward-stable solvers (pH chains)."""
    a = np.asarray(coeffs["alpha"][:m])
    b = np.asarray(coeffs["beta"][:m - 1], dtype=float)
    g = np.asarray(coeffs["gamma"][:m - 1])
    # pseudo-Hermitian chains: alpha real, gamma = beta (extrapolated means may differ in the last bit)
    assert np.abs(a.imag).max(initial=0) <= 1e-14 * np.abs(a).max() and \
        np.abs(g - b).max(initial=0) <= 1e-14 * max(b.max(initial=0), 1e-300), "needs a symmetric T"
    t = sla.eigvalsh_tridiagonal(a.real, b) if m > 1 else a.real
    z = np.asarray(coeffs["z"])[:, :m]
    zn = np.linalg.norm(z, axis=1)
    out = np.zeros((z.shape[0], len(omega)))
    ab = np.zeros((3, m), dtype=np.complex128)
    ab[0, 1:] = -g
    ab[2, :-1] = -b
    rhs = np.zeros(m, dtype=np.complex128)
    rhs[0] = 1.0
    for j, w in enumerate(omega):
        d = np.abs(w + 1j * eta - t)
        kappa = d.max() / d.min()
        ab[1] = w + 1j * eta - a
        xn = np.linalg.norm(sla.solve_banded((1, 1), ab, rhs))
        out[:, j] = 2 * C * U64 * kappa * abs(coeffs["n1"]) * zn * xn
    return out
