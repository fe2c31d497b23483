"""Susceptibility from Lanczos coefficients, and the K = 0 Kubo sum (oracle).

chi_lm(w) = n_1 sum_i z_i^l eta_i with ((w + i eta) I - T) eta = e_1
(Sec. 2.5, Eqs. resolvent_Liouvillian_Lanczos_q and post_processing; the
broadening w -> w + i eta is stated just below them).  The tridiagonal
solve uses LAPACK's zgtsv (Gaussian elimination with partial pivoting).
Two independent evaluations serve as cross-checks: the continued fraction
for the (1,1) element and the pole-residue form from the eigenvectors of T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg.lapack as lapack


def tridiag(coeffs, m_use):
    a = np.asarray(coeffs["alpha"][:m_use], dtype=np.complex128)
    b = np.asarray(coeffs["beta"][:m_use - 1], dtype=np.complex128)
    g = np.asarray(coeffs["gamma"][:m_use - 1], dtype=np.complex128)
    T = np.diag(a) + np.diag(b, -1) + np.diag(g, 1)
    return T


def chi_lanczos(coeffs, omega, eta, m_use=None):
    """chi[l][w] from the coefficients (zgtsv per frequency)."""
    m = coeffs["steps_done"] if m_use is None else m_use
    a = np.asarray(coeffs["alpha"][:m], dtype=np.complex128)
    b = np.asarray(coeffs["beta"][:m - 1], dtype=np.complex128)
    g = np.asarray(coeffs["gamma"][:m - 1], dtype=np.complex128)
    z = coeffs["z"][:, :m]
    out = np.zeros((z.shape[0], len(omega)), dtype=np.complex128)
    for j, w in enumerate(omega):
        d = (w + 1j * eta) - a
        rhs = np.zeros(m, dtype=np.complex128)
        rhs[0] = 1.0
        if m == 1:
            x = rhs / d
        else:
            _, _, _, x, info = lapack.zgtsv(-b.copy(), d.copy(), -g.copy(), rhs)
            if info != 0:
                raise np.linalg.LinAlgError(f"zgtsv info={info}")
        out[:, j] = coeffs["n1"] * (z @ x)
    return out


def continued_fraction_11(coeffs, omega, eta, m_use=None):
    """[((w + i eta) - T)^{-1}]_{11} by the backward continued fraction."""
    m = coeffs["steps_done"] if m_use is None else m_use
    a = coeffs["alpha"][:m]
    bg = np.asarray(coeffs["beta"][:m - 1]) * np.asarray(coeffs["gamma"][:m - 1])
    out = np.zeros(len(omega), dtype=np.complex128)
    for j, w in enumerate(omega):
        wc = w + 1j * eta
        t = wc - a[m - 1]
        for i in range(m - 2, -1, -1):
            t = wc - a[i] - bg[i] / t
        out[j] = 1.0 / t
    return out


def chi_pole_residue(coeffs, omega, eta, m_use=None):
    m = coeffs["steps_done"] if m_use is None else m_use
    T = tridiag(coeffs, m)
    lam, R = np.linalg.eig(T)
    left = np.linalg.solve(R, np.eye(m)[:, 0])
    zR = coeffs["z"][:, :m] @ R
    wc = np.asarray(omega)[None, :] + 1j * eta
    return coeffs["n1"] * np.einsum("lj,j,jw->lw", zR, left, 1.0 / (wc - lam[:, None]))


def extrapolate(coeffs, m_use, m_total, mode):
    """Coefficients extended from m_use computed steps to m_total.

    The paper names two schemes ('constant' and the bi-constant 'osc'; Sec. 2.5,
    last paragraph, and the turbo_spectrum inputs of Sec. 3.3) without formulas.
    Reading: past m_use, alpha, beta and gamma take their mean over the second
    half of the computed coefficients -- one mean ('constant') or one for each
    parity of the index ('osc') -- and z is zero there (nothing was measured).
    """
    out = {k: coeffs[k] for k in ("n1",)}
    a = np.zeros(m_total, dtype=np.complex128)
    b = np.zeros(m_total)
    g = np.zeros(m_total, dtype=np.complex128)
    z = np.zeros((coeffs["z"].shape[0], m_total), dtype=np.complex128)
    a[:m_use] = coeffs["alpha"][:m_use]
    b[:m_use] = coeffs["beta"][:m_use]
    g[:m_use] = coeffs["gamma"][:m_use]
    z[:, :m_use] = coeffs["z"][:, :m_use]
    if m_total > m_use:
        period = {"constant": 1, "osc": 2}[mode]
        window = np.arange(m_use // 2, m_use)
        for p in range(period):
            sel = window[window % period == p]
            tail = np.arange(m_use, m_total)
            tail = tail[tail % period == p]
            a[tail] = a[sel].mean()
            b[tail] = b[sel].mean()
            g[tail] = g[sel].mean()
    out.update(alpha=a, beta=b, gamma=g, z=z, steps_done=m_total)
    return out


def structure_factor(q, chi):
    """S(q, w) = -Im Tr[P_perp(q) chi(w)] (Eq. S_def), chi[lambda][mu][w]."""
    q = np.asarray(q, dtype=float)
    P = np.eye(3) - np.outer(q, q) / q.dot(q)
    return -np.einsum("ab,baw->w", P, chi).imag


def kubo_k0(gs, prob, lam, mu, omega, eta):
    """Textbook K = 0 (independent-particle) transverse susceptibility.

    chi0_lm = (1/Nk) sum_k { sum_{v in k, c in k+q} <v|s_l|c><c|s_m|v> / (w' - (e_c - e_v))
                           - sum_{v in -k, c in -k-q} <v|s_m|c><c|s_l|v> / (w' + (e_c - e_v)) }

    with w' = w + i eta, c running over the empty eigenvectors of H at k+q
    (resp. -k-q) from a full diagonalisation, and the occupied v restricted to
    the sphere of k+q (resp. -k-q).  No time reversal is used anywhere.
    """
    from . import grid
    from .liouvillian import DIRECTIONS, role_state
    sl, sm = DIRECTIONS[lam], DIRECTIONS[mu]
    wc = np.asarray(omega) + 1j * eta
    nb = prob.nb
    out = np.zeros(len(omega), dtype=np.complex128)
    for ik in range(prob.nk):
        for sign, (rv, rc) in ((+1, (0, 2)), (-1, (1, 3))):
            _, m_v, e_v, et_v = role_state(prob.point_states, prob.qset, ik, rv)
            _, m_c, _, _ = role_state(prob.point_states, prob.qset, ik, rc)
            kc = prob.qset.points[prob.qset.roles[ik][rc]] + prob.qset.shifts[ik][rc] @ gs.sysd.recip
            H = gs.hamiltonian(kc, m_c)
            ec, vc = np.linalg.eigh(H)
            npw = m_c.shape[0]
            vc = vc.T.reshape(-1, 2, npw)[nb:]
            ec = ec[nb:]
            v = grid.restrict(m_v, e_v[:nb], m_c)
            A = np.einsum("nsg,st,ctg->nc", v.conj(), sl, vc)   # <v|s_l|c>
            Bm = np.einsum("nsg,st,ctg->nc", v.conj(), sm, vc)  # <v|s_m|c>
            # <c|s|v> = conj(<v|s^dag|c>); the sigma matrices used are Hermitian
            om = ec[None, :] - et_v[:nb, None]
            if sign > 0:
                num = A * Bm.conj()
                out += np.einsum("nc,wnc->w", num, 1.0 / (wc[:, None, None] - om[None]))
            else:
                num = Bm * A.conj()
                out -= np.einsum("nc,wnc->w", num, 1.0 / (wc[:, None, None] + om[None]))
    return out / prob.nk
