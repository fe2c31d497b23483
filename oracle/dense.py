"""Transition-space ("sum over transitions") Liouvillian for tiny systems (oracle).

An independent construction of the same operator as ``liouvillian.Problem``:
instead of applying V' to u_n through grids, the Liouvillian is written out as
a dense matrix in the orthonormal basis of the empty manifold,

    X side: |c> (x) band n, c an empty eigenvector of H_{k+q};
    Y side: T|c'> (x) band n, c' an empty eigenvector of H_{-k-q},

so that the D blocks are diagonal (e_c(k+q) - e_n(k) and e_c'(-k-q) - e_n(-k))
and the coupling is a Gram matrix of pair densities,

    K_IJ = (1/Nk) int sum_ab conj(rho_Ia(r)) F_ab rho_Jb(r) dr,
    rho_Ia = u_n^dag S_a c          (X),   s_a u'_n^dag S_a T c'   (Y),

with F the Hartree operator on a = b = 0 plus the local kernel f_ab.  Then
L = J (D + K) reproduces Eq. Liouvillian_BR_q: JL = D + K is Hermitian.
"""
from __future__ import annotations

import numpy as np

from . import grid
from .liouvillian import SIDE_SIGNS, role_state
from .scf import PAULI


class TransitionSpace:
    def __init__(self, prob):
        self.prob = prob
        gs, sysd = prob.gs, prob.sysd
        nb = prob.nb
        sq = np.sqrt(sysd.omega)
        self.labels = []      # (side, ik, n, c)
        self.vecs = []        # basis vectors on the k+q sphere [2][npw]
        self.diag = []
        for s in range(2):
            for ik, kd in enumerate(prob.k):
                role = 2 if s == 0 else 3
                _, m_c, _, _ = role_state(prob.point_states, prob.qset, ik, role)
                kc = prob.qset.points[prob.qset.roles[ik][role]] + \
                    prob.qset.shifts[ik][role] @ sysd.recip
                ec, vc = np.linalg.eigh(gs.hamiltonian(kc, m_c))
                vc = vc.T.reshape(-1, 2, m_c.shape[0])[nb:]
                ec = ec[nb:]
                if s == 1:
                    vc = grid.time_reverse(m_c, vc, kd.mill)
                for n in range(nb):
                    for c in range(len(ec)):
                        self.labels.append((s, ik, n, c))
                        self.vecs.append(vc[c])
                        self.diag.append(ec[c] - kd.eps[s][n])
        self.dim = len(self.labels)
        self.side = np.array([l[0] for l in self.labels])
        self.Jdiag = np.where(self.side == 0, 1.0, -1.0)
        # pair densities
        N = sysd.ngrid
        P = np.zeros((self.dim, 4, N), dtype=np.complex128)
        for I, ((s, ik, n, _), vec) in enumerate(zip(self.labels, self.vecs)):
            kd = prob.k[ik]
            cr = grid.to_grid(sysd.fft, kd.mill, vec) / sq
            u = kd.u_real[s][n]
            for a in range(4):
                P[I, a] = SIDE_SIGNS[s][a] * np.einsum("sxyz,st,txyz->xyz", u.conj(), PAULI[a], cr).ravel()
        self.P = P

    def kernel_matrix(self, hartree=True, xc_on=True):
        prob, sysd = self.prob, self.prob.sysd
        N = sysd.ngrid
        FP = np.zeros_like(self.P)
        if hartree:
            for I in range(self.dim):
                FP[I, 0] += grid.apply_coulomb(prob.hq, self.P[I, 0].reshape(sysd.fft)).ravel()
        if xc_on:
            f = prob.f.reshape(4, 4, N)
            FP += np.einsum("abr,Ibr->Iar", f, self.P)
        w = sysd.omega / N
        return w / prob.nk * (self.P.reshape(self.dim, -1).conj() @ FP.reshape(self.dim, -1).T)

    def liouvillian(self, kernel=True, **kw):
        M = np.diag(np.asarray(self.diag, dtype=np.complex128))
        if kernel:
            M = M + self.kernel_matrix(**kw)
        return self.Jdiag[:, None] * M

    # ---- maps between the batch representation and this basis ----------
    def to_basis(self, xy):
        out = np.zeros(self.dim, dtype=np.complex128)
        for I, ((s, ik, n, _), vec) in enumerate(zip(self.labels, self.vecs)):
            npw = self.prob.k[ik].npw
            out[I] = np.vdot(vec, xy[s, ik, n, :, :npw])
        return out

    def from_basis(self, c):
        xy = self.prob.zeros()
        for I, ((s, ik, n, _), vec) in enumerate(zip(self.labels, self.vecs)):
            npw = self.prob.k[ik].npw
            xy[s, ik, n, :, :npw] += c[I] * vec
        return xy

    def matrix_free_columns(self, **kw):
        """The matrix-free Liouvillian expressed in this basis, column by column."""
        M = np.zeros((self.dim, self.dim), dtype=np.complex128)
        e = np.zeros(self.dim, dtype=np.complex128)
        for J in range(self.dim):
            e[:] = 0
            e[J] = 1
            M[:, J] = self.to_basis(self.prob.apply(self.from_basis(e), **kw))
        return M

    def chi_dense(self, L, u, v, omega, eta):
        """(u, ((w + i eta) - L)^{-1} v) with u, v batch vectors (u projected on the basis)."""
        ut, vt = self.to_basis(u), self.to_basis(v)
        out = np.zeros(len(omega), dtype=np.complex128)
        I = np.eye(self.dim)
        for j, w in enumerate(omega):
            out[j] = np.vdot(ut, np.linalg.solve((w + 1j * eta) * I - L, vt))
        return out / self.prob.nk

    def chi_sot(self, L, u, v, omega, eta):
        """Sum over transitions: sum_j (u, R_j)(L_j, v) / (w + i eta - W_j)."""
        ut, vt = self.to_basis(u), self.to_basis(v)
        lam, R = np.linalg.eig(L)
        left = np.linalg.solve(R, vt)
        right = ut.conj() @ R
        wc = np.asarray(omega)[:, None] + 1j * eta
        return (right[None, :] * left[None, :] / (wc - lam[None, :])).sum(axis=1) / self.prob.nk, lam
