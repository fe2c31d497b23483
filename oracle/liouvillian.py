"""Matrix-free Liouvillian in the batch representation (oracle).

Batch representation (Sec. 2.4, Eq. batch_rho): a response is the pair
(X, Y) of spinor sets x_{n,k+q}, y_{n,k+q}, one per occupied band n and mesh
point k, stored here as one array [2 sides][nk][nb][2 spins][npw_pad] on the
sphere of k+q.  The Liouvillian (Eqs. Liouvillian_BR_q, liouvillian_blocks):

    L (X, Y) = ( P  [ (H_{k+q}  - e_{n,k})  x_n + V'   u_n  ],
                -P+ [ (H+_{k+q} - e_{n,-k}) y_n + V'+  u'_n ] )

with u_n = U_{n,k}, u'_n = T U_{n,-k}; H+ = H with the B field flipped and
V'+ = V' with its magnetic part flipped (both stated in Sec. 2.2); P and P+
project out U_{m,k+q} and T U_{m,-k-q} (Eqs. P_minus_q2, P_plus_q2).  One
projector is applied to the sum of the D and K parts.  V' is built from the
response densities of Eqs. charge_dens_resp_q / spin_dens_resp_q:

    rho'_a = (1/Nk) sum_{k,n} [ u_n^dag S_a x_n + s_a u'_n^dag S_a y_n ],
    S = (sigma_0, sigma_x, sigma_y, sigma_z), s = (+1, -1, -1, -1),

and V' = W_0 sigma_0 + W . sigma with W_a = delta_a0 v'_H + sum_b f_ab rho'_b
(Eqs. V_HXC_resp_q, v_H_q, v_XC_q, b_XC_q).

Start and measure vectors (Sec. 2.5, Eq. off-diag-resolvent and below):
    u^l = ( sigma^l U~_{n,k}, -sigma^l T U~_{n,-k} ),
    v^m = ( P sigma^m U~_{n,k}, P+ sigma^m T U~_{n,-k} ),
with U~ the coefficients restricted to the sphere of k+q.  The charge
channel (l or m = n, sigma^n = sigma_0, the generalized 4x4 susceptibility
of Sec. 2.3) follows the same derivation with the time-reversal parity of
sigma_0, which is +1 where the spin matrices have -1 (T sigma T^-1 = -sigma):
the lower component of u is s_l sigma^l T U~ and that of v is
-s_m P+ sigma^m T U~, s = +1 for n and -1 for the spin directions; for the
spin directions these are the printed vectors.  Inner product
(a, b) = (1/Nk) sum a^dag b, conjugate-linear in a.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import synth
from . import grid, xc
from .scf import PAULI

DIRECTIONS = {
    "n": PAULI[0],
    "x": PAULI[1],
    "y": PAULI[2],
    "z": PAULI[3],
    "+": PAULI[1] + 1j * PAULI[2],
    "-": PAULI[1] - 1j * PAULI[2],
}
SIDE_SIGNS = (np.array([1.0, 1.0, 1.0, 1.0]), np.array([1.0, -1.0, -1.0, -1.0]))
# time-reversal parity s of each direction's matrix: T sigma T^-1 = s sigma
TR_PARITY = {"n": 1.0, "x": -1.0, "y": -1.0, "z": -1.0, "+": -1.0, "-": -1.0}


@dataclass
class KData:
    k: np.ndarray
    kq: np.ndarray
    mill: np.ndarray          # sphere of k+q
    kin: np.ndarray           # |k+q+G|^2 / 2
    u_real: list              # [side] -> [nb][2][n1,n2,n3], Omega^{-1/2} normalised
    u_sph: list               # [side] -> [nb][2][npw]  (U~_k, T U~_-k)
    eps: list                 # [side] -> [nb]          (e_k, e_-k)
    occ: list                 # [side] -> [nb][2][npw]  (U_{k+q}, T U_{-k-q})
    beta: np.ndarray          # [nproj][npw] at k+q

    @property
    def npw(self):
        return self.mill.shape[0]


def role_state(point_states, qset, ik, role):
    """(kvec, mill, evc, et) of role (0: k, 1: -k, 2: k+q, 3: -k-q) of mesh point ik.

    A role vector p = points[i] + g.b carries U_p(G) = U_i(G + g.b), i.e. the
    same coefficients on Miller indices shifted by -g.
    """
    i = qset.roles[ik][role]
    g = qset.shifts[ik][role]
    mill, evc, et = point_states[i]
    return None, mill - g[None, :], evc, et


class Problem:
    """Everything the Liouvillian of one q needs, built from a ground state."""

    def __init__(self, gs, qset, point_states=None, fields=None):
        self.gs = gs
        self.sysd = sysd = gs.sysd
        self.qset = qset
        if point_states is None:
            point_states = [gs.solve(p) for p in qset.points]
        self.point_states = point_states
        self.vrs = gs.vrs if fields is None else fields[0]
        rho0 = gs.rho if fields is None else fields[1]
        self.f = xc.kernel(rho0)
        self.hq = grid.coulomb_multiplier(sysd, qset.q)
        self.dmat = synth.dmatrix(sysd)
        self.nk = len(qset.kmesh)
        self.nb = sysd.nbnd
        sq = np.sqrt(sysd.omega)
        self.k = []
        for ik, kvec in enumerate(qset.kmesh):
            kq = kvec + qset.q
            _, m_k, e_k, et_k = role_state(point_states, qset, ik, 0)
            _, m_mk, e_mk, et_mk = role_state(point_states, qset, ik, 1)
            _, m_kq, e_kq, _ = role_state(point_states, qset, ik, 2)
            _, m_mkq, e_mkq, _ = role_state(point_states, qset, ik, 3)
            K = kq + m_kq @ sysd.recip
            kin = 0.5 * np.einsum("ij,ij->i", K, K)
            u0 = grid.to_grid(sysd.fft, m_k, e_k[:self.nb]) / sq
            u1 = grid.time_reverse_real(grid.to_grid(sysd.fft, m_mk, e_mk[:self.nb]) / sq)
            us0 = grid.restrict(m_k, e_k[:self.nb], m_kq)
            us1 = grid.time_reverse(m_mk, e_mk[:self.nb], m_kq)
            occ0 = e_kq[:self.nb].copy()
            occ1 = grid.time_reverse(m_mkq, e_mkq[:self.nb], m_kq)
            beta = synth.projector_table(sysd, kq, m_kq)
            self.k.append(KData(k=kvec, kq=kq, mill=m_kq, kin=kin, u_real=[u0, u1],
                                u_sph=[us0, us1], eps=[et_k[:self.nb], et_mk[:self.nb]],
                                occ=[occ0, occ1], beta=beta))
        self.npw_pad = max(kd.npw for kd in self.k)

    # ---- vector helpers -------------------------------------------------
    def zeros(self):
        return np.zeros((2, self.nk, self.nb, 2, self.npw_pad), dtype=np.complex128)

    def dot(self, a, b):
        return np.vdot(a, b) / self.nk

    @staticmethod
    def J(a):
        out = a.copy()
        out[1] *= -1
        return out

    def project(self, side, ik, phi):
        occ = self.k[ik].occ[side]
        S = np.einsum("msg,nsg->mn", occ.conj(), phi)
        return phi - np.einsum("msg,mn->nsg", occ, S)

    def nonlocal_apply(self, ik, x):
        beta = self.k[ik].beta
        B = np.einsum("ig,nsg->ins", beta.conj(), x)
        W = np.einsum("ijst,jnt->ins", self.dmat, B)
        return np.einsum("ig,ins->nsg", beta, W)

    # ---- response density and potential ---------------------------------
    def response_density(self, xy):
        sysd = self.sysd
        sq = np.sqrt(sysd.omega)
        rho = np.zeros((4,) + tuple(sysd.fft), dtype=np.complex128)
        for ik, kd in enumerate(self.k):
            for s in range(2):
                x = grid.to_grid(sysd.fft, kd.mill, xy[s, ik, :, :, :kd.npw]) / sq
                u = kd.u_real[s]
                for a in range(4):
                    rho[a] += SIDE_SIGNS[s][a] * np.einsum(
                        "nsxyz,st,ntxyz->xyz", u.conj(), PAULI[a], x) / self.nk
        return rho

    def response_potential(self, rho, hartree=True, xc_on=True):
        W = np.zeros_like(rho)
        if hartree:
            W[0] += grid.apply_coulomb(self.hq, rho[0])
        if xc_on:
            W += np.einsum("ab...,b...->a...", self.f, rho)
        return W

    # ---- the Liouvillian ------------------------------------------------
    def apply(self, xy, kernel=True, hartree=True, xc_on=True):
        sysd = self.sysd
        sq = np.sqrt(sysd.omega)
        if kernel:
            W = self.response_potential(self.response_density(xy), hartree, xc_on)
        else:
            W = np.zeros((4,) + tuple(sysd.fft), dtype=np.complex128)
        out = self.zeros()
        for ik, kd in enumerate(self.k):
            for s in range(2):
                sg = 1.0 if s == 0 else -1.0
                xc_ = xy[s, ik, :, :, :kd.npw]
                x = grid.to_grid(sysd.fft, kd.mill, xc_) / sq
                u = kd.u_real[s]
                V0 = self.vrs[0] * PAULI[0][:, :, None, None, None] + sg * np.einsum(
                    "a...,ast->st...", self.vrs[1:], PAULI[1:])
                V1 = W[0] * PAULI[0][:, :, None, None, None] + sg * np.einsum(
                    "a...,ast->st...", W[1:], PAULI[1:])
                phi_r = np.einsum("st...,nt...->ns...", V0, x) + np.einsum("st...,nt...->ns...", V1, u)
                phi = grid.from_grid(sysd.fft, kd.mill, phi_r) * sq
                phi += (kd.kin[None, None, :] - kd.eps[s][:, None, None]) * xc_
                phi += self.nonlocal_apply(ik, xc_)
                phi = self.project(s, ik, phi)
                out[s, ik, :, :, :kd.npw] = sg * phi
        return out

    def apply_dagger(self, xy, **kw):
        """L^dag = J L J (JL is Hermitian)."""
        return self.J(self.apply(self.J(xy), **kw))

    # ---- start and measure vectors --------------------------------------
    def u_vector(self, lam):
        sig = DIRECTIONS[lam]
        u = self.zeros()
        for ik, kd in enumerate(self.k):
            for s in range(2):
                su = np.einsum("st,ntg->nsg", sig, kd.u_sph[s])
                u[s, ik, :, :, :kd.npw] = su if s == 0 else TR_PARITY[lam] * su
        return u

    def v_vector(self, mu):
        sig = DIRECTIONS[mu]
        v = self.zeros()
        for ik, kd in enumerate(self.k):
            for s in range(2):
                su = np.einsum("st,ntg->nsg", sig, kd.u_sph[s])
                if s == 1:
                    su = -TR_PARITY[mu] * su
                v[s, ik, :, :, :kd.npw] = self.project(s, ik, su)
        return v

    def project_all(self, xy):
        out = self.zeros()
        for ik, kd in enumerate(self.k):
            for s in range(2):
                out[s, ik, :, :, :kd.npw] = self.project(s, ik, xy[s, ik, :, :, :kd.npw])
        return out

    def occupied_overlap(self, xy):
        """max |U_occ^dag q| over sides and k (zero for a projected vector)."""
        m = 0.0
        for ik, kd in enumerate(self.k):
            for s in range(2):
                S = np.einsum("msg,nsg->mn", kd.occ[s].conj(), xy[s, ik, :, :, :kd.npw])
                m = max(m, np.abs(S).max())
        return m

    def random_projected(self, seed):
        v = synth.random_br(self.nk, self.nb, [kd.npw for kd in self.k], self.npw_pad, seed)
        return self.project_all(v)


def build_problem(gs, qcart=None, qset=None):
    sysd = gs.sysd
    if qset is None:
        qset = synth.qset_exact(sysd, np.zeros(3) if qcart is None else qcart)
    return Problem(gs, qset)
