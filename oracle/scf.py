"""Dense-matrix noncollinear Kohn-Sham ground state (oracle).

The ground-state Hamiltonian of Sec. 2.2 (Eq. H0_k_plus_q) in the plane-wave
spinor basis {|k+G, s>}, ordered [s][G]:

    H_k = sigma_0 [ |k+G|^2/2 + v_loc + v_H + v_xc ] + V_NL,k + B . sigma

with v_loc the synthetic local potential, v_H(G) = 4 pi n(G) / |G|^2 (G = 0
dropped), v_xc and B from Slater LSDA (``oracle.xc``), and the
Kleinman-Bylander term V_NL = sum_ij |beta_i> D_ij <beta_j| with 2x2 spin
blocks D_ij.  Local fields act as circular convolutions on the FFT grid.
Occupations are the lowest ``nbnd`` spinor bands at every k (insulator
formalism, Sec. 2.1).  Density mixing is Pulay/DIIS on (n, m).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

import synth
from . import grid, xc

PAULI = np.array([[[1, 0], [0, 1]],
                  [[0, 1], [1, 0]],
                  [[0, -1j], [1j, 0]],
                  [[1, 0], [0, -1]]], dtype=np.complex128)


def conv_matrix(F, fft, mill):
    """M[g, g'] = F[(m_g - m_g') mod n]: the matrix of a grid field on the sphere."""
    d = mill[:, None, :] - mill[None, :, :]
    return F[d[..., 0] % fft[0], d[..., 1] % fft[1], d[..., 2] % fft[2]]


def hamiltonian(sysd, kcart, mill, vrs, beta, dmat, bsign=1.0):
    """Dense H_k [2 npw][2 npw]; bsign = -1 flips the B field."""
    npw = mill.shape[0]
    fft = sysd.fft
    Fs = [grid.field_fourier(vrs[a]) for a in range(4)]
    V = conv_matrix(Fs[0], fft, mill)
    Bx, By, Bz = (bsign * conv_matrix(Fs[a], fft, mill) for a in (1, 2, 3))
    K = np.asarray(kcart) + mill @ sysd.recip
    T = 0.5 * np.einsum("ij,ij->i", K, K)
    H = np.zeros((2 * npw, 2 * npw), dtype=np.complex128)
    H[:npw, :npw] = V + Bz + np.diag(T)
    H[npw:, npw:] = V - Bz + np.diag(T)
    H[:npw, npw:] = Bx - 1j * By
    H[npw:, :npw] = Bx + 1j * By
    for s in range(2):
        for t in range(2):
            H[s * npw:(s + 1) * npw, t * npw:(t + 1) * npw] += \
                beta.T @ dmat[:, :, s, t] @ beta.conj()
    return H


def density_from_states(sysd, states, weight):
    """rho = (n, m) with n = sum |U|^2, m = sum U^dag sigma U, U = Omega^{-1/2} psi."""
    rho = np.zeros((4,) + tuple(sysd.fft))
    for mill, evc in states:
        psi = grid.to_grid(sysd.fft, mill, evc)  # [nb][2][grid]
        up, dn = psi[:, 0], psi[:, 1]
        z = np.conj(up) * dn
        rho[0] += weight * np.sum(np.abs(up) ** 2 + np.abs(dn) ** 2, axis=0)
        rho[1] += weight * np.sum(2 * z.real, axis=0)
        rho[2] += weight * np.sum(2 * z.imag, axis=0)
        rho[3] += weight * np.sum(np.abs(up) ** 2 - np.abs(dn) ** 2, axis=0)
    return rho / sysd.omega


def hartree(sysd, n):
    h = grid.coulomb_multiplier(sysd, np.zeros(3))
    return np.real(grid.apply_coulomb(h, n))


def potentials(sysd, vloc, rho):
    """vrs = (v_eff, B_x, B_y, B_z) from the density."""
    vxc, B = xc.potentials(rho)
    veff = vloc + hartree(sysd, rho[0]) + vxc
    return np.concatenate([veff[None], B])


class Pulay:
    def __init__(self, beta=0.3, nhist=8):
        self.beta, self.nhist = beta, nhist
        self.X, self.R = [], []

    def step(self, x_in, x_out):
        self.X.append(x_in.copy())
        self.R.append(x_out - x_in)
        self.X, self.R = self.X[-self.nhist:], self.R[-self.nhist:]
        n = len(self.R)
        A = np.zeros((n + 1, n + 1))
        for i in range(n):
            for j in range(n):
                A[i, j] = np.vdot(self.R[i], self.R[j]).real
        A[:n, :n] /= max(np.max(np.diag(A[:n, :n])), 1e-300)
        A[:n, n] = A[n, :n] = 1.0
        b = np.zeros(n + 1)
        b[n] = 1.0
        c = np.linalg.lstsq(A, b, rcond=None)[0][:n]
        return sum(ci * (x + self.beta * r) for ci, x, r in zip(c, self.X, self.R))


@dataclass
class GroundState:
    sysd: object
    vloc: np.ndarray
    vrs: np.ndarray
    rho: np.ndarray
    residual: float
    niter: int
    mesh_states: list = field(default_factory=list)   # per mesh k: (kcart, mill, evc, et)
    dmat: np.ndarray = None

    def beta(self, kcart, mill):
        return synth.projector_table(self.sysd, kcart, mill)

    def hamiltonian(self, kcart, mill=None, bsign=1.0):
        mill = synth.sphere(self.sysd, kcart) if mill is None else mill
        return hamiltonian(self.sysd, kcart, mill, self.vrs, self.beta(kcart, mill),
                           self.dmat, bsign)

    def solve(self, kcart, nbands=None, mill=None):
        """Non-SCF states at k: (mill, evc [nb][2][npw], et [nb])."""
        mill = synth.sphere(self.sysd, kcart) if mill is None else mill
        H = self.hamiltonian(kcart, mill)
        npw = mill.shape[0]
        nb = self.sysd.nbnd if nbands is None else nbands
        if nb >= 2 * npw:
            e, v = sla.eigh(H)
        else:
            e, v = sla.eigh(H, subset_by_index=[0, nb - 1])
        evc = np.ascontiguousarray(v.T.reshape(-1, 2, npw))
        return mill, evc, e

    @property
    def magnetization(self):
        """Total moment per cell, M = int m dr (units where m = psi^dag sigma psi)."""
        return self.rho[1:4].reshape(3, -1).sum(axis=1) * self.sysd.omega / self.sysd.ngrid

    @property
    def nelec(self):
        return self.rho[0].sum() * self.sysd.omega / self.sysd.ngrid


def initial_density(sysd, mfrac=(0.0, 0.0, 0.5)):
    g = synth.systems._image_sum(sysd, lambda r2, at: np.exp(-r2 / (2 * (1.5 * at.width) ** 2)))
    if g.sum() > 0:
        n = 0.5 * g / (g.sum() * sysd.omega / sysd.ngrid) + 0.5 / sysd.omega
    else:  # no atoms: start from the uniform density
        n = np.full(g.shape, 1.0 / sysd.omega)
    n *= sysd.nbnd
    rho = np.zeros((4,) + n.shape)
    rho[0] = n
    for i in range(3):
        rho[i + 1] = mfrac[i] * n
    return rho


def scf(sysd, tol=1e-10, maxiter=300, mfrac=(0.0, 0.0, 0.5), beta=0.3, nhist=8,
        verbose=False):
    """Self-consistent noncollinear LSDA ground state on the SCF k-mesh."""
    kpts = synth.kmesh_cart(sysd)
    mills = [synth.sphere(sysd, k) for k in kpts]
    betas = [synth.projector_table(sysd, k, m) for k, m in zip(kpts, mills)]
    dmat = synth.dmatrix(sysd)
    vloc = synth.vloc_grid(sysd)
    rho = initial_density(sysd, mfrac)
    mixer = Pulay(beta, nhist)
    w = 1.0 / len(kpts)
    res = np.inf
    for it in range(1, maxiter + 1):
        vrs = potentials(sysd, vloc, rho)
        states = []
        for k, m, b in zip(kpts, mills, betas):
            H = hamiltonian(sysd, k, m, vrs, b, dmat)
            e, v = sla.eigh(H, subset_by_index=[0, sysd.nbnd])
            states.append((k, m, np.ascontiguousarray(v[:, :sysd.nbnd].T.reshape(-1, 2, m.shape[0])), e))
        rho_out = density_from_states(sysd, [(s[1], s[2]) for s in states], w)
        res = np.sqrt(np.sum((rho_out - rho) ** 2) * sysd.omega / sysd.ngrid)
        if verbose:
            print(f"scf {it:3d} res {res:.3e}")
        if res < tol:
            break
        rho = mixer.step(rho, rho_out)
    gs = GroundState(sysd=sysd, vloc=vloc, vrs=vrs, rho=rho, residual=res, niter=it,
                     dmat=dmat)
    gs.mesh_states = [(k, m, evc, e[:sysd.nbnd]) for k, m, evc, e in states]
    gs.gaps = [e[sysd.nbnd] - e[sysd.nbnd - 1] for _, _, _, e in states]
    return gs
