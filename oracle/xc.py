"""Slater-exchange LSDA potentials and the adiabatic response kernel (oracle).

The paper works in the adiabatic LSDA (Sec. 2.2, Eqs. v_XC_q and b_XC_q: the
response potentials are the derivatives of v_xc and b_xc with respect to n
and m at the ground state).  The functional used here is Dirac/Slater
exchange with the usual spin scaling:

    e_x(n_up, n_dn) = -(3/4) (6/pi)^{1/3} (n_up^{4/3} + n_dn^{4/3}),
    n_up/dn = (n +- s) / 2,  s = |m|,  m = psi^dag sigma psi.

Hamiltonian term: v_xc sigma_0 + B . sigma with v_xc = de/dn and B = de/dm
(so B = -b_xc of the paper with mu_B = 1).

Thresholds (the paper is silent): n < NMIN -> all xc quantities 0;
s < SREL * n -> isotropic limit (no B, kernel e_nn sigma_0 + e_ss identity);
spin densities clamped to >= 0 in v and to >= NSIG_MIN in dv/dn.
"""
from __future__ import annotations

import numpy as np

CX = (6.0 / np.pi) ** (1.0 / 3.0)
NMIN = 1e-10
SREL = 1e-10
NSIG_MIN = 1e-12


def _split(rho):
    n = rho[0]
    m = rho[1:4]
    s = np.sqrt(np.sum(m * m, axis=0))
    return n, m, s


def energy_density(rho):
    n, m, s = _split(rho)
    nu = np.maximum(0.5 * (n + s), 0.0)
    nd = np.maximum(0.5 * (n - s), 0.0)
    e = -0.75 * CX * (nu ** (4.0 / 3.0) + nd ** (4.0 / 3.0))
    return np.where(n < NMIN, 0.0, e)


def potentials(rho):
    """(v_xc, B[3]) from rho = (n, m_x, m_y, m_z) on the grid."""
    n, m, s = _split(rho)
    nu = np.maximum(0.5 * (n + s), 0.0)
    nd = np.maximum(0.5 * (n - s), 0.0)
    vu = -CX * np.cbrt(nu)
    vd = -CX * np.cbrt(nd)
    vxc = 0.5 * (vu + vd)
    mag = s >= SREL * n
    sd = np.where(mag, s, 1.0)
    bmag = np.where(mag, 0.5 * (vu - vd), 0.0)
    B = bmag * m / sd
    vxc = np.where(n < NMIN, 0.0, vxc)
    B = np.where(n < NMIN, 0.0, B)
    return vxc, B


def kernel(rho):
    """Response kernel f[a][b] (4x4, real symmetric per grid point).

    W_a = sum_b f_ab rho'_b gives the xc part of V' = W_0 sigma_0 + W . sigma:
      f_nn = e_nn,  f_n,i = e_ns mhat_i,
      f_ij = e_ss mhat_i mhat_j + (e_s/s)(delta_ij - mhat_i mhat_j),
    with g_sigma = dv_sigma/dn_sigma = -(1/3) CX n_sigma^{-2/3},
    e_nn = e_ss = (g_up + g_dn)/4, e_ns = (g_up - g_dn)/4,
    e_s/s = (v_up - v_dn)/(2 s)  (the same v_sigma as the ground-state B, so
    that a rigid rotation of m is a zero mode).
    """
    n, m, s = _split(rho)
    nu = np.maximum(0.5 * (n + s), 0.0)
    nd = np.maximum(0.5 * (n - s), 0.0)
    vu = -CX * np.cbrt(nu)
    vd = -CX * np.cbrt(nd)
    gu = -(CX / 3.0) * np.maximum(nu, NSIG_MIN) ** (-2.0 / 3.0)
    gd = -(CX / 3.0) * np.maximum(nd, NSIG_MIN) ** (-2.0 / 3.0)
    enn = 0.25 * (gu + gd)
    ess = 0.25 * (gu + gd)
    ens = 0.25 * (gu - gd)
    mag = s >= SREL * n
    sd = np.where(mag, s, 1.0)
    mh = np.where(mag, m / sd, 0.0)
    es_s = np.where(mag, 0.5 * (vu - vd) / sd, ess)
    ens = np.where(mag, ens, 0.0)
    f = np.zeros((4, 4) + n.shape)
    f[0, 0] = enn
    for i in range(3):
        f[0, i + 1] = ens * mh[i]
        f[i + 1, 0] = ens * mh[i]
        for j in range(3):
            f[i + 1, j + 1] = ess * mh[i] * mh[j] + es_s * ((i == j) - mh[i] * mh[j])
    f = np.where(n < NMIN, 0.0, f)
    return f
