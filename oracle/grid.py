"""Sphere <-> grid transforms (oracle).

A lattice-periodic spinor component is U(r) = Omega^{-1/2} sum_G c(G) exp(iG.r)
with G on the plane-wave sphere (Sec. 2.2 defines the periodic parts U of the
Bloch spinors).  On the FFT grid the sum is a plain backward DFT, so
``to_grid`` returns psi(r_j) = sum_G c(G) exp(iG.r_j) (no Omega factor) and
``from_grid`` is its inverse, c(G) = (1/N) sum_j f(r_j) exp(-iG.r_j).
Products of grid functions are therefore circular convolutions in G, which
is how the operator is defined at finite grid size.

The transforms are scipy.fft's (the same discrete Fourier sums as numpy.fft,
pinned against a direct DFT sum in the tests), run on every host thread the
process may use.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def _fftn(a, axes=None):
    return sfft.fftn(a, axes=axes, workers=WORKERS)


def _ifftn(a, axes=None):
    return sfft.ifftn(a, axes=axes, workers=WORKERS)


def grid_index(fft, mill):
    n = np.asarray(fft)
    m = np.asarray(mill)
    return m[:, 0] % n[0], m[:, 1] % n[1], m[:, 2] % n[2]


def to_grid(fft, mill, coef):
    """coef [..., npw] on the sphere -> psi [..., n1, n2, n3] = sum_G c(G) e^{iG.r}."""
    coef = np.asarray(coef)
    lead = coef.shape[:-1]
    g = np.zeros(lead + tuple(fft), dtype=np.complex128)
    i1, i2, i3 = grid_index(fft, mill)
    g[..., i1, i2, i3] = coef
    return _ifftn(g, axes=(-3, -2, -1)) * np.prod(fft)


def from_grid(fft, mill, f):
    """f [..., n1, n2, n3] -> c [..., npw] = (1/N) sum_j f(r_j) e^{-iG.r_j}."""
    F = _fftn(f, axes=(-3, -2, -1)) / np.prod(fft)
    i1, i2, i3 = grid_index(fft, mill)
    return F[..., i1, i2, i3]


def field_fourier(f):
    """Fourier coefficients F[m mod n] = (1/N) sum_j f(r_j) e^{-iG.r_j} of a grid field."""
    return _fftn(f, axes=(-3, -2, -1)) / f.shape[-1] / f.shape[-2] / f.shape[-3]


def grid_gvectors(sysd):
    """Cartesian G of every grid index (canonical Miller m in [-n/2, n/2)) and a
    mask that is False on the Nyquist planes of even-sized axes."""
    n1, n2, n3 = sysd.fft
    ms = []
    ok = []
    for n in (n1, n2, n3):
        i = np.arange(n)
        m = np.where(i < (n + 1) // 2, i, i - n)
        ms.append(m)
        ok.append(~((n % 2 == 0) & (i == n // 2)))
    M = np.stack(np.meshgrid(*ms, indexing="ij"), axis=-1)
    mask = ok[0][:, None, None] & ok[1][None, :, None] & ok[2][None, None, :]
    return M @ sysd.recip, mask


def coulomb_multiplier(sysd, qcart):
    """4 pi / |G+q|^2 on the grid (Eq. v_H_q in reciprocal space); 0 on Nyquist
    planes and where G+q = 0 (the neutralising background)."""
    G, mask = grid_gvectors(sysd)
    K = G + np.asarray(qcart, dtype=float)
    k2 = np.einsum("...i,...i->...", K, K)
    h = np.zeros_like(k2)
    good = mask & (k2 > 1e-12)
    h[good] = 4 * np.pi / k2[good]
    return h


def apply_coulomb(h, f):
    """Grid function f -> inverse FFT of h(G) * FFT(f)."""
    return _ifftn(h * _fftn(f))


def miller_lookup(mill):
    return {tuple(m): i for i, m in enumerate(np.asarray(mill).tolist())}


def restrict(mill_from, coef, mill_to):
    """Copy coefficients [..., npw_from] onto sphere mill_to (zeros where missing)."""
    lut = miller_lookup(mill_from)
    idx = np.array([lut.get(tuple(m), -1) for m in np.asarray(mill_to).tolist()])
    out = np.zeros(coef.shape[:-1] + (len(idx),), dtype=np.complex128)
    have = idx >= 0
    out[..., have] = coef[..., idx[have]]
    return out


def time_reverse(mill_from, coef, mill_to):
    """T = i sigma_y K on spinor coefficients [..., 2, npw_from] (Sec. 2.2).

    (T U)(r) = i sigma_y U*(r): in G space (TU)_up(G) = conj(U_dn(-G)) and
    (TU)_dn(G) = -conj(U_up(-G)).  The result is placed on sphere mill_to
    (zeros where -G is missing from mill_from).
    """
    lut = miller_lookup(mill_from)
    idx = np.array([lut.get(tuple(-m for m in mm), -1) for mm in np.asarray(mill_to).tolist()])
    out = np.zeros(coef.shape[:-2] + (2, len(idx)), dtype=np.complex128)
    have = idx >= 0
    out[..., 0, have] = np.conj(coef[..., 1, idx[have]])
    out[..., 1, have] = -np.conj(coef[..., 0, idx[have]])
    return out


def time_reverse_real(psi):
    """T on real-space spinors [..., 2, n1, n2, n3]: (a, b) -> (conj b, -conj a)."""
    out = np.empty_like(psi)
    out[..., 0, :, :, :] = np.conj(psi[..., 1, :, :, :])
    out[..., 1, :, :, :] = -np.conj(psi[..., 0, :, :, :])
    return out
