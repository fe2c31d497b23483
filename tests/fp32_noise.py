"""Error model of the single-precision bulk mode, run on the FP64 oracle.

An apply whose bulk runs in single precision returns L x plus a rounding
perturbation.  Its size is modelled as a backward error of the whole
operator at single-precision unit roundoff u = 2^-24: ||delta|| =
u * Lam * ||x||, with Lam the largest kinetic energy on the response spheres
(the scale of ||L||), in a direction drawn at random (complex Gaussian,
seeded).  This overstates the measured single-precision apply error (about
2e-8 relative to max |L x|, while u * Lam * ||x|| >= u ||L x||), so the
spread of the resulting spectra bounds what the GPU mode may deviate.

Each chain is the oracle's own recursion (pseudo-Hermitian or
non-Hermitian) with the perturbed apply in place of L; the spectrum error is
measured exactly as the GPU single-precision test measures it: the relative
L2 difference of Im chi over 400 frequencies 0..1.995 eV with eta = 5 meV,
and the shift of the strongest interior peak of |Im chi| located on a
0.01 meV grid within 10 meV.
"""
from __future__ import annotations

import numpy as np

from oracle import chi as ochi
from oracle import lanczos as olanczos

EV = 27.211386245988
U32 = 2.0 ** -24
OMEGA = np.arange(400) * 5e-3 / EV
ETA = 5e-3 / EV


def _noisy(apply, prob, rng, lam, eps):
    mask = np.zeros(prob.zeros().shape, dtype=bool)
    for ik, kd in enumerate(prob.k):
        mask[:, ik, :, :, :kd.npw] = True

    def ap(x):
        y = apply(x)
        xi = (rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape)) * mask
        return y + (eps * lam * np.linalg.norm(x) / np.linalg.norm(xi)) * xi
    return ap


def chain(prob, mu, flavour, m, seed=None, eps=U32):
    """Oracle chain; with a seed, every apply is perturbed by the model's noise."""
    v = prob.v_vector(mu)
    us = [prob.u_vector(l) for l in ("x", "y", "z")]
    lam = olanczos.operator_scale(prob)
    ap = prob.apply
    apd = prob.apply_dagger
    if seed is not None:
        rng = np.random.default_rng(seed)
        ap = _noisy(prob.apply, prob, rng, lam, eps)
        apd = _noisy(prob.apply_dagger, prob, rng, lam, eps)
    if flavour == "pH":
        return olanczos.pseudo_hermitian(ap, v, us, m, prob.dot, prob.J, lam, prob.project_all)
    return olanczos.non_hermitian(ap, apd, v, us, m, prob.dot, lam, prob.project_all)


def strongest_peak(chi):
    """(component, omega) of the largest interior local maximum of |Im chi| on
    OMEGA, or None when no component has one above zero (a longitudinal
    spectrum that only falls off, components that vanish by symmetry)."""
    a = np.abs(chi.imag)
    best = None
    for c in range(a.shape[0]):
        for i in range(1, a.shape[1] - 1):
            if a[c, i] > 0 and a[c, i] >= a[c, i - 1] and a[c, i] >= a[c, i + 1] and (
                    best is None or a[c, i] > best[2]):
                best = (c, i, a[c, i])
    return None if best is None else (best[0], OMEGA[best[1]])


def peak(coeffs, m, w0, comp):
    w = w0 + np.arange(-1000, 1001) * 1e-5 / EV
    c = np.abs(ochi.chi_lanczos(coeffs, w, ETA, m)[comp].imag)
    return w[int(np.argmax(c))]


def spectrum_error(ref, got, m):
    """(relative L2 of Im chi, peak shift in meV or None without a peak) of
    chain `got` against chain `ref`."""
    x0 = ochi.chi_lanczos(ref, OMEGA, ETA, m)
    x1 = ochi.chi_lanczos(got, OMEGA, ETA, m)
    l2 = float(np.linalg.norm(x1.imag - x0.imag) / np.linalg.norm(x0.imag))
    pk = strongest_peak(x0)
    if pk is None:
        return l2, None
    comp, w0 = pk
    shift = float(abs(peak(got, m, w0, comp) - peak(ref, m, w0, comp)) * EV * 1e3)
    return l2, shift
