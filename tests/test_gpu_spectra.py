"""Extrapolated susceptibility and S(q, omega) through the C ABI (needs an MI355X).

Same coefficients in, so the GPU solver and the oracle's zgtsv (both
Gaussian elimination with partial pivoting, in different operation orders)
agree to their forward error: at every frequency and measure row, within
2 c u kappa(A) |n_1| ||z|| ||x|| (tests/chi_bound.py, pinned on the CPU with
two solvers), which grows with the condition of (w + i eta) I - T and so
with the length of the (extrapolated) chain.
"""
import numpy as np
import pytest

from oracle import chi as ochi
from oracle import liouvillian as lv

import chi_bound as cb
from gpu_util import desc_from_problem, rel_err, say

pytestmark = pytest.mark.gpu

EV = 27.211386245988


@pytest.fixture(scope="module")
def cubic(cubic_gs, cubic_q):
    import torch
    import paper_2203_01120_amd as tm
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    prob = lv.build_problem(cubic_gs, cubic_q)
    h = tm.tm_system_create(desc_from_problem(prob))
    yield tm, prob, h
    tm.tm_system_destroy(h)


@pytest.mark.parametrize("mode", ["constant", "osc"])
def test_extrapolated_chi_matches_oracle(cubic, mode):
    tm, prob, h = cubic
    say(f"extrapolated chi ({mode})")
    c = tm.tm_lanczos_run(h, 0, "+", "pH", 60)
    omega = np.arange(400) * 5e-3 / EV
    eta = 5e-3 / EV
    for m_use, m_total in ((60, 60), (60, 2000), (24, 500)):
        got = tm.tm_chi_extrapolated(c, m_use, m_total, mode if m_total > m_use else "no", omega, eta)
        e = ochi.extrapolate(c, m_use, m_total, mode)
        ref = ochi.chi_lanczos(e, omega, eta, m_total)
        bound = cb.chi_difference_bound(e, m_total, omega, eta)
        say(f"  {m_use} -> {m_total}: rel err {rel_err(got, ref):.2e}, "
            f"largest |diff| / bound {(np.abs(got - ref) / np.maximum(bound, 1e-300)).max():.2e}")
        assert np.all(np.abs(got - ref) <= bound), (m_use, m_total, rel_err(got, ref))
    # a closed-form chain through the GPU solver: constant tail -> infinite-chain Green's function
    a, b, e2 = 0.3, 0.5, 0.05
    z = np.zeros((3, 8), complex)
    z[0, 0] = 1.0
    co = dict(alpha=np.full(8, a, complex), beta=np.full(8, b), gamma=np.full(8, b, complex), z=z, n1=1.0,
              steps_done=8)
    w = np.linspace(-1.5, 2.0, 71)
    got = tm.tm_chi_extrapolated(co, 8, 3000, "constant", w, e2)[0]
    wc = w + 1j * e2
    r = np.sqrt((wc - a) ** 2 - 4 * b * b)
    G = np.where(((wc - a - r) / (2 * b * b)).imag < 0, (wc - a - r) / (2 * b * b), (wc - a + r) / (2 * b * b))
    assert np.abs(got - G).max() <= 1e-8 * np.abs(G).max()


def test_chi_tensor_extrapolated_matches_oracle(cubic):
    """The 4 x 4 column (rows n, x, y, z) with the bi-constant extrapolation."""
    tm, prob, h = cubic
    say("chi tensor column, extrapolated")
    c = tm.tm_lanczos_run(h, 0, "n", "pH", 40)
    omega = np.arange(300) * 5e-3 / EV
    eta = 5e-3 / EV
    got = tm.tm_chi_tensor(c, 40, omega, eta, m_total=1000, mode="osc")
    four = dict(c, z=np.vstack([c["zn"][None], c["z"]]))
    e = ochi.extrapolate(four, 40, 1000, "osc")
    ref = ochi.chi_lanczos(e, omega, eta, 1000)
    assert np.all(np.abs(got - ref) <= cb.chi_difference_bound(e, 1000, omega, eta)), rel_err(got, ref)
    with pytest.raises(tm.TmError):
        tm.tm_chi_tensor(dict(c, zn=None), 40, omega, eta)


def test_structure_factor_matches_oracle(cubic):
    tm, prob, h = cubic
    say("structure factor from three chains")
    omega = np.linspace(0.0, 0.1, 64)
    eta = 1e-3
    chi3 = np.zeros((3, 3, omega.size), complex)
    for mu_i, mu in enumerate("xyz"):
        c = tm.tm_lanczos_run(h, 0, mu, "nH", 16)
        chi3[:, mu_i, :] = tm.tm_chi(c, 16, omega, eta)
    q = np.asarray(prob.qset.q, float)
    got = tm.tm_structure_factor(q, chi3)
    ref = ochi.structure_factor(q, chi3)
    assert np.abs(got - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1e-300)
    with pytest.raises(tm.TmError):
        tm.tm_structure_factor(np.zeros(3), chi3)
    c = tm.tm_lanczos_run(h, 0, "z", "nH", 8)
    with pytest.raises(tm.TmError):
        tm.tm_chi_extrapolated(c, 8, 6, "constant", omega, eta)
