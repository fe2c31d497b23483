"""Pin P12: the Lanczos coefficients of a long chain settle at the spectral edges.

For an operator whose spectrum fills [W_min, W_max], the recursion
coefficients of a Lanczos chain tend to alpha -> (W_min + W_max) / 2 and
beta -> (W_max - W_min) / 4 (the Jacobi-matrix limit of a measure on an
interval); the paper's long chains show beta oscillating about such a
constant (Sec. 5.5), which is what the constant and bi-constant
extrapolations of the coefficients assume.  Here the spectrum of L is
computed independently from the dense transition-space matrix of a small
system (954 transitions, eigenvalues +-W in pairs, so the centre is 0), and
300-step chains of both flavours must sit at its centre and quarter-width:
mean beta over steps 50..299 within 10 % of (W_max - W_min) / 4, mean alpha
within 1 % of the width from the centre.  A chain with L scaled or shifted
by a planted error (here: the kinetic term dropped) misses both.
"""
import numpy as np
import pytest

import synth
from oracle import dense
from oracle import lanczos as olanczos
from oracle import liouvillian as lv
from oracle import scf


@pytest.fixture(scope="module")
def small():
    gs = scf.scf(synth.make_tiny(ecut=4.0, fft=(12, 12, 12)), tol=1e-11, beta=0.5)
    prob = lv.build_problem(gs, np.array([0.1, 0.05, 0.0]) * 2 * np.pi / 6.0)
    lam = np.linalg.eigvals(dense.TransitionSpace(prob).liouvillian())
    assert np.abs(lam.imag).max() <= 1e-10 * np.abs(lam).max()
    return prob, lam.real.min(), lam.real.max()


@pytest.mark.parametrize("mu,flavour", [("z", "pH"), ("x", "nH")])
def test_beta_asymptote(small, mu, flavour):
    prob, wmin, wmax = small
    c = olanczos.run(prob, mu, flavour, 300)
    assert c["steps_done"] == 300
    b = c["beta"][50:300].mean()
    a = c["alpha"][50:300].real.mean()
    width = wmax - wmin
    assert abs(b / (width / 4) - 1) <= 0.1, (b, width / 4)
    assert abs(a - 0.5 * (wmin + wmax)) <= 0.01 * width, a


def test_beta_asymptote_catches_a_planted_error(small):
    prob, wmin, wmax = small
    kin = [kd.kin.copy() for kd in prob.k]
    try:
        for kd in prob.k:
            kd.kin[:] = 0.0        # planted: kinetic term dropped from L
        c = olanczos.run(prob, "z", "pH", 300)
    finally:
        for kd, k0 in zip(prob.k, kin):
            kd.kin[:] = k0
    n = c["steps_done"]
    b = c["beta"][min(50, n // 2):n].mean()
    assert abs(b / ((wmax - wmin) / 4) - 1) > 0.1
