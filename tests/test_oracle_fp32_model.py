"""The single-precision error model (tests/fp32_noise.py) on the oracle.

* The stored bounds (tests/golden/fp32_bound.json) are reproduced: one seed
  of each chain recomputed here gives the stored deviation.
* The model's deviation is linear in the perturbation size (halving the
  noise halves the L2 error within 20 %), so the bound scales with the
  assumed unit roundoff as a first-order error should.
* Without noise the perturbed chain is the unperturbed one (eps = 0).
"""
import json
import os

import numpy as np
import pytest

import fp32_noise as fn

HERE = os.path.dirname(os.path.abspath(__file__))
STORED = json.load(open(os.path.join(HERE, "golden", "fp32_bound.json")))


@pytest.fixture(scope="module")
def cubic_prob(cubic_gs, cubic_q):
    from oracle import liouvillian as lv
    return lv.build_problem(cubic_gs, cubic_q)


@pytest.mark.parametrize("flavour,mu,seed", [("pH", "+", 5), ("nH", "z", 3)])
def test_stored_bound_reproduced(cubic_prob, flavour, mu, seed):
    m = STORED["steps"]
    ref = fn.chain(cubic_prob, mu, flavour, m)
    got = fn.chain(cubic_prob, mu, flavour, m, seed=seed)
    l2, shift = fn.spectrum_error(ref, got, m)
    row = [r for r in STORED["chains"][f"{flavour}{mu}"]["per_seed"] if r["seed"] == seed][0]
    assert l2 == pytest.approx(row["l2_rel_im_chi"], rel=1e-6)
    assert (shift is None) == (row["peak_shift_meV"] is None)
    if shift is not None:
        assert shift == pytest.approx(row["peak_shift_meV"], abs=1e-9)
    c = STORED["chains"][f"{flavour}{mu}"]
    assert c["bound_l2"] >= 2 * c["l2_max"] * 0.95


def test_model_is_first_order(cubic_prob):
    m = 30
    ref = fn.chain(cubic_prob, "+", "pH", m)
    a, _ = fn.spectrum_error(ref, fn.chain(cubic_prob, "+", "pH", m, seed=1, eps=fn.U32), m)
    b, _ = fn.spectrum_error(ref, fn.chain(cubic_prob, "+", "pH", m, seed=1, eps=fn.U32 / 2), m)
    assert 0.4 <= b / a <= 0.6, (a, b)
    zero = fn.chain(cubic_prob, "+", "pH", m, seed=1, eps=0.0)
    for k in ("alpha", "beta"):
        assert np.array_equal(zero[k], ref[k])
