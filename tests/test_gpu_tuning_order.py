"""Results of a system do not depend on which call tuned it.

The autotuner times the launch variants of a shape before the first tunable
launch of a system: the start vectors' projection, the first FP64 apply, a
chain's begin.  The contraction variants sum in different K splits, so a
launch issued before tuning could differ in the last bits from the same
launch after it, and a Lanczos chain amplifies such differences over its
steps.  Here a multi-lane chain is the first call on a shape no other test
uses; single-direction chains run afterwards must give the same coefficients
bit for bit, and start vectors taken before and after must be equal.
"""
import numpy as np
import pytest

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu


def _desc(tm, nbnd):
    sysd = synth.make_cubic(24, nbnd, 1)
    inp = synth.synthetic_inputs_multi(sysd, np.array([[0.1, 0.05, 0.0]]) * 2 * np.pi / 10.0, seed=3)
    pts = [tm.Point(xk=p, mill=m, evc=e, et=et, vkb=v) for (p, m, e, et, v) in inp["points"]]
    return tm.SystemDesc(cell=sysd.cell, fft=sysd.fft, nbnd=sysd.nbnd, points=pts, vrs=inp["vrs"],
                         rho=inp["rho"], dvan=inp["dvan"], xq=inp["xq"], roles=inp["roles"],
                         shifts=inp["shifts"])


def _tuned(tm, nbnd):
    return [e for e in tm.tm_autotune_report() if f"24x24x24, {nbnd} bands" in e["shape"]]


def test_chain_that_tunes_equals_chains_after_it():
    import torch
    import paper_2203_01120_amd as tm
    tm.load()
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    assert not _tuned(tm, 10), "another test already tuned this shape"
    h = tm.tm_system_create(_desc(tm, 10))
    try:
        steps = 24
        say(f"lanes z, y pH {steps} steps as the first call on grid 24^3, 10 bands")
        lanes = tm.tm_tensor_run(h, 0, ["z", "y"], "pH", steps)
        assert _tuned(tm, 10), "the chain's begin did not tune the system"
        for lane, direction in zip(lanes, ["z", "y"]):
            single = tm.tm_lanczos_run(h, 0, direction, "pH", steps)
            for key in ("alpha", "beta", "gamma", "z"):
                assert np.array_equal(lane[key], single[key]), (direction, key)
            assert lane["n1"] == single["n1"]
    finally:
        tm.tm_system_destroy(h)


def test_start_vectors_before_any_apply_equal_later_ones():
    import torch
    import paper_2203_01120_amd as tm
    tm.load()
    assert not _tuned(tm, 6), "another test already tuned this shape"
    h = tm.tm_system_create(_desc(tm, 6))
    try:
        say("start vectors as the first call on grid 24^3, 6 bands")
        n = tm.tm_qset_info_get(h, 0)["nelem"]
        first = torch.empty(n, dtype=torch.complex128, device="cuda")
        tm.tm_start_vectors(h, 0, "x", None, first)
        assert _tuned(tm, 6), "tm_start_vectors with v did not tune the system"
        y = torch.empty_like(first)
        tm.tm_liouvillian_apply(h, 0, first, y)
        again = torch.empty_like(first)
        tm.tm_start_vectors(h, 0, "x", None, again)
        torch.cuda.synchronize()
        assert torch.equal(first, again)
    finally:
        tm.tm_system_destroy(h)
