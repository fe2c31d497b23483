"""The batched q-path form (72 chains) against single chains and the oracle.

The benchmark's batched form on the 20^3 system with 24 q along
Gamma-M-K-Gamma: one system holding the 24 q sets, the three directions
(m_+, m_-, m_z) of a q set as the lanes of one chain, all 24 chains stepped
together over three workspace slots (the launch configuration the q-path
benchmark times).  Every lane's coefficients equal the single chain of its
direction run alone bit for bit (same kernels, same per-right-hand-side
arithmetic), and three chains sampled along the path (q indices 0, 11 and
23, each with another direction) match the oracle's pseudo-Hermitian
recursion on the same synthetic inputs.

Near Gamma the chain is ill-conditioned: a relative change of 1e-16 in its
start vector (no change at all in exact arithmetic) moves single
coefficients by O(1) after some 15 steps, while chi barely moves.  So the
coefficients are compared at 1e-10 over the steps the oracle itself shows to
be fixed by the data to 1e-12 (its chain run twice, the second time from a
start vector scaled by 1 + 2^-50), and chi(omega) over all steps at 100 times
the oracle's own drift between those two runs (at least 1e-10).
"""
import numpy as np
import pytest

import synth
from oracle import chi as ochi
from oracle import lanczos as olanczos
from oracle import liouvillian as lv

from gpu_util import say

pytestmark = pytest.mark.gpu

STEPS = 40
DIRS = ["+", "-", "z"]


@pytest.fixture(scope="module")
def qpath():
    import torch
    import paper_2203_01120_amd as tm
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    sysd = synth.make_cubic20()
    qs = np.array([synth.cart_from_frac(sysd, f) for f in synth.q_path(24)])
    say("q path: building inputs (24 q sets)")
    inp = synth.synthetic_inputs_multi(sysd, qs, seed=1)
    pts = [tm.Point(xk=p, mill=m, evc=e, et=et, vkb=v) for (p, m, e, et, v) in inp["points"]]
    desc = tm.SystemDesc(cell=sysd.cell, fft=sysd.fft, nbnd=sysd.nbnd, points=pts, vrs=inp["vrs"],
                         rho=inp["rho"], dvan=inp["dvan"], xq=inp["xq"], roles=inp["roles"], shifts=inp["shifts"])
    h = tm.tm_system_create(desc)
    tm.tm_system_set_chain_slots(h, 3)
    yield tm, h, inp, sysd
    tm.tm_system_destroy(h)


def oracle_problem(inp, sysd, iq):
    """The oracle's Problem for q set iq of the multi-q inputs."""
    class _GS:
        pass
    gs = _GS()
    gs.sysd, gs.vrs, gs.rho = sysd, inp["vrs"], inp["rho"]
    qset = synth.QSetDef(q=inp["xq"][iq], kmesh=synth.kmesh_cart(sysd),
                         points=np.array([p for (p, _, _, _, _) in inp["points"]]),
                         roles=inp["roles"][iq], shifts=inp["shifts"][iq])
    return lv.Problem(gs, qset, point_states=[(m, e, et) for (_, m, e, et, _) in inp["points"]])


def test_qpath_batched_lanes_equal_single_chains_and_oracle(qpath):
    tm, h, inp, sysd = qpath
    nq = inp["xq"].shape[0]
    say(f"q path: {nq} chains x {len(DIRS)} lanes x {STEPS} steps, batched over 3 slots")
    chains = [tm.tm_chain_begin_multi(h, iq, DIRS, "pH", STEPS) for iq in range(nq)]
    try:
        tm.tm_chains_step(chains, STEPS)
        lanes = [tm.tm_chain_coeffs_lanes(c, STEPS) for c in chains]
    finally:
        for c in chains:
            tm.tm_chain_end(c)
    assert all(co["steps_done"] == STEPS and not co["breakdown"] for ls in lanes for co in ls)
    for iq, r in ((0, 0), (5, 2), (11, 1), (17, 0), (23, 2)):
        alone = tm.tm_lanczos_run(h, iq, DIRS[r], "pH", STEPS)
        for k in ("alpha", "beta", "gamma", "z", "zn"):
            assert np.array_equal(lanes[iq][r][k], alone[k]), (iq, DIRS[r], k)
    om = np.linspace(0.0, 1.0, 201)
    for iq, r in ((0, 0), (11, 1), (23, 2)):
        say(f"q path: oracle chain q {iq} direction {DIRS[r]}")
        prob = oracle_problem(inp, sysd, iq)
        measure = ("x", "y", "z", "n")
        ref = olanczos.run(prob, DIRS[r], "pH", STEPS, measure=measure)
        assert ref["steps_done"] == STEPS
        # the chain's conditioning, from the oracle alone: the same chain with
        # its start vector scaled by 1 + 2^-50 (identical in exact arithmetic)
        v0 = prob.v_vector
        prob.v_vector = lambda mu: v0(mu) * (1.0 + 2.0 ** -50)
        pert = olanczos.run(prob, DIRS[r], "pH", STEPS, measure=measure)
        drift = np.max([np.abs(pert[k] - ref[k]).reshape(-1, STEPS).max(axis=0) / np.abs(ref[k]).max()
                        for k in ("alpha", "beta", "gamma", "z")], axis=0)
        m = int(np.argmax(drift > 1e-12)) if (drift > 1e-12).any() else STEPS
        say(f"  coefficients fixed by the data to 1e-12 over the first {m} steps")
        assert m >= 6, m
        got = lanes[iq][r]
        for k in ("alpha", "beta", "gamma"):
            err = np.abs(got[k][:m] - ref[k][:m]).max() / np.abs(ref[k][:m]).max()
            say(f"  {k} rel err {err:.2e} (steps 0..{m - 1})")
            assert err <= 1e-10, (iq, k, err)
        zs = np.abs(ref["z"][:, :m]).max()
        assert np.abs(got["z"][:, :m] - ref["z"][:3, :m]).max() <= 1e-10 * zs
        assert np.abs(got["zn"][:m] - ref["z"][3, :m]).max() <= 1e-10 * zs
        # chi over all steps: a robust function of the chain even where single
        # coefficients are not; the bar is 100 times the oracle's own drift (at
        # least the coefficients' 1e-10)
        cref = ochi.chi_lanczos(ref, om, 0.02)
        cmax = np.abs(cref).max()
        own = np.abs(ochi.chi_lanczos(pert, om, 0.02) - cref).max() / cmax
        cgot = ochi.chi_lanczos(dict(got, z=np.vstack([got["z"], got["zn"][None]])), om, 0.02)
        err = np.abs(cgot - cref).max() / cmax
        say(f"  chi rel err {err:.2e} (oracle drift {own:.2e})")
        assert err <= max(100 * own, 1e-10), (iq, err, own)


def test_lane_group_chain_equals_single_chains(qpath):
    """One chain whose 72 lanes are the three directions of all 24 q sets
    (every kernel of a step runs once for all of them) gives, lane by lane,
    the coefficients of the single chain of that q set and direction."""
    tm, h, inp, sysd = qpath
    nq = inp["xq"].shape[0]
    iqs = [iq for iq in range(nq) for _ in DIRS]
    dirs = DIRS * nq
    say(f"lane group: one chain of {len(iqs)} lanes x {STEPS} steps")
    c = tm.tm_chain_begin_lanes(h, iqs, dirs, "pH", STEPS)
    try:
        assert tm.tm_chain_lanes(c) == len(iqs)
        tm.tm_chains_step([c], STEPS)
        lanes = tm.tm_chain_coeffs_lanes(c, STEPS)
    finally:
        tm.tm_chain_end(c)
    assert all(co["steps_done"] == STEPS and not co["breakdown"] for co in lanes)
    for g in (0, 4, 17, 35, 52, 71):
        alone = tm.tm_lanczos_run(h, iqs[g], dirs[g], "pH", STEPS)
        for k in ("alpha", "beta", "gamma", "z", "zn"):
            assert np.array_equal(lanes[g][k], alone[k]), (g, iqs[g], dirs[g], k)
        assert lanes[g]["n1"] == alone["n1"]


@pytest.mark.parametrize("flavour,m,cut", [("pH", 30, 13), ("nH", 12, 5)])
def test_lane_group_mixed_order_and_restart(qpath, flavour, m, cut):
    """Lanes in any order, the same q set in several lanes, the charge
    channel among them; a checkpoint taken part-way continues exactly."""
    tm, h, inp, sysd = qpath
    iqs = [5, 0, 5, 23, 11, 0]
    dirs = ["z", "+", "-", "z", "n", "x"]
    say(f"lane group {flavour}: lanes {list(zip(iqs, dirs))}, {m} steps, checkpoint after {cut}")
    c = tm.tm_chain_begin_lanes(h, iqs, dirs, flavour, m)
    try:
        tm.tm_chains_step([c], m)
        whole = tm.tm_chain_coeffs_lanes(c, m)
    finally:
        tm.tm_chain_end(c)
    for g in range(len(iqs)):
        alone = tm.tm_lanczos_run(h, iqs[g], dirs[g], flavour, m)
        for k in ("alpha", "beta", "gamma", "z", "zn"):
            assert np.array_equal(whole[g][k], alone[k]), (g, k)
    c = tm.tm_chain_begin_lanes(h, iqs, dirs, flavour, m)
    try:
        tm.tm_chains_step([c], cut)
        blob = tm.tm_chain_save(c)
    finally:
        tm.tm_chain_end(c)
    r = tm.tm_chain_restore(h, blob)
    try:
        assert tm.tm_chain_lanes(r) == len(iqs)
        tm.tm_chains_step([r], m - cut)
        resumed = tm.tm_chain_coeffs_lanes(r, m)
    finally:
        tm.tm_chain_end(r)
    for g in range(len(iqs)):
        for k in ("alpha", "beta", "gamma", "z", "zn"):
            assert np.array_equal(resumed[g][k], whole[g][k]), (g, k)


def test_lane_group_invalid_arguments(qpath):
    tm, h, inp, sysd = qpath
    nq = inp["xq"].shape[0]
    for iqs, dirs in (([], []), ([0] * 97, ["z"] * 97), ([0, nq], ["z", "z"]), ([-1], ["x"])):
        with pytest.raises(tm.TmError) as e:
            tm.tm_chain_begin_lanes(h, iqs, dirs, "pH", 4)
        assert e.value.code == tm.TM_EINVAL
