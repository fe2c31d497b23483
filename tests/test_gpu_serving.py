"""Continuous-batching server (paper_2203_01120_amd.serving) on the GPU.

Each request's chi must be identical whether its chain runs alone or
interleaved with others on per-system streams under a memory budget, or as
one lane of a chain shared with other requests: the same per-request
arithmetic runs on the same data, so the comparison is exact.
"""
import numpy as np
import pytest

from oracle import liouvillian as lv

from gpu_util import desc_from_problem, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool(tiny_gs, tiny_q, cubic_gs, cubic_q):
    import torch
    import paper_2203_01120_amd as tm
    from paper_2203_01120_amd import serving as sv
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    slots = {}
    for name, gs, q in (("tiny", tiny_gs, tiny_q), ("cubic20", cubic_gs, cubic_q)):
        h = tm.tm_system_create(desc_from_problem(lv.build_problem(gs, q)))
        slots[name] = sv.SystemSlot(handle=h, nelem={0: tm.tm_qset_info_get(h, 0)["nelem"]})
    yield tm, sv, slots
    for s in slots.values():
        tm.tm_system_destroy(s.handle)


def requests(sv, omega, eta, stagger):
    spec = [("tiny", "z", "pH", 24), ("cubic20", "+", "pH", 30), ("cubic20", "z", "nH", 14),
            ("tiny", "-", "nH", 10), ("cubic20", "-", "pH", 18), ("tiny", "x", "nH", 7)]
    return [sv.Request(rid=i, system=s, iq=0, direction=d, flavour=f, nsteps=m, omega=omega, eta=eta,
                       arrival=stagger * i) for i, (s, d, f, m) in enumerate(spec)]


@pytest.mark.parametrize("stagger,lanes,slack,cap,cslots", [(0.0, 1, 1.0, 0, 1), (0.02, 1, 1.0, 0, 1),
                                                            (0.0, 4, 2.0, 0, 1), (0.0, 4, 4.0, 1, 1),
                                                            (0.0, 1, 1.0, 0, 3)])
def test_server_chi_identical_to_alone(pool, stagger, lanes, slack, cap, cslots):
    tm, sv, slots = pool
    omega = np.linspace(0.0, 0.07, 64)
    eta = 2e-4
    # a budget of about two cubic20 chains forces admissions to wait
    budget = 2 * sv.chain_bytes(slots["cubic20"].nelem[0], "nH", 30)
    say(f"server run, stagger {stagger}, lanes {lanes}, chains per system {cap}, slots {cslots}, budget {budget} B")
    server = sv.Server(slots, budget_bytes=budget, lanes=lanes, lane_slack=slack, max_chains=cap,
                       chain_slots=cslots)
    peak = [0]
    widest = [1]
    orig = server._admit

    def admit():
        orig()
        peak[0] = max(peak[0], server.used)
        for s in slots.values():
            assert not cap or len(s.active) <= cap
            for a in s.active:
                widest[0] = max(widest[0], len(a.reqs))
    server._admit = admit
    done = server.run(requests(sv, omega, eta, stagger))
    assert len(done) == 6 and server.used == 0
    assert peak[0] <= budget
    assert (widest[0] > 1) == (lanes > 1)    # the lane runs really shared chains
    for r in done:
        alone = tm.tm_lanczos_run(slots[r.system].handle, 0, r.direction, r.flavour, r.nsteps)
        assert r.coeffs["steps_done"] == alone["steps_done"]
        for key in ("alpha", "beta", "gamma", "z", "zn"):
            assert np.array_equal(r.coeffs[key], alone[key]), (r.rid, key)
        ref = tm.tm_chi(alone, max(1, alone["steps_done"]), omega, eta)
        assert np.array_equal(r.chi, ref)
        assert r.t_admit >= r.arrival - 1e-9 and r.t_done >= r.t_admit


def test_one_at_a_time_reference_matches(pool):
    tm, sv, slots = pool
    omega = np.linspace(0.0, 0.07, 32)
    eta = 2e-4
    say("one-at-a-time reference path")
    plain = sv.run_one_at_a_time(slots, requests(sv, omega, eta, 0.0))
    server = sv.Server(slots, budget_bytes=1 << 30)
    batched = {r.rid: r for r in server.run(requests(sv, omega, eta, 0.0))}
    for r in plain:
        assert np.array_equal(r.chi, batched[r.rid].chi), r.rid
    s = sv.summary(plain)
    assert s["requests"] == 6 and s["p99_s"] >= s["p50_s"] >= 0
