"""Continuous-batching server (paper_2203_01120_amd.serving) on the GPU.

Each request's chi must be identical whether its chain runs alone or
interleaved with others on per-system streams under a memory budget, or as
one lane of a chain shared with other requests, or on a system the server
created on demand (after evicting another): the same per-request arithmetic
runs on the same data, so the comparison is exact.  The budget counts the
systems' footprints (tables, ground state, workspaces) and the chains; a
request that breaks down before its first step finishes with an error
instead of failing the server.
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
    # the systems' footprints plus about two cubic20 chains: admissions must wait
    base = sum(sv.SystemPool({k: v}, 1 << 62, lanes=lanes, chain_slots=cslots).used for k, v in slots.items())
    budget = base + 2 * sv.chain_bytes(slots["cubic20"].nelem[0], "nH", 30)
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
    assert len(done) == 6 and server.used == base
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
    server = sv.Server(slots, budget_bytes=1 << 36)
    batched = {r.rid: r for r in server.run(requests(sv, omega, eta, 0.0))}
    for r in plain:
        assert np.array_equal(r.chi, batched[r.rid].chi), r.rid
    s = sv.summary(plain)
    assert s["requests"] == 6 and s["p99_s"] >= s["p50_s"] >= 0


def test_footprint_from_descriptor_matches_the_system(tiny_gs, tiny_q, cubic_gs, cubic_q):
    """tm_system_footprint (descriptor only) against tm_system_memory of the created
    system after a chain: the same resident, column and workspace sizes, and a
    table estimate at or above the real tables."""
    import paper_2203_01120_amd as tm
    tm.load()
    for gs, q in ((tiny_gs, tiny_q), (cubic_gs, cubic_q)):
        d = desc_from_problem(lv.build_problem(gs, q))
        est = tm.tm_system_footprint(d)
        h = tm.tm_system_create(d)
        try:
            tm.tm_lanczos_run(h, 0, "z", "pH", 4)
            got = tm.tm_system_memory(h)
        finally:
            tm.tm_system_destroy(h)
        say(f"footprint estimate {est} vs {got}")
        for k in ("resident_full", "columns_full", "workspace_per_rhs"):
            assert est[k] == got[k], k
        assert got["resident"] == got["resident_full"] > 0
        assert got["tables"] <= est["tables"] <= 1.5 * got["tables"] + (16 << 20)
        assert got["workspace"] >= got["workspace_per_rhs"]


def test_goldstone_request_finishes_with_an_error(tiny_gs_nosoc):
    """pH along x at q = 0 without SOC: the start vector is a zero mode of JL, the
    chain breaks down before its first step; the request finishes (chi = 0,
    breakdown, error set), the server's memory returns and the other request runs."""
    import paper_2203_01120_amd as tm
    from paper_2203_01120_amd import serving as sv
    tm.load()
    h = tm.tm_system_create(desc_from_problem(lv.build_problem(tiny_gs_nosoc, np.zeros(3))))
    try:
        slots = {"gold": sv.SystemSlot(handle=h, nelem={0: tm.tm_qset_info_get(h, 0)["nelem"]})}
        server = sv.Server(slots, budget_bytes=1 << 34)
        base = server.used
        omega = np.linspace(0.0, 0.05, 16)
        reqs = [sv.Request(rid=0, system="gold", iq=0, direction="x", flavour="pH", nsteps=12, omega=omega,
                           eta=1e-3),
                sv.Request(rid=1, system="gold", iq=0, direction="z", flavour="pH", nsteps=12, omega=omega,
                           eta=1e-3)]
        done = {r.rid: r for r in server.run(reqs)}
        assert server.used == base
        g = done[0]
        assert g.coeffs["steps_done"] == 0 and g.coeffs["breakdown"] and g.error
        assert np.all(g.chi == 0)
        assert done[1].error is None and done[1].coeffs["steps_done"] == 12
        plain = sv.run_one_at_a_time(slots, [sv.Request(rid=0, system="gold", iq=0, direction="x", flavour="pH",
                                                        nsteps=12, omega=omega, eta=1e-3)])
        assert plain[0].error and plain[0].coeffs["steps_done"] == 0
    finally:
        tm.tm_system_destroy(h)


def test_systems_created_and_evicted_on_demand(cubic_gs, cubic_q):
    """Spec systems (the 20^3 system at two q) under a budget that holds one of
    them (plus its chains) at a time: the server creates, evicts and
    re-creates them, and every chi equals the request run alone on a system
    of its own."""
    import paper_2203_01120_amd as tm
    from paper_2203_01120_amd import serving as sv
    tm.load()
    q2 = np.array([0.0, 0.1, 0.05]) * 2 * np.pi / 10.0
    descs = {"a": desc_from_problem(lv.build_problem(cubic_gs, cubic_q)),
             "b": desc_from_problem(lv.build_problem(cubic_gs, q2))}
    specs = {k: sv.SystemSpec(make_desc=(lambda d=d: d)) for k, d in descs.items()}
    probe = sv.SystemPool({}, 1 << 62, specs, lanes=1)
    foot = {k: probe.footprint(k) for k in specs}
    budget = max(foot.values()) + 2 * sv.chain_bytes(_nelem(tm, descs["a"]), "nH", 40)
    real = 0
    for d in descs.values():      # the systems' real footprints: two never fit together
        h = tm.tm_system_create(d)
        try:
            real += sv.SystemPool({"x": sv.SystemSlot(handle=h, nelem={})}, 1 << 62, lanes=1).used
        finally:
            tm.tm_system_destroy(h)
    assert budget < real
    omega = np.linspace(0.0, 0.07, 24)
    eta = 2e-4
    spec = [("a", "z", "pH", 24), ("b", "+", "pH", 30), ("a", "-", "nH", 10), ("b", "z", "nH", 14),
            ("a", "x", "pH", 18)]
    reqs = [sv.Request(rid=i, system=s, iq=0, direction=d, flavour=f, nsteps=m, omega=omega, eta=eta,
                       arrival=0.0) for i, (s, d, f, m) in enumerate(spec)]
    server = sv.Server({}, budget_bytes=budget, specs=specs, lanes=1)
    peak = [0]
    orig = server._admit

    def admit():
        orig()
        peak[0] = max(peak[0], server.used)
    server._admit = admit
    try:
        done = server.run(reqs)
    finally:
        server.close()
    say(f"created {server.pool.created}, evicted {server.pool.evicted}, peak {peak[0]} of {budget}")
    assert len(done) == 5 and server.used == 0 and peak[0] <= budget
    assert all(r.error is None for r in done)
    assert server.pool.created >= 5 and server.pool.evicted >= 5
    for r in done:
        h = tm.tm_system_create(descs[r.system])
        try:
            # the server's resident choice for this system (it fits: the full copy)
            alone = tm.tm_lanczos_run(h, 0, r.direction, r.flavour, r.nsteps)
        finally:
            tm.tm_system_destroy(h)
        for key in ("alpha", "beta", "gamma", "z", "zn"):
            assert np.array_equal(r.coeffs[key], alone[key]), (r.rid, key)


def _nelem(tm, d):
    from paper_2203_01120_amd.serving import _nelem_of_desc
    return _nelem_of_desc(d, 0)
