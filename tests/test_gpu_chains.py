"""Chain-level interface (tm_chain_*) through the C ABI (needs an MI355X).

A chain stepped in pieces, or interleaved with other chains (on one stream,
or on the concurrent streams of the workspace slots), runs the same kernels
on the same data as tm_lanczos_run, so its coefficients agree bit for bit; against the oracle the tolerance is the one
of the Lanczos parity tests (1e-10 relative).
"""
import numpy as np
import pytest

from oracle import lanczos as olanczos
from oracle import liouvillian as lv

from gpu_util import desc_from_problem, desc_from_problems, from_gpu, rel_err, say, to_gpu

pytestmark = pytest.mark.gpu

KEYS = ("alpha", "beta", "gamma", "z", "zn")


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2203_01120_amd as tm
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    return tm


@pytest.fixture(scope="module")
def systems(lib, tiny_gs, tiny_q, cubic_gs, cubic_q):
    say("create tiny and cubic20 systems")
    out = {}
    for name, gs, q in (("tiny", tiny_gs, tiny_q), ("cubic20", cubic_gs, cubic_q)):
        prob = lv.build_problem(gs, q)
        out[name] = (prob, lib.tm_system_create(desc_from_problem(prob)))
    yield out
    for _, h in out.values():
        lib.tm_system_destroy(h)


def same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
    assert a["steps_done"] == b["steps_done"] and a["n1"] == b["n1"]


def test_chain_in_pieces_equals_lanczos_run(lib, systems):
    prob, h = systems["cubic20"]
    for flavour, mu, pieces in (("pH", "+", (7, 13, 40)), ("nH", "z", (1, 5, 14))):
        say(f"chain in pieces cubic20 {flavour} {mu} {pieces}")
        m = sum(pieces)
        ref = lib.tm_lanczos_run(h, 0, mu, flavour, m)
        c = lib.tm_chain_begin(h, 0, mu, flavour, m)
        try:
            for k in pieces:
                lib.tm_chains_step([c], k)
            got = lib.tm_chain_coeffs(c, m)
        finally:
            lib.tm_chain_end(c)
        same(got, ref)
        oref = olanczos.run(prob, mu, flavour, m)
        assert np.abs(got["beta"] - oref["beta"]).max() <= 1e-10 * oref["beta"].max()


def test_interleaved_chains_match_alone(lib, systems):
    """Chains of two systems and two chains of one system, stepped in turn."""
    pt, ht = systems["tiny"]
    pc, hc = systems["cubic20"]
    specs = [(ht, "z", "pH", 20), (hc, "+", "pH", 30), (hc, "-", "nH", 12), (ht, "x", "nH", 9)]
    alone = [lib.tm_lanczos_run(h, 0, mu, f, m) for h, mu, f, m in specs]
    say("interleaved chains")
    chains = [lib.tm_chain_begin(h, 0, mu, f, m) for h, mu, f, m in specs]
    try:
        lib.tm_chains_step(chains, 4)
        lib.tm_chains_step(chains[1:], 3)
        lib.tm_chains_step(chains, 100)   # capped at each chain's capacity
        got = [lib.tm_chain_coeffs(c, m) for c, (_, _, _, m) in zip(chains, specs)]
    finally:
        for c in chains:
            lib.tm_chain_end(c)
    for g, a, (_, _, _, m) in zip(got, alone, specs):
        assert g["steps_done"] == m
        same(g, a)


def test_chain_slots_overlap_and_match(lib, systems):
    """Chains of one small system spread over the workspace slots run on
    concurrent streams inside tm_chains_step; each equals its chain run alone,
    with the default slots and with one slot, and an apply issued between the
    steps (on the caller's stream, in whichever slot is current) is unchanged."""
    import torch
    prob, h = systems["cubic20"]
    specs = [("x", "pH", 18), ("y", "nH", 9), ("z", "pH", 24), ("+", "pH", 12), ("-", "nH", 6), ("n", "pH", 30)]
    alone = [lib.tm_lanczos_run(h, 0, mu, f, m) for mu, f, m in specs]
    info = lib.tm_qset_info_get(h, 0)
    x = to_gpu(prob.random_projected(5), info["npw_pad"])
    y0 = torch.empty_like(x)
    lib.tm_liouvillian_apply(h, 0, x, y0)
    for nslots in (3, 1, 6):
        say(f"chains over {nslots} workspace slots")
        lib.tm_system_set_chain_slots(h, nslots)
        chains = [lib.tm_chain_begin(h, 0, mu, f, m) for mu, f, m in specs]
        try:
            with pytest.raises(lib.TmError):
                lib.tm_system_set_chain_slots(h, 2)       # chains exist
            lib.tm_chains_step(chains, 5)
            y = torch.empty_like(x)
            lib.tm_liouvillian_apply(h, 0, x, y)
            lib.tm_chains_step(chains[::2], 7)
            lib.tm_chains_step(chains, 100)
            got = [lib.tm_chain_coeffs(c, m) for c, (_, _, m) in zip(chains, specs)]
            torch.cuda.synchronize()
        finally:
            for c in chains:
                lib.tm_chain_end(c)
        assert torch.equal(y, y0)
        for g, a, (_, _, m) in zip(got, alone, specs):
            assert g["steps_done"] == m
            same(g, a)
    for bad in (0, 17):
        with pytest.raises(lib.TmError):
            lib.tm_system_set_chain_slots(h, bad)


def test_graph_replay_matches_direct_issue(lib, systems):
    """Captured periods replayed many times, with eager work of the same system
    (a direct apply) and host synchronisations between the replays."""
    import torch
    prob, h = systems["cubic20"]
    info = lib.tm_qset_info_get(h, 0)
    for flavour, mu, m in (("pH", "+", 60), ("nH", "z", 21)):
        say(f"graph vs direct cubic20 {flavour} {mu} {m}")
        lib.tm_chains_use_graphs(False)
        try:
            direct = lib.tm_lanczos_run(h, 0, mu, flavour, m)
        finally:
            lib.tm_chains_use_graphs(True)
        x = torch.zeros(info["nelem"], dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        lib.tm_start_vectors(h, 0, "x", None, x)
        c = lib.tm_chain_begin(h, 0, mu, flavour, m)
        try:
            done = 0
            while done < m:
                k = min(12, m - done)
                lib.tm_chains_step([c], k)
                lib.tm_liouvillian_apply(h, 0, x, y)
                torch.cuda.synchronize()
                part = lib.tm_chain_coeffs(c, m)
                done += k
                assert part["steps_done"] == done
                # every replay so far agrees with the directly issued chain
                for key in ("beta", "alpha"):
                    assert np.array_equal(part[key][:done], direct[key][:done]), key
            got = lib.tm_chain_coeffs(c, m)
        finally:
            lib.tm_chain_end(c)
        same(got, direct)


def test_several_q_sets_in_one_system(lib, tiny_gs):
    """Chains on different q sets of one system, stepped together (workspace
    sized for all sets, graphs of one set unaffected by the others)."""
    qs = [np.array(v) * 2 * np.pi / 6.0 for v in ((0.1, 0.05, 0.0), (0.0, 0.2, 0.1), (0.25, 0.0, 0.0))]
    probs = [lv.build_problem(tiny_gs, q) for q in qs]
    h = lib.tm_system_create(desc_from_problems(probs))
    try:
        # (the tiny system's JL is indefinite at q != 0: pseudo-Hermitian chains along m_z only)
        specs = [(0, "z", "pH", 20), (1, "z", "pH", 18), (2, "-", "nH", 9), (1, "x", "nH", 6)]
        say("chains on three q sets")
        chains = [lib.tm_chain_begin(h, iq, mu, f, m) for iq, mu, f, m in specs]
        try:
            lib.tm_chains_step(chains, 25)
            got = [lib.tm_chain_coeffs(c, m) for c, (_, _, _, m) in zip(chains, specs)]
        finally:
            for c in chains:
                lib.tm_chain_end(c)
        for g, (iq, mu, f, m) in zip(got, specs):
            ref = olanczos.run(probs[iq], mu, f, m)
            assert g["steps_done"] == ref["steps_done"] == m
            assert np.abs(g["beta"] - ref["beta"]).max() <= 1e-10 * ref["beta"].max()
            assert np.abs(g["alpha"] - ref["alpha"]).max() <= 1e-10 * np.abs(ref["alpha"]).max()
        # a direct apply on the middle set
        import torch
        prob = probs[1]
        info = lib.tm_qset_info_get(h, 1)
        x = prob.random_projected(5)
        xin = to_gpu(x, info["npw_pad"])
        out = torch.empty_like(xin)
        lib.tm_liouvillian_apply(h, 1, xin, out)
        torch.cuda.synchronize()
        gotx, _ = from_gpu(out, (2, prob.nk, prob.nb, 2, info["npw_pad"]), prob.npw_pad)
        assert rel_err(gotx, prob.apply(x)) <= 1e-12
    finally:
        lib.tm_system_destroy(h)


@pytest.mark.parametrize("flavour,mu,k,m", [("pH", "+", 30, 60), ("nH", "z", 7, 20)])
def test_checkpoint_restart_continues_exactly(lib, systems, flavour, mu, k, m):
    """Stop at step k, save, end; restore with a larger capacity and run on:
    the coefficients equal an uninterrupted chain bit for bit."""
    prob, h = systems["cubic20"]
    say(f"checkpoint {flavour} {mu}: {k} + {m - k} steps")
    ref = lib.tm_lanczos_run(h, 0, mu, flavour, m)
    c = lib.tm_chain_begin(h, 0, mu, flavour, k)
    try:
        lib.tm_chains_step([c], k)
        blob = lib.tm_chain_save(c)
        first = lib.tm_chain_coeffs(c, k)
    finally:
        lib.tm_chain_end(c)
    c2 = lib.tm_chain_restore(h, blob, capacity=m)
    try:
        mid = lib.tm_chain_coeffs(c2, m)
        assert mid["steps_done"] == k
        for key in KEYS:
            assert np.array_equal(mid[key][..., :k], first[key][..., :k]), key
        lib.tm_chains_step([c2], m)
        got = lib.tm_chain_coeffs(c2, m)
    finally:
        lib.tm_chain_end(c2)
    same(got, ref)
    with pytest.raises(lib.TmError):
        lib.tm_chain_restore(h, blob[:100])


def test_chain_breakdown(lib, tiny_gs_nosoc):
    prob = lv.build_problem(tiny_gs_nosoc, np.zeros(3))
    h = lib.tm_system_create(desc_from_problem(prob))
    try:
        say("chain breakdown (Goldstone mode)")
        c = lib.tm_chain_begin(h, 0, "x", "nH", 6)
        try:
            lib.tm_chains_step([c], 6)
            r = lib.tm_chain_coeffs(c, 6)
        finally:
            lib.tm_chain_end(c)
        assert r["breakdown"] and r["steps_done"] == 1
    finally:
        lib.tm_system_destroy(h)


def test_chain_invalid_arguments(lib, systems):
    _, h = systems["tiny"]
    with pytest.raises(lib.TmError):
        lib.tm_chain_begin(h, 0, "x", "pH", 0)
    with pytest.raises(lib.TmError):
        lib.tm_chain_begin(h, 3, "x", "pH", 5)
    with pytest.raises(lib.TmError):
        lib.tm_chain_begin(h, 0, "x", "pH", 5, prec=7)   # no such precision


def test_degenerate_sizes(lib, systems):
    """One-step chains, capacity 1 stepped past it, chi from one coefficient,
    an empty frequency grid, a one-direction tensor run."""
    prob, h = systems["cubic20"]
    say("degenerate sizes")
    for flavour in ("pH", "nH"):
        one = lib.tm_lanczos_run(h, 0, "z", flavour, 1)
        assert one["steps_done"] == 1
        ref = olanczos.run(prob, "z", flavour, 1)
        lam = lib.tm_qset_info_get(h, 0)["lam"]      # the operator's scale (alpha_0 may be tiny)
        assert abs(one["alpha"][0] - ref["alpha"][0]) <= 1e-12 * lam
        c = lib.tm_chain_begin(h, 0, "z", flavour, 1)
        try:
            lib.tm_chains_step([c], 5)               # never past the capacity
            got = lib.tm_chain_coeffs(c, 1)
        finally:
            lib.tm_chain_end(c)
        same(got, one)
        w = np.linspace(0.0, 0.1, 7)
        chi1 = lib.tm_chi(one, 1, w, 1e-3)
        # one coefficient: chi = n1 z_0 / (w + i eta - alpha_0)
        expect = one["n1"] * one["z"][:, :1] / (w[None, :] + 1e-3j - one["alpha"][0])
        assert np.abs(chi1 - expect).max() <= 1e-12 * np.abs(expect).max()
        assert lib.tm_chi(one, 1, np.zeros(0), 1e-3).shape == (3, 0)
        same(lib.tm_tensor_run(h, 0, ["z"], flavour, 1)[0], one)
