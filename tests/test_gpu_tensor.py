"""Several field directions in one pass: multi-right-hand-side applies and
multi-lane chains through the C ABI (needs an MI355X).

The batched kernels do, per right-hand side, the same arithmetic in the same
order as a single apply (the contractions choose their K split from the
single-right-hand-side batch count), so every comparison with the
single-direction path is exact.  Against the oracle the tolerances are those
of the parity tests.
"""
import numpy as np
import pytest

from oracle import lanczos as olanczos
from oracle import liouvillian as lv

from gpu_util import desc_from_problem, from_gpu, rel_err, say, to_gpu

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
def cubic(lib, cubic_gs, cubic_q):
    say("create cubic20 system")
    prob = lv.build_problem(cubic_gs, cubic_q)
    h = lib.tm_system_create(desc_from_problem(prob))
    yield prob, h
    lib.tm_system_destroy(h)


def same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
    assert a["steps_done"] == b["steps_done"] and a["n1"] == b["n1"]


def batched_vs_single(lib, prob, h, nrhs, prec, seed0):
    import torch
    info = lib.tm_qset_info_get(h, 0)
    xs = [to_gpu(prob.random_projected(seed0 + r), info["npw_pad"]) for r in range(nrhs)]
    xin = torch.cat(xs)
    out = torch.empty_like(xin)
    lib.tm_liouvillian_apply_multi(h, 0, nrhs, xin, out, prec)
    singles = []
    for x in xs:
        o = torch.empty_like(x)
        lib.tm_liouvillian_apply(h, 0, x, o, prec)
        singles.append(o)
    torch.cuda.synchronize()
    for r, o in enumerate(singles):
        assert torch.equal(out[r * o.numel():(r + 1) * o.numel()], o), r
    return xs, out


@pytest.mark.parametrize("resident", [True, False], ids=["resident", "columns"])
def test_apply_multi_equals_single_applies(lib, cubic, resident):
    prob, h = cubic
    lib.tm_system_set_resident_limit(h, -1 if resident else 0)
    try:
        for nrhs in (2, 4):
            say(f"apply_multi cubic20 nrhs {nrhs} resident={resident}")
            xs, out = batched_vs_single(lib, prob, h, nrhs, lib.TM_FP64, 20 + nrhs)
            # and one of them against the oracle
            info = lib.tm_qset_info_get(h, 0)
            n = xs[0].numel()
            got, _ = from_gpu(out[n:2 * n], (2, prob.nk, prob.nb, 2, info["npw_pad"]), prob.npw_pad)
            assert rel_err(got, prob.apply(prob.random_projected(20 + nrhs + 1))) <= 1e-12
        if resident:
            say("apply_multi cubic20 fp32 nrhs 3")
            batched_vs_single(lib, prob, h, 3, lib.TM_FP32, 40)
    finally:
        lib.tm_system_set_resident_limit(h, -1)


def test_apply_multi_generic_plane_path(lib):
    """10^3 grid: generic plane and z kernels with batched right-hand sides."""
    import synth
    from oracle import scf
    say("apply_multi tiny 10^3 (generic kernels)")
    gs = scf.scf(synth.make_tiny(fft=(10, 10, 10), seed=3), tol=1e-12, beta=0.5)
    prob = lv.build_problem(gs, np.array([0.05, 0.1, 0.0]) * 2 * np.pi / 6.0)
    h = lib.tm_system_create(desc_from_problem(prob))
    try:
        batched_vs_single(lib, prob, h, 3, lib.TM_FP64, 7)
    finally:
        lib.tm_system_destroy(h)


@pytest.mark.parametrize("flavour,dirs,m", [("pH", "xyz", 30), ("nH", "nxyz", 12), ("pH", "n+", 24)])
def test_tensor_run_equals_single_chains(lib, cubic, flavour, dirs, m):
    prob, h = cubic
    say(f"tensor run cubic20 {flavour} {dirs} {m}")
    lanes = lib.tm_tensor_run(h, 0, list(dirs), flavour, m)
    for d, got in zip(dirs, lanes):
        same(got, lib.tm_lanczos_run(h, 0, d, flavour, m))
        assert not got["breakdown"]
    # one lane against the oracle chain
    ref = olanczos.run(prob, dirs[-1], flavour, m, measure=("x", "y", "z", "n"))
    got = lanes[-1]
    assert np.abs(got["beta"] - ref["beta"]).max() <= 1e-10 * ref["beta"].max()
    assert np.abs(got["zn"] - ref["z"][3]).max() <= 1e-10 * np.abs(ref["z"]).max()


def test_fp32_lanes_equal_single_fp32_chains_and_restart(lib, cubic):
    """Single-precision bulk with lanes: each lane equals its FP32 single chain, and a
    saved FP32 chain restores as FP32."""
    prob, h = cubic
    say("fp32 tensor run and restart")
    lanes = lib.tm_tensor_run(h, 0, ["x", "z"], "nH", 9, lib.TM_FP32)
    for d, got in zip("xz", lanes):
        same(got, lib.tm_lanczos_run(h, 0, d, "nH", 9, lib.TM_FP32))
    c = lib.tm_chain_begin_multi(h, 0, ["x", "z"], "nH", 3, lib.TM_FP32)
    try:
        lib.tm_chains_step([c], 3)
        blob = lib.tm_chain_save(c)
    finally:
        lib.tm_chain_end(c)
    c2 = lib.tm_chain_restore(h, blob, capacity=9)
    try:
        lib.tm_chains_step([c2], 9)
        got = lib.tm_chain_coeffs_lanes(c2, 9)
    finally:
        lib.tm_chain_end(c2)
    for a, b in zip(got, lanes):
        same(a, b)


def test_multi_chain_in_pieces_graphs_and_restart(lib, cubic):
    """A two-lane chain stepped in pieces (graph replay and direct steps), saved,
    restored with a larger capacity and run on equals one tensor run."""
    prob, h = cubic
    say("multi-lane chain: pieces, graphs, restart")
    ref = lib.tm_tensor_run(h, 0, ["+", "z"], "pH", 36)
    c = lib.tm_chain_begin_multi(h, 0, ["+", "z"], "pH", 18)
    try:
        assert lib.tm_chain_lanes(c) == 2
        for k in (5, 1, 12):
            lib.tm_chains_step([c], k)
        blob = lib.tm_chain_save(c)
    finally:
        lib.tm_chain_end(c)
    c2 = lib.tm_chain_restore(h, blob, capacity=36)
    try:
        lib.tm_chains_step([c2], 36)
        got = lib.tm_chain_coeffs_lanes(c2, 36)
    finally:
        lib.tm_chain_end(c2)
    for a, b in zip(got, ref):
        same(a, b)


def test_workspace_growth_recaptures_graphs(lib, cubic_gs, cubic_q):
    """A single chain with a captured graph keeps running correctly after a wider
    chain of the same system grows the shared workspace."""
    prob = lv.build_problem(cubic_gs, cubic_q)
    h = lib.tm_system_create(desc_from_problem(prob))
    try:
        say("workspace growth with a captured graph")
        ref = lib.tm_lanczos_run(h, 0, "x", "nH", 18)
        c = lib.tm_chain_begin(h, 0, "x", "nH", 18)
        try:
            lib.tm_chains_step([c], 9)          # graph captured against the width-1 workspace
            w = lib.tm_chain_begin_multi(h, 0, ["y", "z", "n"], "nH", 6)   # grows it to 3
            try:
                lib.tm_chains_step([c, w], 9)
                lanes = lib.tm_chain_coeffs_lanes(w, 6)
            finally:
                lib.tm_chain_end(w)
            got = lib.tm_chain_coeffs(c, 18)
        finally:
            lib.tm_chain_end(c)
        same(got, ref)
        for d, lane in zip("yzn", lanes):
            same(lane, lib.tm_lanczos_run(h, 0, d, "nH", 6))
    finally:
        lib.tm_system_destroy(h)


def test_lane_breakdown_leaves_other_lanes_running(lib, tiny_gs_nosoc):
    """Goldstone mode: at q = 0 without SOC the x lane breaks down at step 1; the
    z lane in the same chain runs all its steps."""
    prob = lv.build_problem(tiny_gs_nosoc, np.zeros(3))
    h = lib.tm_system_create(desc_from_problem(prob))
    try:
        say("lane breakdown (Goldstone x lane next to a z lane)")
        lx, lz = lib.tm_tensor_run(h, 0, ["x", "z"], "nH", 8)
        assert lx["breakdown"] and lx["steps_done"] == 1
        assert lz["steps_done"] == 8
        same(lz, lib.tm_lanczos_run(h, 0, "z", "nH", 8))
    finally:
        lib.tm_system_destroy(h)


def test_tensor_invalid_arguments(lib, cubic):
    _, h = cubic
    with pytest.raises(lib.TmError):
        lib.tm_tensor_run(h, 0, list("xyzn+"), "pH", 4)    # more than 4 directions
    with pytest.raises(lib.TmError):
        lib.tm_tensor_run(h, 0, [], "pH", 4)
    with pytest.raises(ValueError):
        import torch
        x = torch.zeros(8, dtype=torch.complex128, device="cuda")
        lib.tm_liouvillian_apply_multi(h, 0, 2, x, x)
