"""The benchmark system at full size: 48 x 48 x 180 grid, 104 bands, in the
launch configuration the benchmark times (resident real-space ground state,
wave plane kernels, the 180-point z passes, LDS-staged contractions with
7 x 7 output tiles of 16, the line-FFT potential on 414 720 points).

Element-wise against the oracle, on the same system restricted to one mesh
point (k index 7 of the 6 x 6 x 1 mesh; every per-k kernel then runs at its
real shape, and one oracle apply is about 10 s of host time):

* L applied to two projected random vectors, 1e-12 relative;
* a 3-step pseudo-Hermitian m_+ chain and a 2-step non-Hermitian m_- chain:
  alpha, beta, gamma, z and zn to 1e-10 relative.

With one mesh point the contractions pick their K split from 2 batches
instead of 72; that split and the number of batches are the only launch
differences from the 36-point benchmark run.

On the full 36-point system, where an oracle apply would take minutes, the
checks are properties that hold at any size:

* JL is Hermitian: (a, J L b) = conj((b, J L a)) for projected a, b; FP64
  sums over 1.9e8 elements, so 1e-11 relative.
* Linearity: L(a + 2 b) = L a + 2 L b to 1e-12 relative.
* The chain start: the library's alpha_0 = (Lv, J Lv) / (v, J Lv) for the
  start vector v equals the same ratio formed with torch (1e-10).
* Several right-hand sides in one pass equal single applies bit for bit, and
  lanes of a chain equal single chains bit for bit.
* FP32 bulk stays within 2e-5 of the FP64 apply (the bound of the FP32 tests).
"""
import os
import sys

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TIMEOUT = 900      # seconds: about ten oracle applies at full grid size


@pytest.fixture(scope="module")
def slab1k():
    """The benchmark system on mesh point 7 alone: library handle and oracle Problem."""
    import torch
    import paper_2203_01120_amd as tm
    import synth
    from oracle import liouvillian as lv
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    sys.path.insert(0, ROOT)
    import bench
    say("one-point slab: building inputs")
    sysd = synth.make_hexslab()
    inp = synth.synthetic_inputs(sysd, synth.cart_from_frac(sysd, [1.0 / 6.0, 0.0, 0.0]), seed=1,
                                 kmesh_subset=[7])

    class _GS:      # the oracle Problem reads only these ground-state fields
        pass
    gs = _GS()
    gs.sysd, gs.vrs, gs.rho = inp["sysd"], inp["vrs"], inp["rho"]
    prob = lv.Problem(gs, inp["qset"], point_states=[(m, e, et) for (_, m, e, et, _) in inp["points"]])
    say("one-point slab: creating the system")
    h = tm.tm_system_create(bench.make_desc(inp))
    info = tm.tm_qset_info_get(h, 0)
    assert info["nk"] == 1 and info["nbnd"] == 104
    yield tm, h, info, prob
    tm.tm_system_destroy(h)


@pytest.mark.timeout(ORACLE_TIMEOUT)
def test_fullsize_apply_matches_oracle(slab1k):
    import torch
    from gpu_util import from_gpu, rel_err, to_gpu
    tm, h, info, prob = slab1k
    shape = (2, 1, prob.nb, 2, info["npw_pad"])
    for seed in (1, 2):
        say(f"one-point slab: apply seed {seed} (GPU)")
        x = prob.random_projected(seed)
        xin = to_gpu(x, info["npw_pad"])
        out = torch.empty_like(xin)
        tm.tm_liouvillian_apply(h, 0, xin, out)
        torch.cuda.synchronize()
        got, raw = from_gpu(out, shape, prob.npw_pad)
        say(f"one-point slab: apply seed {seed} (oracle)")
        ref = prob.apply(x)
        err = rel_err(got, ref)
        say(f"one-point slab: apply seed {seed} rel err {err:.2e}")
        assert err <= 1e-12, err
        assert np.all(raw[:, 0, :, :, prob.k[0].npw:] == 0)
    n1, n2, n3 = prob.sysd.fft
    # the resident real-space ground state ran: one slot per side, all bands and planes
    assert tm.tm_system_resident_bytes(h) == 2 * prob.nb * n3 * 2 * n1 * n2 * 16


@pytest.mark.timeout(ORACLE_TIMEOUT)
def test_fullsize_every_tuned_variant_matches_oracle(slab1k):
    """Each autotuner candidate of this shape (plane kernels of 48 x 48, z
    passes of 180, the 104-band contractions), forced in turn, against one
    oracle apply at 1e-12."""
    import torch
    from gpu_util import from_gpu, rel_err, to_gpu
    tm, h, info, prob = slab1k
    x = prob.random_projected(3)
    xin = to_gpu(x, info["npw_pad"])
    out = torch.empty_like(xin)
    tm.tm_liouvillian_apply(h, 0, xin, out)
    torch.cuda.synchronize()
    say("one-point slab: oracle apply for the variants")
    ref = prob.apply(x)
    entries = [e for e in tm.tm_autotune_report() if "grid 48x48x180, 104 bands, 1 k" in e["shape"]]
    say("tuned: " + "; ".join(f"{e['op']} {e['chosen']}/{e['variants']} {e['us']}" for e in entries))
    assert {e["op"] for e in entries} >= {"plane_density", "plane_apply", "zpass_inverse", "zpass_forward",
                                          "contraction"}
    for e in entries:
        try:
            for v in range(e["variants"]):
                tm.tm_autotune_force(e["op"], v)
                tm.tm_liouvillian_apply(h, 0, xin, out)
                torch.cuda.synchronize()
                got, _ = from_gpu(out, (2, 1, prob.nb, 2, info["npw_pad"]), prob.npw_pad)
                err = rel_err(got, ref)
                say(f"  {e['op']} variant {v}: rel err {err:.2e}")
                assert err <= 1e-12, (e["op"], v, err)
        finally:
            tm.tm_autotune_force(e["op"], -1)


@pytest.mark.timeout(ORACLE_TIMEOUT)
@pytest.mark.parametrize("flavour,mu,m", [("pH", "+", 3), ("nH", "-", 2)], ids=["pH+3", "nH-2"])
def test_fullsize_chain_matches_oracle(slab1k, flavour, mu, m):
    from oracle import lanczos as olanczos
    tm, h, info, prob = slab1k
    say(f"one-point slab: {flavour} {mu} {m} steps (GPU)")
    co = tm.tm_lanczos_run(h, 0, mu, flavour, m)
    say(f"one-point slab: {flavour} {mu} {m} steps (oracle)")
    oc = olanczos.run(prob, mu, flavour, m, measure=("x", "y", "z", "n"))
    assert co["steps_done"] == oc["steps_done"] == m
    assert abs(co["n1"] - oc["n1"]) <= 1e-10 * oc["n1"]
    for k in ("alpha", "beta", "gamma"):
        err = np.abs(co[k] - oc[k]).max() / np.abs(oc[k]).max()
        say(f"  {k} rel err {err:.2e}")
        assert err <= 1e-10, (k, err)
    zref = oc["z"]
    zs = np.abs(zref).max()
    assert np.abs(co["z"] - zref[:3]).max() <= 1e-10 * zs
    assert np.abs(co["zn"] - zref[3]).max() <= 1e-10 * zs


@pytest.fixture(scope="module")
def slab():
    import torch
    import paper_2203_01120_amd as tm
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    sys.path.insert(0, ROOT)
    import bench
    say("full-size slab: building inputs")
    inp = bench.build_inputs("hexslab", 1)
    say("full-size slab: creating the system")
    h = tm.tm_system_create(bench.make_desc(inp))
    info = tm.tm_qset_info_get(h, 0)
    yield tm, h, info
    tm.tm_system_destroy(h)


def jdot(a, b, half):
    """(a, J b) with J = diag(1, -1) over the two sides (weights cancel in ratios)."""
    import torch
    return (torch.vdot(a[:half], b[:half]) - torch.vdot(a[half:], b[half:])).item()


def test_fullsize_apply_properties(slab):
    import torch
    tm, h, info = slab
    n = info["nelem"]
    half = n // 2
    g = torch.Generator(device="cuda").manual_seed(11)
    say("full-size slab: projected random vectors")
    raw = torch.randn(2 * n, dtype=torch.complex128, device="cuda", generator=g)
    ab = torch.empty_like(raw)
    tm.tm_liouvillian_apply_multi(h, 0, 2, raw, ab)        # outputs of L are projected
    ab /= ab.abs().max()
    a, b = ab[:n], ab[n:]
    say("full-size slab: L a, L b (batched and single)")
    lab = torch.empty_like(ab)
    tm.tm_liouvillian_apply_multi(h, 0, 2, ab, lab)
    la = torch.empty_like(a)
    lb = torch.empty_like(b)
    tm.tm_liouvillian_apply(h, 0, a, la)
    tm.tm_liouvillian_apply(h, 0, b, lb)
    torch.cuda.synchronize()
    assert torch.equal(lab[:n], la) and torch.equal(lab[n:], lb)
    say("full-size slab: JL Hermitian")
    x, y = jdot(a, lb, half), np.conj(jdot(b, la, half))
    assert abs(x - y) <= 1e-11 * max(abs(x), abs(y)), (x, y)
    say("full-size slab: linearity")
    c = a + 2.0 * b
    lc = torch.empty_like(c)
    tm.tm_liouvillian_apply(h, 0, c, lc)
    torch.cuda.synchronize()
    ref = la + 2.0 * lb
    assert ((lc - ref).abs().max() / ref.abs().max()).item() <= 1e-12
    say("full-size slab: FP32 bulk")
    l32 = torch.empty_like(a)
    tm.tm_liouvillian_apply(h, 0, a, l32, tm.TM_FP32)
    torch.cuda.synchronize()
    assert ((l32 - la).abs().max() / la.abs().max()).item() <= 2e-5


def test_fullsize_chain_start_matches_torch(slab):
    import torch
    tm, h, info = slab
    n = info["nelem"]
    say("full-size slab: chain start")
    v = torch.empty(n, dtype=torch.complex128, device="cuda")
    tm.tm_start_vectors(h, 0, "+", None, v)           # v = P sigma^+ U
    lv = torch.empty_like(v)
    tm.tm_liouvillian_apply(h, 0, v, lv)
    co = tm.tm_lanczos_run(h, 0, "+", "pH", 1)
    torch.cuda.synchronize()
    a0 = jdot(lv, lv, half=n // 2) / jdot(v, lv, half=n // 2)
    assert abs(co["alpha"][0] - a0) <= 1e-10 * abs(a0)


def test_fullsize_lanes_equal_single_chains(slab):
    tm, h, info = slab
    say("full-size slab: two-lane chain vs single chains (2 steps)")
    lanes = tm.tm_tensor_run(h, 0, ["+", "z"], "pH", 2)
    for d, got in zip("+z", lanes):
        ref = tm.tm_lanczos_run(h, 0, d, "pH", 2)
        for k in ("alpha", "beta", "gamma", "z", "zn"):
            assert np.array_equal(got[k], ref[k]), (d, k)
