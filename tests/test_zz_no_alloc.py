"""The allocation-free apply (tm_liouvillian_apply_noalloc) through the C ABI.

Same kernels as tm_liouvillian_apply, with the workspace in the library's
static per-device scratch instead of allocated buffers, so its output is
compared with the ordinary entry point's on the same inputs at the parity
bar of the apply (1e-12 relative; the arithmetic is the same, so equality is
expected): two calls in a row, the first on the 20^3 / 8-band system, the
second on the smaller 8^3 / 3-band one (the scratch keeps the first call's
contents), and then the first system again.  A system whose workspace
exceeds the scratch, and a q set whose ground-state caches are not built
yet, are refused with an error.
"""
import numpy as np
import pytest

import synth
from oracle import liouvillian as lv

from gpu_util import desc_from_problem, rel_err, say

pytestmark = pytest.mark.gpu


def _both(tm, h, prob, seed):
    import torch
    info = tm.tm_qset_info_get(h, 0)
    x = prob.random_projected(seed)
    out = np.zeros(x.shape[:-1] + (info["npw_pad"],), complex)
    out[..., :x.shape[-1]] = x
    xin = torch.from_numpy(out.ravel()).to("cuda")
    ref = torch.empty_like(xin)
    got = torch.full_like(xin, float("nan"))
    tm.tm_liouvillian_apply(h, 0, xin, ref)
    torch.cuda.synchronize()
    tm.tm_liouvillian_apply_noalloc(h, 0, xin, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_apply_matches_the_allocating_apply(tiny_gs, tiny_q, cubic_gs, cubic_q):
    import torch
    import paper_2203_01120_amd as tm
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    big = lv.build_problem(cubic_gs, cubic_q)
    small = lv.build_problem(tiny_gs, tiny_q)
    hb = tm.tm_system_create(desc_from_problem(big))
    hs = tm.tm_system_create(desc_from_problem(small))
    try:
        # ground-state caches not built yet: refused, nothing written
        n = tm.tm_qset_info_get(hs, 0)["nelem"]
        x = torch.zeros(n, dtype=torch.complex128, device="cuda")
        y = torch.zeros_like(x)
        with pytest.raises(tm.TmError) as e:
            tm.tm_liouvillian_apply_noalloc(hs, 0, x, y)
        assert e.value.code == tm.TM_EINVAL
        for name, h, prob, seed in (("cubic20", hb, big, 1), ("tiny", hs, small, 2), ("cubic20", hb, big, 3)):
            say(f"noalloc apply {name} seed {seed}")
            got, ref = _both(tm, h, prob, seed)
            err = rel_err(got, ref)
            say(f"  rel diff to the allocating apply {err:.2e}")
            assert np.all(np.isfinite(got)) and err <= 1e-12, err
            # and the oracle, at the same bar
            shape = (2, prob.nk, prob.nb, 2, tm.tm_qset_info_get(h, 0)["npw_pad"])
            g = got.reshape(shape)[..., :prob.npw_pad]
            assert rel_err(g, prob.apply(prob.random_projected(seed))) <= 1e-12
    finally:
        tm.tm_system_destroy(hb)
        tm.tm_system_destroy(hs)


def test_noalloc_apply_refuses_a_workspace_beyond_the_scratch():
    import torch
    import paper_2203_01120_amd as tm
    tm.load()
    sysd = synth.make_cubic(32, 32, 3)
    inp = synth.synthetic_inputs_multi(sysd, np.array([[0.1, 0.0, 0.0]]) * 2 * np.pi / 10.0, seed=1)
    pts = [tm.Point(xk=p, mill=m, evc=e, et=et, vkb=v) for (p, m, e, et, v) in inp["points"]]
    d = tm.SystemDesc(cell=sysd.cell, fft=sysd.fft, nbnd=sysd.nbnd, points=pts, vrs=inp["vrs"], rho=inp["rho"],
                      dvan=inp["dvan"], xq=inp["xq"], roles=inp["roles"], shifts=inp["shifts"])
    assert tm.tm_system_footprint(d)["workspace_per_rhs"] > 64 << 20
    h = tm.tm_system_create(d)
    try:
        n = tm.tm_qset_info_get(h, 0)["nelem"]
        x = torch.zeros(n, dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        tm.tm_liouvillian_apply(h, 0, x, y)          # builds the caches
        torch.cuda.synchronize()
        with pytest.raises(tm.TmError) as e:
            tm.tm_liouvillian_apply_noalloc(h, 0, x, y)
        assert e.value.code == -5
    finally:
        tm.tm_system_destroy(h)
