"""The autotuner's candidates (tm_autotune_*) through the C ABI.

Every compiled variant of every tunable launch, forced in turn, gives the
oracle's apply at 1e-12 on systems that reach them: the 20^3 system (20 x 20
plane kernels, z passes of 20), a cubic cell on a 48^3 grid (the benchmark's
48 x 48 plane kernels, z passes of 48), the serving pool's 48 x 48 x 96 slab (z
passes of 96), a 32^3 grid and a 24^3 grid with 48 bands (the LDS-staged
contractions and their K splits).  Plane, z-pass and update variants only split the work or
order the loads differently, so their outputs are identical to variant 0's;
the contraction variants sum K in other splits.  The full-size system's
variants (z passes of 180, 104-band contractions) are checked in the
full-size tests.
"""
import numpy as np
import pytest

import synth
from oracle import liouvillian as lv

from gpu_util import desc_from_problem, from_gpu, rel_err, say, to_gpu

pytestmark = pytest.mark.gpu

BITWISE = ("plane_density", "plane_apply", "zpass_inverse", "zpass_forward", "update")


def _synthetic_problem(sd, qcart, seed):
    inp = synth.synthetic_inputs(sd, qcart, seed=seed)

    class _GS:
        pass
    gs = _GS()
    gs.sysd, gs.vrs, gs.rho = inp["sysd"], inp["vrs"], inp["rho"]
    return lv.Problem(gs, inp["qset"], point_states=[(m, e, et) for (_, m, e, et, _) in inp["points"]])


def check_every_variant(tm, h, prob, shape, expect_ops):
    import torch
    info = tm.tm_qset_info_get(h, 0)
    x = prob.random_projected(4)
    ref = prob.apply(x)
    xin = to_gpu(x, info["npw_pad"])
    out = torch.empty_like(xin)
    tm.tm_liouvillian_apply(h, 0, xin, out)          # the first apply tunes this shape
    torch.cuda.synchronize()
    entries = [e for e in tm.tm_autotune_report() if shape in e["shape"]]
    say(f"tuned for {shape}: " + "; ".join(f"{e['op']} {e['chosen']}/{e['variants']} {e['us']}" for e in entries))
    assert {e["op"] for e in entries} >= set(expect_ops), entries
    for e in entries:
        base = None
        try:
            for v in range(e["variants"]):
                tm.tm_autotune_force(e["op"], v)
                tm.tm_liouvillian_apply(h, 0, xin, out)
                torch.cuda.synchronize()
                got, raw = from_gpu(out, (2, prob.nk, prob.nb, 2, info["npw_pad"]), prob.npw_pad)
                err = rel_err(got, ref)
                say(f"  {e['op']} variant {v}: rel err {err:.2e}")
                assert err <= 1e-12, (e["op"], v, err)
                if e["op"] in BITWISE:
                    if base is None:
                        base = raw.copy()
                    assert np.array_equal(raw, base), (e["op"], v)
        finally:
            tm.tm_autotune_force(e["op"], -1)


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2203_01120_amd as tm
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    return tm


def test_variants_cubic20(lib, cubic_gs, cubic_q):
    prob = lv.build_problem(cubic_gs, cubic_q)
    h = lib.tm_system_create(desc_from_problem(prob))
    try:
        check_every_variant(lib, h, prob, "grid 20x20x20, 8 bands, 1 k",
                            ["plane_density", "plane_apply", "zpass_inverse", "zpass_forward"])
    finally:
        lib.tm_system_destroy(h)


@pytest.mark.parametrize("n,nb", [(48, 4), (24, 48), (32, 4)], ids=["48^3-4bands", "24^3-48bands", "32^3-4bands"])
def test_variants_synthetic(lib, n, nb):
    prob = _synthetic_problem(synth.make_cubic(n, nb, 1), np.array([0.1, 0.05, 0.0]) * 2 * np.pi / 10.0, 5)
    h = lib.tm_system_create(desc_from_problem(prob))
    try:
        ops = ["plane_density", "plane_apply", "zpass_inverse", "zpass_forward"]
        if nb == 48:
            ops += ["contraction", "update"]
        check_every_variant(lib, h, prob, f"grid {n}x{n}x{n}, {nb} bands, 1 k", ops)
    finally:
        lib.tm_system_destroy(h)


def test_variants_slab96(lib):
    """The 48 x 48 x 96 slab of the serving pool (4 bands, Gamma only): the
    plane kernels of 48 x 48 and the z passes of 96."""
    sd = synth.make_hexslab(c=16.5, fft=(48, 48, 96), nbnd=4, nk=1)
    prob = _synthetic_problem(sd, synth.cart_from_frac(sd, [0.25, 0.0, 0.0]), 3)
    h = lib.tm_system_create(desc_from_problem(prob))
    try:
        check_every_variant(lib, h, prob, "grid 48x48x96, 4 bands, 1 k",
                            ["plane_density", "plane_apply", "zpass_inverse", "zpass_forward"])
    finally:
        lib.tm_system_destroy(h)


def test_force_out_of_range_is_an_error(lib, tiny_gs, tiny_q):
    import torch
    prob = lv.build_problem(tiny_gs, tiny_q)
    h = lib.tm_system_create(desc_from_problem(prob))
    try:
        n = lib.tm_qset_info_get(h, 0)["nelem"]
        x = torch.zeros(n, dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        lib.tm_autotune_force("plane_apply", 99)
        with pytest.raises(lib.TmError) as e:
            lib.tm_liouvillian_apply(h, 0, x, y)
        assert e.value.code == lib.TM_EINVAL
    finally:
        lib.tm_autotune_force("plane_apply", -1)
        lib.tm_system_destroy(h)
