"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X).

Tolerances: FP64 throughout.  The apply and the start vectors agree to
1e-12 relative (different summation orders only).  Lanczos coefficients of
short chains agree to 1e-10 relative (the recursion amplifies rounding
differences as Ritz values converge).  chi from identical coefficients agrees
to 1e-12.
"""
import numpy as np
import pytest

import synth
from oracle import chi as ochi
from oracle import lanczos as olanczos
from oracle import liouvillian as lv

from gpu_util import desc_from_problem, from_gpu, rel_err, say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2203_01120_amd as tm
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    tm.load()
    return tm


class Sys:
    def __init__(self, tm, prob):
        self.tm, self.prob = tm, prob
        self.h = tm.tm_system_create(desc_from_problem(prob))
        self.info = tm.tm_qset_info_get(self.h, 0)
        self.shape = (2, prob.nk, prob.nb, 2, self.info["npw_pad"])

    def apply(self, x, kernel=True):
        import torch
        xin = to_gpu(x, self.info["npw_pad"])
        out = torch.empty_like(xin)
        self.tm.tm_liouvillian_apply(self.h, 0, xin, out)
        torch.cuda.synchronize()
        return from_gpu(out, self.shape, self.prob.npw_pad)

    def resident(self, on):
        """Switch between the resident real-space ground state and the column path."""
        self.tm.tm_system_set_resident_limit(self.h, -1 if on else 0)

    def resident_bytes(self):
        return self.tm.tm_system_resident_bytes(self.h)

    def close(self):
        self.tm.tm_system_destroy(self.h)


@pytest.fixture(scope="module")
def tiny(lib, tiny_gs, tiny_q):
    say("create tiny system")
    s = Sys(lib, lv.build_problem(tiny_gs, tiny_q))
    yield s
    s.close()


@pytest.fixture(scope="module")
def cubic20(lib, cubic_gs, cubic_q):
    say("create cubic20 system")
    s = Sys(lib, lv.build_problem(cubic_gs, cubic_q))
    yield s
    s.close()


@pytest.mark.parametrize("resident", [True, False], ids=["resident", "columns"])
@pytest.mark.parametrize("which", ["tiny", "cubic20"])
def test_apply_matches_oracle(which, resident, request):
    s = request.getfixturevalue(which)
    s.resident(resident)
    try:
        for seed in (1, 2):
            say(f"apply {which} resident={resident} seed {seed}")
            x = s.prob.random_projected(seed)
            got, raw = s.apply(x)
            ref = s.prob.apply(x)
            assert rel_err(got, ref) <= 1e-12, rel_err(got, ref)
            # padding of the output is zero
            npw = [kd.npw for kd in s.prob.k]
            for ik, n in enumerate(npw):
                assert np.all(raw[:, ik, :, :, n:] == 0)
        # which path ran: one slot per distinct (point, side), all bands and planes
        nslot = 2 * s.prob.nk
        n1, n2, n3 = s.prob.gs.sysd.fft
        expect = nslot * s.prob.nb * n3 * 2 * n1 * n2 * 16 if resident else 0
        assert s.resident_bytes() == expect
    finally:
        s.resident(True)


def test_apply_generic_plane_path(lib):
    """A 10^3 grid has no fixed-size plane kernel: the generic kernels run."""
    import synth
    from oracle import scf
    say("apply tiny 10^3 (generic plane kernels)")
    gs = scf.scf(synth.make_tiny(fft=(10, 10, 10), seed=3), tol=1e-12, beta=0.5)
    s = Sys(lib, lv.build_problem(gs, np.array([0.05, 0.1, 0.0]) * 2 * np.pi / 6.0))
    try:
        x = s.prob.random_projected(9)
        got, _ = s.apply(x)
        assert rel_err(got, s.prob.apply(x)) <= 1e-12
    finally:
        s.close()


@pytest.mark.parametrize("fft", [(12, 10, 8), (24, 20, 18)], ids=["12x10x8", "24x20x18"])
def test_apply_noncubic_grids(lib, fft):
    """Grid sides that differ (n1 != n2 != n3): the generic plane kernels and z
    passes, and the response potential on the in-LDS path (960 points) and on
    the line-FFT path (8640 points), where a swapped axis would show."""
    import synth
    from oracle import scf
    say(f"apply tiny {fft} (non-cubic grid)")
    gs = scf.scf(synth.make_tiny(fft=fft, seed=3), tol=1e-12, beta=0.5)
    s = Sys(lib, lv.build_problem(gs, np.array([0.05, 0.1, 0.0]) * 2 * np.pi / 6.0))
    try:
        for seed in (1, 2):
            x = s.prob.random_projected(seed)
            got, _ = s.apply(x)
            assert rel_err(got, s.prob.apply(x)) <= 1e-12
        got = lib.tm_lanczos_run(s.h, 0, "+", "pH", 10)
        ref = olanczos.run(s.prob, "+", "pH", 10)
        assert np.abs(got["beta"] - ref["beta"]).max() <= 1e-10 * ref["beta"].max()
    finally:
        s.close()


def test_apply_many_bands_staged_contractions(lib):
    """48 bands: the projector contractions have 3 x 3 output tiles, enough for
    the LDS-staged kernel the benchmark system runs; synthetic occupied
    manifold (no SCF), 24^3 grid."""
    say("apply cubic24, 48 bands (staged contractions)")
    prob = _synthetic_problem(synth.make_cubic(24, 48, 1), np.array([0.1, 0.0, 0.0]) * 2 * np.pi / 10.0, 3)
    s = Sys(lib, prob)
    try:
        for seed in (1, 2):
            x = prob.random_projected(seed)
            got, _ = s.apply(x)
            assert rel_err(got, prob.apply(x)) <= 1e-12
        got = lib.tm_lanczos_run(s.h, 0, "z", "pH", 12)
        ref = olanczos.run(prob, "z", "pH", 12)
        assert np.abs(got["beta"] - ref["beta"]).max() <= 1e-10 * ref["beta"].max()
    finally:
        s.close()


def _synthetic_problem(sd, qcart, seed):
    inp = synth.synthetic_inputs(sd, qcart, seed=seed)

    class _GS:
        pass
    gs = _GS()
    gs.sysd, gs.vrs, gs.rho = inp["sysd"], inp["vrs"], inp["rho"]
    return lv.Problem(gs, inp["qset"], point_states=[(m, e, et) for (_, m, e, et, _) in inp["points"]])


@pytest.mark.parametrize("n", [32, 48])
def test_apply_wave_plane_kernels_32_48(lib, n):
    """The wave plane kernels at 32 x 32 and at the benchmark's 48 x 48 planes
    (fused last column stage, field table, resident point order) against the
    oracle: cubic cell with the sphere filling an n^3 grid, 4 bands, synthetic
    occupied manifold.  FP64 to 1e-12, the single-precision bulk to 2e-5, two
    right-hand sides in one pass equal to single applies bit for bit."""
    import torch
    say(f"apply cubic{n}, 4 bands (wave plane kernels)")
    prob = _synthetic_problem(synth.make_cubic(n, 4, 1), np.array([0.1, 0.05, 0.0]) * 2 * np.pi / 10.0, 5)
    s = Sys(lib, prob)
    try:
        xs = [prob.random_projected(seed) for seed in (1, 2)]
        for x in xs:
            got, _ = s.apply(x)
            assert rel_err(got, prob.apply(x)) <= 1e-12, rel_err(got, prob.apply(x))
        assert s.resident_bytes() > 0
        npw_pad = s.info["npw_pad"]
        xin = torch.cat([to_gpu(x, npw_pad) for x in xs])
        n1 = xin.numel() // 2
        for prec, tol in ((lib.TM_FP32, 2e-5), (lib.TM_FP64, 1e-12)):
            out = torch.empty_like(xin)
            lib.tm_liouvillian_apply_multi(s.h, 0, 2, xin, out, prec)
            single = torch.empty_like(xin[:n1])
            lib.tm_liouvillian_apply(s.h, 0, xin[n1:], single, prec)
            torch.cuda.synchronize()
            assert torch.equal(out[n1:], single)
            got, _ = from_gpu(out[:n1], s.shape, prob.npw_pad)
            assert rel_err(got, prob.apply(xs[0])) <= tol
    finally:
        s.close()


def test_apply_two_kpoints_folded(lib):
    """Two-point mesh, q on the mesh: sister points folded with Miller shifts."""
    import synth
    from oracle import scf
    say("apply tiny 2-k mesh, folded roles")
    sd = synth.make_tiny(kmesh=((0.0, 0.0, 0.0), (0.5, 0.0, 0.0)), nbnd=3, seed=11)
    gs = scf.scf(sd, tol=1e-12, beta=0.5)
    qs = synth.qset_folded(sd, (0.5, 0.0, 0.0))
    assert np.any(qs.shifts != 0)
    prob = lv.Problem(gs, qs)
    s = Sys(lib, prob)
    try:
        for resident in (True, False):
            s.resident(resident)
            for seed in (1, 2):
                x = prob.random_projected(seed)
                got, _ = s.apply(x)
                assert rel_err(got, prob.apply(x)) <= 1e-12
            assert (s.resident_bytes() > 0) == resident
        s.resident(True)
        got = lib.tm_lanczos_run(s.h, 0, "z", "nH", 8)
        ref = olanczos.run(prob, "z", "nH", 8)
        assert np.abs(got["beta"] - ref["beta"]).max() <= 1e-10 * ref["beta"].max()
    finally:
        s.close()


def test_apply_is_linear_and_orthogonal(cubic20):
    say("apply linearity cubic20")
    a = cubic20.prob.random_projected(3)
    b = cubic20.prob.random_projected(4)
    la, _ = cubic20.apply(a)
    lb, _ = cubic20.apply(b)
    lab, _ = cubic20.apply(a + (0.3 - 0.7j) * b)
    assert rel_err(lab, la + (0.3 - 0.7j) * lb) <= 1e-12
    assert cubic20.prob.occupied_overlap(la) <= 1e-12 * np.abs(la).max()


@pytest.mark.parametrize("direction", ["x", "y", "z", "+", "-", "n"])
def test_start_vectors_match_oracle(cubic20, direction):
    import torch
    say(f"start vectors {direction}")
    n = cubic20.info["nelem"]
    u = torch.empty(n, dtype=torch.complex128, device="cuda")
    v = torch.empty_like(u)
    cubic20.tm.tm_start_vectors(cubic20.h, 0, direction, u, v)
    torch.cuda.synchronize()
    gu, _ = from_gpu(u, cubic20.shape, cubic20.prob.npw_pad)
    gv, _ = from_gpu(v, cubic20.shape, cubic20.prob.npw_pad)
    assert rel_err(gv, cubic20.prob.v_vector(direction)) <= 1e-12
    if direction in "xyzn":
        assert rel_err(gu, cubic20.prob.u_vector(direction)) <= 1e-13


@pytest.mark.parametrize("flavour,mu,nsteps", [("pH", "+", 60), ("nH", "+", 20), ("pH", "z", 20), ("pH", "n", 30),
                                               ("nH", "n", 16)])
def test_lanczos_coefficients_match_oracle(cubic20, flavour, mu, nsteps):
    """Coefficients and the overlaps with all four measure vectors (x, y, z and the charge n)."""
    say(f"lanczos cubic20 {flavour} {mu} {nsteps}")
    got = cubic20.tm.tm_lanczos_run(cubic20.h, 0, mu, flavour, nsteps)
    ref = olanczos.run(cubic20.prob, mu, flavour, nsteps, measure=("x", "y", "z", "n"))
    assert got["steps_done"] == ref["steps_done"] == nsteps
    assert not got["breakdown"]
    assert abs(got["n1"] - ref["n1"]) <= 1e-12 * ref["n1"]
    ascale = np.abs(ref["alpha"]).max()
    assert np.abs(got["alpha"] - ref["alpha"]).max() <= 1e-10 * ascale
    assert np.abs(got["beta"] - ref["beta"]).max() <= 1e-10 * ref["beta"].max()
    assert np.abs(got["gamma"] - ref["gamma"]).max() <= 1e-10 * np.abs(ref["gamma"]).max()
    zs = np.abs(ref["z"]).max()
    assert np.abs(got["z"] - ref["z"][:3]).max() <= 1e-10 * zs
    assert np.abs(got["zn"] - ref["z"][3]).max() <= 1e-10 * zs


def test_chi_tensor_matches_oracle(cubic20):
    """A column of the 4 x 4 (charge + spin) susceptibility for a charge and a spin field."""
    omega = np.arange(200) * 1e-2 / 27.211386245988
    eta = 1e-2 / 27.211386245988
    for mu, flavour in (("n", "pH"), ("z", "nH")):
        say(f"chi tensor column {mu} {flavour}")
        coeffs = cubic20.tm.tm_lanczos_run(cubic20.h, 0, mu, flavour, 24)
        got = cubic20.tm.tm_chi_tensor(coeffs, 24, omega, eta)
        four = dict(coeffs, z=np.vstack([coeffs["zn"][None], coeffs["z"]]))
        ref = ochi.chi_lanczos(four, omega, eta, 24)
        assert rel_err(got, ref) <= 1e-12
        assert np.array_equal(got[1:], cubic20.tm.tm_chi(coeffs, 24, omega, eta))
        oref = olanczos.run(cubic20.prob, mu, flavour, 24, measure=("n", "x", "y", "z"))
        assert rel_err(got, ochi.chi_lanczos(oref, omega, eta, 24)) <= 1e-9


def test_chi_matches_oracle(cubic20):
    say("chi cubic20")
    coeffs = cubic20.tm.tm_lanczos_run(cubic20.h, 0, "+", "pH", 60)
    omega = np.arange(400) * 5e-3 / 27.211386245988   # 0 .. 1.995 eV in Ha
    eta = 5e-3 / 27.211386245988
    got = cubic20.tm.tm_chi(coeffs, 60, omega, eta)
    ref = ochi.chi_lanczos(coeffs, omega, eta, 60)
    assert rel_err(got, ref) <= 1e-12
    # and against the chain run entirely by the oracle
    oref = olanczos.run(cubic20.prob, "+", "pH", 60)
    cref = ochi.chi_lanczos(oref, omega, eta, 60)
    assert rel_err(got, cref) <= 1e-9


def test_nonhermitian_chi_solver_with_pivoting(lib, tiny):
    """Complex alpha/gamma and near-singular leading entries exercise the row interchanges."""
    say("chi solver pivoting")
    rng = np.random.default_rng(7)
    M = 40
    co = dict(alpha=rng.standard_normal(M) * 1e-3 + 1j * rng.standard_normal(M) * 1e-4,
              beta=np.abs(rng.standard_normal(M)) + 0.5,
              gamma=rng.standard_normal(M) + 1j * rng.standard_normal(M),
              z=rng.standard_normal((3, M)) + 1j * rng.standard_normal((3, M)),
              n1=1.7, steps_done=M)
    omega = np.linspace(-0.01, 0.01, 33)
    got = lib.tm_chi(co, M, omega, 1e-6)
    ref = ochi.chi_lanczos(co, omega, 1e-6, M)
    assert rel_err(got, ref) <= 1e-10


def test_goldstone_breakdown(lib, tiny_gs_nosoc):
    say("goldstone breakdown")
    prob = lv.build_problem(tiny_gs_nosoc, np.zeros(3))
    s = Sys(lib, prob)
    try:
        r = lib.tm_lanczos_run(s.h, 0, "x", "nH", 5)
        assert r["breakdown"] and r["steps_done"] == 1
        r = lib.tm_lanczos_run(s.h, 0, "x", "pH", 5)
        assert r["breakdown"] and r["steps_done"] == 0
        ref = olanczos.run(prob, "x", "pH", 5)
        assert ref["breakdown"] and ref["steps_done"] == 0
    finally:
        s.close()


def test_invalid_arguments(lib, tiny):
    import torch
    say("invalid arguments")
    n = tiny.info["nelem"]
    x = torch.zeros(n, dtype=torch.complex128, device="cuda")
    with pytest.raises(lib.TmError) as e:
        lib.tm_liouvillian_apply(tiny.h, 0, x, x)
    assert e.value.code == lib.TM_EINVAL
    with pytest.raises(lib.TmError) as e:
        lib.tm_liouvillian_apply(tiny.h, 3, x, torch.zeros_like(x))
    assert e.value.code == lib.TM_EINVAL
    with pytest.raises(lib.TmError) as e:
        lib.tm_liouvillian_apply(tiny.h, 0, x, torch.zeros_like(x), prec=7)   # no such precision
    assert e.value.code == lib.TM_EINVAL
    co = dict(alpha=np.zeros(3, complex), beta=np.zeros(3), gamma=np.zeros(3, complex),
              z=np.zeros((3, 3), complex), n1=1.0, steps_done=2)
    with pytest.raises(lib.TmError):
        lib.tm_chi(co, 3, np.zeros(4), 0.1)
