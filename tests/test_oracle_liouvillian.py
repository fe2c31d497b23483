"""Oracle pins for the Liouvillian, its start vectors and the Lanczos chains.

Independent references: the transition-space construction (sum over
transitions with pair densities), the textbook K = 0 Kubo sum from full
diagonalisations, the spin commutator identity behind the sum rule, the
Goldstone zero mode, time reversal applied literally, Krylov moments.
"""
import numpy as np
import pytest

import synth
from oracle import chi, dense, grid, lanczos, liouvillian as lv


@pytest.fixture(scope="module")
def tiny_prob(tiny_gs, tiny_q):
    return lv.build_problem(tiny_gs, tiny_q)


@pytest.fixture(scope="module")
def tiny_ts(tiny_prob):
    return dense.TransitionSpace(tiny_prob)


def test_scf_converged(tiny_gs, cubic_gs):
    assert tiny_gs.residual < 1e-12
    assert cubic_gs.residual < 1e-10
    assert cubic_gs.gaps[0] >= 0.02
    assert np.linalg.norm(cubic_gs.magnetization) >= 0.5


def test_matrix_free_equals_transition_space(tiny_ts):
    """P4: the grid-based Liouvillian equals J(D + P^dag F P) column by column."""
    Lmf = tiny_ts.matrix_free_columns()
    Ld = tiny_ts.liouvillian()
    assert np.abs(Lmf - Ld).max() <= 1e-12 * np.abs(Ld).max()
    Lmf0 = tiny_ts.matrix_free_columns(kernel=False)
    assert np.abs(Lmf0 - tiny_ts.liouvillian(kernel=False)).max() <= 1e-12 * np.abs(Ld).max()


def test_pseudo_hermitian_structure(tiny_ts, tiny_prob):
    """P5: JL is Hermitian; matrix-free probes a^dag J L b = conj(b^dag J L a)."""
    Ld = tiny_ts.liouvillian()
    JL = tiny_ts.Jdiag[:, None] * Ld
    assert np.abs(JL - JL.conj().T).max() <= 1e-13 * np.abs(JL).max()
    a = tiny_prob.random_projected(1)
    b = tiny_prob.random_projected(2)
    lhs = tiny_prob.dot(a, tiny_prob.J(tiny_prob.apply(b)))
    rhs = np.conj(tiny_prob.dot(b, tiny_prob.J(tiny_prob.apply(a))))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_output_orthogonal_to_occupied(tiny_prob):
    y = tiny_prob.apply(tiny_prob.random_projected(5))
    assert tiny_prob.occupied_overlap(y) < 1e-12 * np.abs(y).max()


@pytest.mark.parametrize("lam,mu", [("x", "x"), ("x", "y"), ("y", "x"), ("z", "z"), ("x", "z"),
                                    ("n", "n"), ("n", "z"), ("z", "n"), ("x", "n")])
def test_k0_matches_kubo_sum(tiny_gs, tiny_prob, tiny_ts, lam, mu):
    """P2: with the kernel off, (u, (w - L)^{-1} v) is the textbook Kubo sum
    (n: the charge channel, sigma_0; pins its time-reversal signs)."""
    om = np.linspace(-2.0, 2.0, 41)
    L0 = tiny_ts.liouvillian(kernel=False)
    cd = tiny_ts.chi_dense(L0, tiny_prob.u_vector(lam), tiny_prob.v_vector(mu), om, 0.05)
    ck = chi.kubo_k0(tiny_gs, tiny_prob, lam, mu, om, 0.05)
    scale = max(np.abs(ck).max(), 1.0)
    assert np.abs(cd - ck).max() <= 1e-12 * scale


def test_sum_over_transitions_equals_resolvent(tiny_prob, tiny_ts):
    om = np.linspace(-1.0, 1.0, 21)
    L = tiny_ts.liouvillian()
    u, v = tiny_prob.u_vector("y"), tiny_prob.v_vector("+")
    cs, lam = tiny_ts.chi_sot(L, u, v, om, 0.05)
    cd = tiny_ts.chi_dense(L, u, v, om, 0.05)
    assert np.abs(cs - cd).max() <= 1e-10 * np.abs(cd).max()


def test_sum_rule_identity_at_q0(tiny_gs):
    """P6: (u^l, v^m) = 2 i eps_lmn M_n (the commutator [s_l, s_m] = 2i eps s_n)."""
    prob = lv.build_problem(tiny_gs, np.zeros(3))
    # moment of the occupied states themselves (the SCF density differs by its residual)
    _, evc, _ = prob.point_states[0]
    M = np.array([np.einsum("nsg,st,ntg->", evc.conj(), lv.DIRECTIONS[c], evc).real for c in "xyz"])
    assert np.allclose(M, tiny_gs.magnetization, atol=1e-10)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1
    for i, l in enumerate("xyz"):
        for j, m in enumerate("xyz"):
            val = prob.dot(prob.u_vector(l), prob.v_vector(m))
            assert abs(val - 2j * eps[i, j] @ M) < 1e-12


def test_charge_channel_commutes_at_q0(tiny_gs):
    """P6 for the charge row and column: sigma_0 commutes with every sigma, so
    (u^n, v^m) = 0 at q = 0 while both vectors are nonzero; and a uniform
    potential moves no charge, so v^n itself vanishes at q = 0 (the occupied
    states are projected out of themselves) but not at finite q."""
    prob = lv.build_problem(tiny_gs, np.zeros(3))
    un = prob.u_vector("n")
    assert np.linalg.norm(un) > 0.1
    for m in "xy+":   # (v^z may vanish too: the tiny system keeps S_z)
        vm = prob.v_vector(m)
        assert np.linalg.norm(vm) > 1e-3
        assert abs(prob.dot(un, vm)) < 1e-12
    assert np.abs(prob.v_vector("n")).max() < 1e-13
    assert np.linalg.norm(lv.build_problem(tiny_gs, synth.cart_from_frac(tiny_gs.sysd, (0.1, 0.05, 0))).v_vector("n")) > 1e-2


def test_sum_rule_frequency_integral(tiny_prob):
    """P6 (integral form): int chi_lm dw = -i pi (u^l, v^m) for any M and eta;
    checked by numerical quadrature of the Lanczos chi over a wide window."""
    res = lanczos.run(tiny_prob, "y", "nH", 30)
    om = np.concatenate([np.linspace(-400, -10, 40001), np.linspace(-10, 10, 200001)[1:-1],
                         np.linspace(10, 400, 40001)])
    c = chi.chi_lanczos(res, om, 0.5)
    integ = np.trapezoid(c[0], om)
    target = -1j * np.pi * tiny_prob.dot(tiny_prob.u_vector("x"), tiny_prob.v_vector("y"))
    assert abs(integ - target) <= 0.01 * abs(target)


def test_goldstone_zero_mode(tiny_gs_nosoc):
    """P7: at q = 0 without SOC, the rigid-rotation vectors v^x, v^y are zero modes."""
    prob = lv.build_problem(tiny_gs_nosoc, np.zeros(3))
    M = tiny_gs_nosoc.magnetization
    assert abs(M[0]) < 1e-10 and abs(M[1]) < 1e-10 and abs(M[2]) > 0.5
    r = prob.random_projected(3)
    r *= np.linalg.norm(prob.v_vector("x")) / np.linalg.norm(r)
    ref = np.linalg.norm(prob.apply(r))
    for mu in "xy":
        v = prob.v_vector(mu)
        assert np.linalg.norm(v) > 0.1
        assert np.linalg.norm(prob.apply(v)) < 1e-8 * ref
    # exact breakdown of the two-sided chain right at the first step
    res = lanczos.run(prob, "x", "nH", 5)
    assert res["breakdown"] and res["steps_done"] == 1


def test_time_reversal_shortcut(tiny_gs, tiny_q):
    """P13: T H_{-k-q} T^{-1} equals H_{k+q} with the B field reversed."""
    kq = tiny_q
    m_kq = synth.sphere(tiny_gs.sysd, kq)
    m_m = synth.sphere(tiny_gs.sysd, -kq)
    Hp = tiny_gs.hamiltonian(kq, m_kq, bsign=-1.0)
    Hm = tiny_gs.hamiltonian(-kq, m_m)
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((2, len(m_kq))) + 1j * rng.standard_normal((2, len(m_kq)))
    # T^{-1} = -T for spin 1/2
    tinv = -grid.time_reverse(m_kq, psi, m_m)
    h = (Hm @ tinv.ravel()).reshape(2, -1)
    lhs = grid.time_reverse(m_m, h, m_kq)
    rhs = (Hp @ psi.ravel()).reshape(2, -1)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


@pytest.mark.parametrize("flavour,mu", [("pH", "z"), ("nH", "+"), ("nH", "z")])
def test_lanczos_moments(tiny_prob, flavour, mu):
    """P10: (u, L^k v) = n1 z^T T^k e1 for k < M (any Krylov method)."""
    M = 8
    res = lanczos.run(tiny_prob, mu, flavour, M)
    assert res["steps_done"] == M
    T = chi.tridiag(res, M)
    v = tiny_prob.v_vector(mu)
    Lkv = v.copy()
    e = np.zeros(M, dtype=complex)
    e[0] = 1
    for k in range(M - 1):
        for l, lam in enumerate("xyz"):
            lhs = tiny_prob.dot(tiny_prob.u_vector(lam), Lkv)
            rhs = res["n1"] * res["z"][l] @ e
            scale = np.linalg.norm(Lkv) * np.linalg.norm(tiny_prob.u_vector(lam)) / tiny_prob.nk
            assert abs(lhs - rhs) <= 1e-11 * scale
        Lkv = tiny_prob.apply(Lkv)
        e = T @ e


def test_flavours_agree_with_dense(tiny_prob, tiny_ts):
    """P11: pseudo-Hermitian and non-Hermitian chi converge to the dense resolvent."""
    om = np.linspace(-3.0, 3.0, 61)
    L = tiny_ts.liouvillian()
    v = tiny_prob.v_vector("z")
    cd = np.array([tiny_ts.chi_dense(L, tiny_prob.u_vector(l), v, om, 0.3) for l in "xyz"])
    for fl in ("pH", "nH"):
        res = lanczos.run(tiny_prob, "z", fl, 60)
        cl = chi.chi_lanczos(res, om, 0.3)
        assert np.abs(cl - cd).max() <= 1e-6 * np.abs(cd).max(), fl
    res = lanczos.run(tiny_prob, "+", "nH", 60)
    cl = chi.chi_lanczos(res, om, 0.3)
    cd = np.array([tiny_ts.chi_dense(L, tiny_prob.u_vector(l), tiny_prob.v_vector("+"), om, 0.3)
                   for l in "xyz"])
    assert np.abs(cl - cd).max() <= 1e-6 * np.abs(cd).max()


def test_symmetry_zeros_without_transverse_coupling(tiny_prob):
    """P9: H commutes with S_z here, so longitudinal and transverse sectors decouple:
    z^{x,z} = z^{y,z} = 0 and chi_xy = -chi_yx."""
    res = lanczos.run(tiny_prob, "z", "pH", 20)
    assert np.abs(res["z"][0]).max() < 1e-13 and np.abs(res["z"][1]).max() < 1e-13
    om = np.linspace(-1, 1, 11)
    rx = lanczos.run(tiny_prob, "x", "nH", 40)
    ry = lanczos.run(tiny_prob, "y", "nH", 40)
    cxy = chi.chi_lanczos(ry, om, 0.2)[0]
    cyx = chi.chi_lanczos(rx, om, 0.2)[1]
    assert np.abs(cxy + cyx).max() <= 1e-6 * np.abs(cxy).max()


def test_chi_solvers_agree(tiny_prob):
    """P14: zgtsv vs continued fraction vs pole-residue."""
    res = lanczos.run(tiny_prob, "+", "nH", 25)
    om = np.linspace(-2, 2, 31)
    c1 = chi.chi_lanczos(res, om, 0.1)
    c2 = chi.chi_pole_residue(res, om, 0.1)
    assert np.abs(c1 - c2).max() <= 1e-10 * np.abs(c1).max()
    cf = chi.continued_fraction_11(res, om, 0.1)
    z1 = np.zeros_like(res["z"])
    z1[:, 0] = res["z"][:, 0]
    c3 = chi.chi_lanczos(dict(res, z=z1), om, 0.1)
    assert np.abs(c3[0] - res["n1"] * res["z"][0, 0] * cf).max() <= 1e-12 * np.abs(c3[0]).max()


def test_cubic20_pseudo_hermitian_probe_and_chain(cubic_gs, cubic_q):
    """cubic20: JL symmetric on random probes; a short pH chain runs without breakdown."""
    prob = lv.build_problem(cubic_gs, cubic_q)
    a, b = prob.random_projected(11), prob.random_projected(12)
    lhs = prob.dot(a, prob.J(prob.apply(b)))
    rhs = np.conj(prob.dot(b, prob.J(prob.apply(a))))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    res = lanczos.run(prob, "+", "pH", 6)
    assert res["steps_done"] == 6 and not res["breakdown"]
    assert np.all(res["beta"][:6] > 0)


@pytest.mark.parametrize("flavour,mu,m", [("pH", "z", 20), ("nH", "+", 12)])
def test_reprojection_is_the_identity_on_short_chains(tiny_prob, flavour, mu, m):
    """Projecting the recursion's vectors back onto the empty manifold changes
    nothing in exact arithmetic: short chains agree with and without it."""
    a = lanczos.run(tiny_prob, mu, flavour, m, reproject=True)
    b = lanczos.run(tiny_prob, mu, flavour, m, reproject=False)
    assert a["steps_done"] == b["steps_done"] == m
    for key in ("alpha", "beta", "gamma"):
        assert np.abs(a[key] - b[key]).max() <= 1e-9 * np.abs(b[key]).max(), key


def _synthetic_problem(sysd, q, seed):
    """Oracle Problem on seeded synthetic inputs (no SCF), as the benchmark builds them."""
    class _GS:
        pass
    inp = synth.synthetic_inputs(sysd, q, seed=seed)
    gs = _GS()
    gs.sysd, gs.vrs, gs.rho = inp["sysd"], inp["vrs"], inp["rho"]
    return lv.Problem(gs, inp["qset"], point_states=[(m, e, et) for (_, m, e, et, _) in inp["points"]])


def test_reprojection_removes_occupied_leakage():
    """Without re-projection, rounding-level occupied components (null space of
    the metric JL) grow until the pseudo-Hermitian chain breaks down; with it
    the chain runs on, and its leading coefficients agree with the unprojected
    chain (identity in exact arithmetic)."""
    sysd = synth.make_cubic20()
    prob = _synthetic_problem(sysd, synth.cart_from_frac(sysd, synth.q_path(24)[4]), seed=1)
    b = lanczos.run(prob, "+", "pH", 180, reproject=False)
    assert b["breakdown"] and b["steps_done"] < 180
    a = lanczos.run(prob, "+", "pH", 180, reproject=True)
    assert not a["breakdown"] and a["steps_done"] == 180
    k = 40
    assert np.abs(a["beta"][:k] - b["beta"][:k]).max() <= 1e-8 * b["beta"][:k].max()
    assert lanczos.run(prob, "+", "pH", 1)["n1"] > 0
    assert prob.occupied_overlap(prob.random_projected(3)) < 1e-12


def _chain(alpha, beta, gamma):
    m = len(alpha)
    z = np.zeros((3, m), dtype=np.complex128)
    z[0, 0] = 1.0
    return dict(alpha=np.asarray(alpha, dtype=np.complex128), beta=np.asarray(beta, dtype=float),
                gamma=np.asarray(gamma, dtype=np.complex128), z=z, n1=1.0, steps_done=m)


def test_constant_extrapolation_reaches_the_infinite_chain():
    """A chain with constant a, b continued by 'constant' extrapolation tends to
    the closed-form Green's function of the infinite chain,
    G = (w' - a - sqrt((w' - a)^2 - 4 b^2)) / (2 b^2), Im G < 0."""
    a, b, eta = 0.3, 0.5, 0.05
    co = _chain([a] * 8, [b] * 8, [b] * 8)
    omega = np.linspace(-1.5, 2.0, 71)
    ext = chi.extrapolate(co, 8, 3000, "constant")
    got = chi.chi_lanczos(ext, omega, eta, 3000)[0]
    wc = omega + 1j * eta
    r = np.sqrt((wc - a) ** 2 - 4 * b * b)
    G = np.where(((wc - a - r) / (2 * b * b)).imag < 0, (wc - a - r) / (2 * b * b), (wc - a + r) / (2 * b * b))
    assert np.abs(got - G).max() <= 1e-8 * np.abs(G).max()
    # without extrapolation the 8-step chain is visibly different (finite poles)
    assert np.abs(chi.chi_lanczos(co, omega, eta, 8)[0] - G).max() > 1e-2 * np.abs(G).max()


def test_osc_extrapolation_reaches_the_two_periodic_chain():
    """Alternating couplings b1, b2 (alpha = 0) continued by the bi-constant scheme
    tend to the closed form of the 2-periodic infinite chain:
    w b2^2 G^2 - (w^2 - b1^2 + b2^2) G + w = 0 (the root with Im G < 0)."""
    b1, b2, eta = 0.6, 0.25, 0.04
    co = _chain([0.0] * 8, [b1, b2] * 4, [b1, b2] * 4)
    omega = np.linspace(0.05, 1.2, 47)
    ext = chi.extrapolate(co, 8, 4000, "osc")
    got = chi.chi_lanczos(ext, omega, eta, 4000)[0]
    w = omega + 1j * eta
    A, B, Cc = w * b2 ** 2, -(w ** 2 - b1 ** 2 + b2 ** 2), w
    disc = np.sqrt(B * B - 4 * A * Cc)
    r1, r2 = (-B + disc) / (2 * A), (-B - disc) / (2 * A)
    G = np.where(r1.imag < 0, r1, r2)
    assert np.all(G.imag < 0)
    assert np.abs(got - G).max() <= 1e-8 * np.abs(G).max()
    # the constant scheme averages b1 and b2 and misses the gap structure
    cst = chi.chi_lanczos(chi.extrapolate(co, 8, 4000, "constant"), omega, eta, 4000)[0]
    assert np.abs(cst - G).max() > 1e-2 * np.abs(G).max()


def test_no_extrapolation_is_the_plain_chain(tiny_prob):
    c = lanczos.run(tiny_prob, "z", "pH", 12)
    omega = np.linspace(0.0, 0.1, 9)
    ext = chi.extrapolate(c, 12, 12, "constant")
    assert np.array_equal(chi.chi_lanczos(ext, omega, 1e-3, 12), chi.chi_lanczos(c, omega, 1e-3, 12))


def test_structure_factor_transverse_projector():
    """q along z keeps -Im(chi_xx + chi_yy); S is invariant under a common rotation of q and chi."""
    rng = np.random.default_rng(4)
    c3 = rng.standard_normal((3, 3, 5)) + 1j * rng.standard_normal((3, 3, 5))
    s = chi.structure_factor([0, 0, 0.7], c3)
    assert np.allclose(s, -(c3[0, 0] + c3[1, 1]).imag, atol=1e-14)
    th = 0.83
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(0.4), -np.sin(0.4)], [0, np.sin(0.4), np.cos(0.4)]])
    R = Rx @ Rz
    q = np.array([0.2, -0.1, 0.5])
    rot = np.einsum("ab,bcw,dc->adw", R, c3, R)
    assert np.allclose(chi.structure_factor(R @ q, rot), chi.structure_factor(q, c3), atol=1e-13)
