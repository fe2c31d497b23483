"""Oracle pins for the grid conventions, the Hartree operator and the xc kernel.

Each check compares the oracle with something it does not compute itself:
direct DFT sums, closed-form electrostatics, finite differences, a supercell
construction.
"""
import numpy as np
import pytest
from scipy.special import erf

import synth
from oracle import grid, scf, xc


def _box(a=(4.0, 5.0, 6.0), fft=(4, 5, 6), ecut=3.0):
    cell = np.diag(a)
    return synth.SystemDef(name="box", cell=cell, atoms=[], ecut=ecut, fft=fft, nbnd=1,
                           kmesh=np.zeros((1, 3)))


def test_to_grid_is_direct_dft():
    """P1: sphere->grid equals sum_G c(G) exp(i (G).r_j) written out pointwise."""
    sd = _box()
    k = np.array([0.1, -0.2, 0.05])
    mill = synth.sphere(sd, k, ecut=2.0)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(len(mill)) + 1j * rng.standard_normal(len(mill))
    psi = grid.to_grid(sd.fft, mill, c)
    r = synth.grid_points(sd)
    G = mill @ sd.recip
    direct = np.einsum("g,xyzg->xyz", c, np.exp(1j * np.einsum("xyzi,gi->xyzg", r, G)))
    assert np.abs(psi - direct).max() < 1e-12
    back = grid.from_grid(sd.fft, mill, psi)
    assert np.abs(back - c).max() < 1e-13
    # Parseval: (1/N) sum |psi|^2 = sum |c|^2
    assert abs(np.mean(np.abs(psi) ** 2) - np.sum(np.abs(c) ** 2)) < 1e-12


def test_sphere_count_matches_volume_estimate():
    sd = synth.make_cubic20()
    n = len(synth.sphere(sd, np.zeros(3)))
    est = sd.omega * (2 * sd.ecut) ** 1.5 / (6 * np.pi ** 2)
    assert abs(n - est) / est < 0.05
    mill = synth.sphere(sd, np.zeros(3))
    K = mill @ sd.recip
    assert np.all(0.5 * np.sum(K * K, axis=1) < sd.ecut)


def test_density_integrates_to_electron_count(tiny_gs):
    assert abs(tiny_gs.nelec - tiny_gs.sysd.nbnd) < 1e-10


def test_hartree_of_gaussian_matches_erf_potential():
    """v_H of a unit Gaussian charge in a cubic box (neutralising background):
    near the charge v(r) - v(0) = erf(r/(sqrt2 s))/r - sqrt(2/pi)/s + (2 pi/3) nbar r^2
    (the image sum adds no r^2 term for cubic symmetry)."""
    L, n, s = 24.0, 48, 1.0
    sd = _box((L, L, L), (n, n, n))
    r = synth.grid_points(sd)
    c = np.array([L / 2, L / 2, L / 2])
    d = np.linalg.norm(r - c, axis=-1)
    rho = np.exp(-d ** 2 / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5
    v = scf.hartree(sd, rho)
    nbar = 1.0 / L ** 3
    sel = (d < 2.0) & (d > 0)
    v0 = v[n // 2, n // 2, n // 2]
    ref = erf(d[sel] / (np.sqrt(2) * s)) / d[sel] - np.sqrt(2 / np.pi) / s + 2 * np.pi / 3 * nbar * d[sel] ** 2
    assert np.abs((v[sel] - v0) - ref).max() < 2e-5


def test_response_hartree_equals_supercell_hartree():
    """v'_H for q = b1/2 on the cell equals exp(-iq.r) times the q=0 Hartree
    potential of exp(iq.r) n'(r) computed in the doubled supercell."""
    sd = _box((5.0, 5.0, 5.0), (10, 10, 10))
    rng = np.random.default_rng(3)
    npr = rng.standard_normal(sd.fft) + 1j * rng.standard_normal(sd.fft)
    # smooth it so that the supercell grid represents it exactly
    F = np.fft.fftn(npr)
    Gm, mask = grid.grid_gvectors(sd)
    F *= np.exp(-0.5 * np.sum(Gm ** 2, axis=-1)) * mask
    npr = np.fft.ifftn(F)
    q = sd.recip[0] / 2
    vq = grid.apply_coulomb(grid.coulomb_multiplier(sd, q), npr)
    sc = _box((10.0, 5.0, 5.0), (20, 10, 10))
    r = synth.grid_points(sc)
    ph = np.exp(1j * r @ q)
    big = np.concatenate([npr, npr], axis=0) * ph
    vbig = grid.apply_coulomb(grid.coulomb_multiplier(sc, np.zeros(3)), big) / ph
    assert np.abs(vbig[:10] - vq).max() < 1e-10 * np.abs(vq).max()
    assert np.abs(vbig[10:] - vq).max() < 1e-10 * np.abs(vq).max()


def test_slater_energy_limits():
    """Unpolarised Dirac exchange -(3/4)(3/pi)^{1/3} n^{4/3}; full polarisation x 2^{1/3}."""
    n = np.array([0.01, 0.3, 2.0])
    rho = np.stack([n, 0 * n, 0 * n, 0 * n])
    assert np.allclose(xc.energy_density(rho), -0.75 * (3 / np.pi) ** (1 / 3) * n ** (4 / 3), rtol=1e-13)
    rho = np.stack([n, 0 * n, 0 * n, n])
    assert np.allclose(xc.energy_density(rho), -0.75 * (3 / np.pi) ** (1 / 3) * 2 ** (1 / 3) * n ** (4 / 3),
                       rtol=1e-13)


def _fd_grad(fun, x, h):
    g = []
    for i in range(4):
        e = np.zeros(4)
        e[i] = h
        g.append((fun(x + e) - fun(x - e)) / (2 * h))
    return np.array(g)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_potentials_are_energy_derivatives(seed):
    """v_xc = de/dn and B = de/dm by central differences (noncollinear m)."""
    rng = np.random.default_rng(seed)
    n = rng.uniform(0.05, 0.5)
    m = rng.standard_normal(3)
    m *= rng.uniform(0.1, 0.8) * n / np.linalg.norm(m)
    x = np.concatenate([[n], m])
    g = _fd_grad(lambda y: xc.energy_density(y[:, None])[0], x, 1e-6)
    vxc, B = xc.potentials(x[:, None])
    assert np.allclose(g[0], vxc[0], rtol=1e-7)
    assert np.allclose(g[1:], B[:, 0], rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_kernel_is_potential_derivative(seed):
    """P3: f_ab = d(v_xc, B)_a / d(n, m)_b by central differences."""
    rng = np.random.default_rng(seed)
    n = rng.uniform(0.05, 0.5)
    m = rng.standard_normal(3)
    m *= rng.uniform(0.1, 0.8) * n / np.linalg.norm(m)
    x = np.concatenate([[n], m])

    def pot(y):
        v, B = xc.potentials(y[:, None])
        return np.concatenate([v, B[:, 0]])

    g = _fd_grad(pot, x, 1e-6).T  # g[a][b] = d pot_a / d x_b
    f = xc.kernel(x[:, None])[:, :, 0]
    assert np.allclose(f, f.T)
    assert np.allclose(g, f, rtol=1e-6, atol=1e-6 * np.abs(f).max())


def test_kernel_isotropic_limit():
    x = np.array([[0.2], [0.0], [0.0], [0.0]])
    f = xc.kernel(x)[:, :, 0]
    g = -(xc.CX / 3) * 0.1 ** (-2 / 3)
    assert np.allclose(f, np.diag([g / 2, g / 2, g / 2, g / 2]), rtol=1e-12)


@pytest.mark.parametrize("nbnd,mfrac", [(1, (0.0, 0.0, 0.5)), (2, (0.0, 0.0, 0.0))])
def test_scf_homogeneous_gas_limit(nbnd, mfrac):
    """Without atoms the SCF ground state is the homogeneous electron gas: the
    G = 0 plane wave(s), a uniform density N / Omega, and eigenvalue
    v_sigma = -(6/pi)^(1/3) n_sigma^(1/3) (Slater exchange; Hartree vanishes for
    a uniform density).  One electron ends fully polarised along the starting
    moment; two unpolarised electrons fill both spins at the same energy."""
    sd = synth.make_tiny(nat=0, nbnd=nbnd, fft=(8, 8, 8))
    gs = scf.scf(sd, tol=1e-12, beta=0.5, mfrac=mfrac)
    _, _, _, e = gs.mesh_states[0]
    n_sigma = 1.0 / sd.omega                       # one electron per occupied spin channel
    v = -(6.0 / np.pi) ** (1.0 / 3.0) * n_sigma ** (1.0 / 3.0)
    assert np.allclose(gs.rho[0], nbnd / sd.omega, rtol=1e-12, atol=0)
    assert np.allclose(e, v, rtol=1e-10, atol=0)
    if nbnd == 1:
        assert np.allclose(gs.rho[3], gs.rho[0], rtol=1e-12, atol=0)   # |m| = n along z
        assert np.abs(gs.rho[1:3]).max() < 1e-14
        assert abs(gs.gaps[0] + v) < 1e-5 * abs(v)     # the empty spin channel sits at v = 0
    else:
        assert np.abs(gs.rho[1:]).max() < 1e-14
