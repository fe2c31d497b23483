"""The chi forward-error bound (tests/chi_bound.py) holds between two CPU solvers.

The oracle's zgtsv and a dense LU solve of the same (w + i eta) I - T, for a
60-step pseudo-Hermitian chain on the cubic 20^3 system and its constant and
bi-constant extrapolations to 500 and 2000 steps (the cases the GPU test
compares), differ by less than a tenth of the bound at every frequency, and
the bound stays a sharp statement (below 1e-9 of max |chi|).
"""
import numpy as np
import pytest

import chi_bound as cb
from oracle import chi as ochi
from oracle import lanczos as olanczos

EV = 27.211386245988


@pytest.fixture(scope="module")
def chain(cubic_gs, cubic_q):
    from oracle import liouvillian as lv
    return olanczos.run(lv.build_problem(cubic_gs, cubic_q), "+", "pH", 60)


@pytest.mark.parametrize("mode,m_use,m_total", [("constant", 60, 60), ("constant", 60, 2000),
                                                ("osc", 24, 500), ("osc", 60, 2000)])
def test_bound_covers_two_solvers(chain, mode, m_use, m_total):
    e = ochi.extrapolate(chain, m_use, m_total, mode)
    omega = np.arange(0, 400, 16) * 5e-3 / EV
    eta = 5e-3 / EV
    ref = ochi.chi_lanczos(e, omega, eta, m_total)
    T = ochi.tridiag(e, m_total)
    rhs = np.zeros(m_total, complex)
    rhs[0] = 1.0
    dense = np.array([e["n1"] * (e["z"] @ np.linalg.solve((w + 1j * eta) * np.eye(m_total) - T, rhs))
                      for w in omega]).T
    bound = cb.chi_difference_bound(e, m_total, omega, eta)
    diff = np.abs(dense - ref)
    live = bound > 0            # components that vanish by symmetry have z = 0
    assert np.all(diff[~live] == 0)
    ratio = (diff[live] / bound[live]).max()
    assert ratio <= 0.1, ratio
    assert bound.max() <= 1e-9 * np.abs(ref).max()
