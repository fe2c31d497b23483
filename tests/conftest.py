import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def tiny_gs():
    import synth
    from oracle import scf
    return scf.scf(synth.make_tiny(), tol=1e-12, beta=0.5)


@pytest.fixture(scope="session")
def tiny_gs_nosoc():
    import synth
    from oracle import scf
    return scf.scf(synth.make_tiny(soc=0.0), tol=1e-13, beta=0.5)


@pytest.fixture(scope="session")
def cubic_gs():
    import synth
    from oracle import scf
    return scf.scf(synth.make_cubic20(), tol=1e-10, beta=0.5)


@pytest.fixture(scope="session")
def tiny_q():
    return np.array([0.1, 0.05, 0.0]) * 2 * np.pi / 6.0


@pytest.fixture(scope="session")
def cubic_q():
    return np.array([0.1, 0.0, 0.0]) * 2 * np.pi / 10.0
