import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def c2_state():
    """Full 2^25 complex128 state of the 25-qubit workload (plain C oracle)."""
    import rqc
    from oracle import statevector as sv
    w = rqc.workload("c2_5x5_m16")
    return w, sv.simulate_c(w["circuit"])
