import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session")
def c1():
    """Config-1 bar: structure, oracle mesh, circuit and dense K."""
    import workloads as W
    from oracle.mesh import RWGMesh
    from oracle.circuit import Circuit
    from oracle import integrals
    s = W.config1_bar()
    m = RWGMesh(s.V, s.T)
    c = Circuit(m, s.ports)
    K = integrals.kernel_dense(m)
    return dict(s=s, mesh=m, circ=c, K=K)
