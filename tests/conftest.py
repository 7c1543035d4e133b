import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


# 4^4 workload of the small parity configuration: epsilon 0.3, seed 0, m_q = -0.2
CFG0_DIMS = (4, 4, 4, 4)
CFG0_EPS = 0.3
CFG0_SEED = 0
CFG0_MASS = -0.2


@pytest.fixture(scope="session")
def cfg0_field():
    from synthetic import gauge_field
    return gauge_field(CFG0_DIMS, CFG0_EPS, CFG0_SEED)


@pytest.fixture(scope="session")
def cfg0_op(cfg0_field):
    from oracle.dirac import WilsonOperator
    return WilsonOperator(cfg0_field, CFG0_MASS)


@pytest.fixture(scope="session")
def cfg0_dense(cfg0_op):
    """Dense A and M of the 4^4 operator plus the eigendecomposition of A."""
    from oracle.dense import dense_A
    A, M = dense_A(cfg0_op)
    lam, X = np.linalg.eigh(A)
    return {"A": A, "M": M, "lam": lam, "X": X}


@pytest.fixture(scope="session")
def cfg0_rhs():
    from synthetic import gaussian_rhs
    return gaussian_rhs(CFG0_DIMS, 1000).reshape(-1)
