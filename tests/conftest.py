import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def cd():
    """The ctypes binding of libchebdav.so (built in-tree if missing)."""
    from paper_2212_04443_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2212_04443_amd import build as b
        b.build()
    from paper_2212_04443_amd import chebdav
    return chebdav


@pytest.fixture(scope="session")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return torch.device("cuda:0")


def sin_max_angle(Q1, Q2):
    """sin of the largest principal angle of span(Q2) to span(Q1) (both orthonormal)."""
    import numpy as np
    return float(np.linalg.norm(Q2 - Q1 @ (Q1.T @ Q2), 2))
