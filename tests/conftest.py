import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


class Spec:
    """Minimal grid spec object for oracle-only tests."""

    def __init__(self, n_mu, n_nu, n_phi, q=4, n_sp=3, c1_scale=2.3, c1_exp=0.25):
        self.t = (n_mu, n_nu, n_phi, q, n_sp, c1_scale, c1_exp)

    def as_tuple(self):
        return self.t


class MiniJob:
    def __init__(self, xyz, Z, basis, aux, spec, pair_grids=None):
        import numpy as np
        self.xyz = np.asarray(xyz, dtype=float)
        self.Z = np.asarray(Z, dtype=float)
        self.basis = np.asarray(basis, dtype=float).reshape(-1, 5)
        self.aux = np.asarray(aux, dtype=float).reshape(-1, 5)
        self.grid = spec
        self.pair_grids = pair_grids or {}


@pytest.fixture
def Spec_():
    return Spec


@pytest.fixture
def MiniJob_():
    return MiniJob
