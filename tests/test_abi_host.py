"""Host-side checks of the C-ABI library (no GPU): it loads, exports every symbol the header
declares, and its planner's routing gives the same pair-point work as the oracle's."""
import os
import re

import numpy as np
import pytest

import oracle as O
from conftest import MiniJob, Spec
from paper_2510_15204_amd import psint
from paper_2510_15204_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "psint.h")).read()
    return sorted(set(re.findall(r"\b(ps_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = psint.lib()
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(psint.exported_symbols()) <= set(names)


def test_status_strings():
    L = psint.lib()
    for code in range(0, -9, -1):
        assert L.ps_status_string(code)


@pytest.mark.parametrize("make", ["diatomic_small", "tri_small", "four_atoms"])
def test_planner_work_matches_oracle_routing(make):
    """The pair-point count sums, over output elements, the points of each distinct grid the element is
    routed to; both sides route independently (3-atom-subset reading), so equal counts pin the routing."""
    if make == "diatomic_small":
        job = W.diatomic_small()
    elif make == "tri_small":
        rng = W.rng_for(1)
        Z = np.array([8.0, 1.0, 1.0])
        basis, aux = W.build_basis(rng, Z.astype(int), "DZ", "auxDZ", n_max=4)
        job = MiniJob(W.triatomic_geometry(), Z, basis, aux, Spec(3, 3, 2, 2, 2))
    else:
        xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.2, 0.0], [-0.4, 1.8, 0.3], [0.6, -0.5, 2.0]])
        basis = [[a, 1, 0, 0, 1.0 + a] for a in range(4)] + [[0, 2, 1, 1, 1.5]]
        aux = [[a, 1, 0, 0, 2.0 + a] for a in range(4)] + [[2, 2, 1, 0, 2.2]]
        job = MiniJob(xyz, [6, 1, 8, 1], basis, aux, Spec(3, 3, 2, 2, 2))
    got = psint.plan_work_host(job)
    ref = O.compute_full(job)
    assert got["pair_points"] == ref["pair_points"]
    assert got["n_grids"] == len(O.grid_list(job))


def test_planner_sizes_of_benchmark_workloads():
    r = psint.plan_work_host(W.triatomic_qz())
    assert r["n_grids"] == 3
    assert r["n_points"] == 3 * (24 * 24 * 12 + 8 * 26) * 64
    assert abs(r["pair_points"] / 1.086e12 - 1) < 0.01


def test_planner_rejects_invalid_job():
    job = MiniJob([[0, 0, 0], [0, 0, 1.0]], [1, 1], [[0, 1, 1, 0, 1.0]], [[0, 1, 0, 0, 1.0]], Spec(4, 4, 4))
    with pytest.raises(psint.PsError) as e:
        psint.plan_work_host(job)
    assert e.value.status == psint.PS_E_INVALID
