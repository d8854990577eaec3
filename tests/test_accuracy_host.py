"""Host logic of the grid-accuracy and geometry-scan harnesses (no GPU)."""
import json
import os

import numpy as np

from paper_2510_15204_amd import accuracy as A
from paper_2510_15204_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table_s3.json")


def test_ladders_are_table_s3():
    g = json.load(open(GOLDEN))
    assert [list(x) for x in A.LADDER_S3] == g["left"]
    assert [list(x) for x in A.NSP_LADDER_S3] == g["right"]
    assert list(A.REFERENCE) == g["reference"]


def test_rmse_is_eq13_by_brute_force():
    rng = np.random.default_rng(0)
    a, b = rng.normal(size=(7, 5)), rng.normal(size=(7, 5))
    s = 0.0
    for x, y in zip(a.ravel(), b.ravel()):
        s += (x - y) ** 2
    assert abs(A.rmse(a, b) - (s / a.size) ** 0.5) < 1e-15
    assert A.rmse(a, a) == 0.0


def test_scan_directions():
    d = A.scan_directions()
    assert d.shape == (16, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    assert len({tuple(np.round(v, 12)) for v in d}) == 16
    # 14 of them come in antipodal pairs (used by the parity check of the scan)
    anti = sum(any(np.allclose(v, -w) for w in d) for v in d)
    assert anti == 14


def test_scan_job_and_value_selection():
    job = A.scan_job([0.0, 0.0, 1.0], 2.5, (6, 6, 4, 4, 3))
    assert np.allclose(job.xyz[1], [0.0, 0.0, 2.5])
    ls = sorted({l for p in A.SCAN_PAIRS for l in p})
    assert job.n_aux == 2 * len(ls)
    assert all(row[3] == 0 and row[4] == 1.0 and row[1] == row[2] + 1 for row in job.aux)
    n = len(ls)
    PQ = np.arange(4 * n * n, dtype=float).reshape(2 * n, 2 * n)
    vals = A.scan_values(PQ)
    for (l1, l2), v in zip(A.SCAN_PAIRS, vals):
        assert v == PQ[ls.index(l1), n + ls.index(l2)]
        assert job.aux[ls.index(l1)][0] == 0 and job.aux[n + ls.index(l2)][0] == 1


def test_scan_deviation_is_relative_per_pair():
    ref = np.ones((3, 5, 2))
    ref[1, :, 0] = 10.0
    got = ref.copy()
    got[1, 2, 0] += 0.5
    got[2, 4, 1] -= 0.25
    dev = A.scan_deviation(got, ref)
    assert dev.shape == (3, 2)
    assert dev[1, 0] == 0.05 and dev[2, 1] == 0.25 and dev[0, 0] == 0.0
    ref[0, :, 1] = 0.0  # a profile that vanishes by symmetry: measured on its pair's scale
    got = ref.copy()
    got[0, 1, 1] = 1e-3
    assert A.scan_deviation(got, ref)[0, 1] == 1e-3


def test_molecule_shapes():
    clf = W.clf_tz()
    assert clf.n_atoms == 2 and abs(np.linalg.norm(clf.xyz[1] - clf.xyz[0]) - 1.628 * W.BOHR_PER_ANGSTROM) < 1e-12
    of2 = W.of2_tz()
    r1, r2 = np.linalg.norm(of2.xyz[1]), np.linalg.norm(of2.xyz[2])
    ang = np.degrees(np.arccos(of2.xyz[1] @ of2.xyz[2] / (r1 * r2)))
    assert abs(r1 - 1.405 * W.BOHR_PER_ANGSTROM) < 1e-12 and abs(ang - 103.1) < 1e-9
    lb = W.of2_tz(long_bond=True)
    assert abs(np.linalg.norm(lb.xyz[1]) - 41.41 * W.BOHR_PER_ANGSTROM) < 1e-9
    assert clf.n_bf == 50 and clf.n_aux == 150 and of2.n_bf == 75
