"""GPU: grid-accuracy (eq. 13, Figs. 3-5) and geometry-scan (Fig. 6) harnesses against the oracle and
an independent axial quadrature."""
import sys

import numpy as np
import pytest

import oracle as O
from axial_reference import Fn, integral as axial_integral
from conftest import MiniJob, Spec
from paper_2510_15204_amd import accuracy as A
from paper_2510_15204_amd import psint
from paper_2510_15204_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = psint.Context(0)
    yield c
    c.close()


def _small(Z, xyz):
    rng = W.rng_for(1)
    basis, aux = W.build_basis(rng, np.asarray(Z, dtype=int), "DZ", "auxDZ", n_max=3)
    return W.Job("small", np.asarray(xyz, dtype=float), np.asarray(Z, dtype=float), basis, aux, W.GridSpec(6, 6, 4, 4, 3))


def _oracle_rmse(job, specs, reference):
    ref = O.compute_full(A._with_spec(job, reference))
    rows = []
    for s in specs:
        out = O.compute_full(A._with_spec(job, s))
        rows.append({t: A.rmse(ref[k], out[k]) for t, k in A.TYPES.items()})
    return rows


def test_grid_ladder_matches_oracle():
    """ClF-shaped diatomic, DZ-sized bases: the RMSE table of the GPU ladder equals the oracle's (both
    are the same quadrature; the tables differ by rounding) and falls along the ladder."""
    job = _small([17, 9], W.clf_tz().xyz)
    specs, ref = [(6, 6, 4), (8, 8, 5), (10, 10, 6)], (16, 16, 10, 4, 3)
    c = psint.Context(0)
    got = A.grid_ladder(c, job, specs, ref)
    c.close()
    orc = _oracle_rmse(job, specs, ref)
    for row, o in zip(got["rows"], orc):
        _say(f"{row['spec']}: " + ", ".join(f"{t} {row['rmse'][t]:.3e}/{o[t]:.3e}" for t in A.TYPES))
        for t in A.TYPES:
            assert abs(row["rmse"][t] - o[t]) <= 1e-11 + 1e-6 * o[t], t
    for t in A.TYPES:
        seq = [r["rmse"][t] for r in got["rows"]]
        assert seq[-1] < seq[0], t


def test_nsp_sweep_matches_oracle():
    """OF2-shaped triatomic: RMSE of V against a finer grid for N_SP = 1, 2, 3, GPU vs oracle."""
    job = _small([8, 9, 9], W.of2_tz().xyz)
    specs, ref = [(6, 6, 4), (8, 8, 4)], (14, 14, 8, 4, 3)
    c = psint.Context(0)
    got = A.nsp_sweep(c, job, specs, nsps=(1, 2, 3), reference=ref)
    c.close()
    orc_ref = O.compute_full(A._with_spec(job, ref))
    for nsp in (1, 2, 3):
        for s, e in zip(specs, got["rmse_V"][nsp]):
            o = A.rmse(orc_ref["V"], O.compute_full(A._with_spec(job, (s[0], s[1], s[2], 4, nsp)))["V"])
            _say(f"N_SP={nsp} {s}: {e:.3e} / oracle {o:.3e}")
            assert abs(e - o) <= 1e-11 + 1e-6 * o


def test_geometry_scan_parity_symmetry_and_axial_reference(ctx):
    """16-direction scan of six (P|Q) profiles through the serving path: (a) sampled points equal the
    oracle, (b) antipodal directions give (-1)^(l1+l2) times the value, (c) along +z the values
    equal an independent adaptive quadrature (relative 2e-8), (d) the scan on a coarse grid stays close to the same
    scan on a finer one (no grid artifacts along the paths)."""
    dist = [1.0, 2.0, 3.5, 5.0, 6.0]
    spec, fine = (24, 24, 14, 4, 3), (40, 40, 24, 4, 3)
    scan = A.geometry_scan(ctx, dist, spec=spec)
    ref = A.geometry_scan(ctx, dist, spec=fine)
    v, dirs = scan["values"], scan["directions"]
    assert v.shape == (16, len(dist), len(A.SCAN_PAIRS)) and scan["jobs"] == 16 * len(dist)
    # (a) oracle at a few (direction, distance) samples
    for di, ri in [(0, 0), (7, 2), (15, 4), (4, 3)]:
        o = O.compute_full(A.scan_job(dirs[di], dist[ri], spec), want=("PQ",))
        assert np.max(np.abs(A.scan_values(o["PQ"]) - v[di, ri])) < 1e-10
    # (b) inversion: Y_l0(-r) = (-1)^l Y_l0(r)
    sign = np.array([(-1) ** (l1 + l2) for l1, l2 in A.SCAN_PAIRS])
    for i in range(16):
        for j in range(16):
            if np.allclose(dirs[i], -dirs[j]):
                assert np.max(np.abs(v[i] - sign * v[j])) < 1e-11
    # (c) +z: centre 1 at (0, 0, R) is the axial helper's centre A, the origin its centre B
    zi = 4
    assert np.allclose(dirs[zi], [0, 0, 1])
    for ri in (1, 3):
        R = dist[ri]
        for k, (l1, l2) in enumerate(A.SCAN_PAIRS[:3]):
            exact = axial_integral([Fn("B", l1 + 1, l1, 0, 1.0, "pot"), Fn("A", l2 + 1, l2, 0, 1.0, "chi")], R / 2)
            _say(f"+z R={R} (l1,l2)=({l1},{l2}): {v[zi, ri, k]:.12f} exact {exact:.12f}")
            assert abs(v[zi, ri, k] - exact) < 2e-8 * abs(exact) + 1e-9
    # (d) against the finer grid along every path (measured: at most 1e-3 of a pair's scale, at the
    # shortest distance where the two unit-exponent functions overlap most)
    dev = A.scan_deviation(v, ref["values"])
    _say(f"scan deviation vs finer grid per pair: {np.array2string(dev.max(axis=0), precision=2)}; "
         f"{scan['jobs']} jobs in {scan['wall_s']:.2f} s")
    assert dev.max() < 5e-3
