"""GPU parity on the edge and degenerate cases of the method (through the C ABI, vs the oracle).

Empty basis or auxiliary sets, single functions, the highest supported quantum numbers (l = 6,
n = 12), one and sixteen Gauss-Legendre points per cell axis, the largest third-centre split, a third
centre on the pair axis (frame fallback, no azimuth reference), a third centre beyond the last mu
line (nothing moves), and exact distance ties in the routing (equilateral triangle)."""
import sys

import numpy as np
import pytest

import oracle as O
from conftest import MiniJob, Spec
from paper_2510_15204_amd import psint

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
KINDS = ("S", "T", "V", "PQ", "abP")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = psint.Context(0)
    yield c
    c.close()


def _check(ctx, job, label, scale_rel=False):
    got, st, rc = ctx.compute(job)
    ref = O.compute_full(job)
    assert rc == ref["status"], (label, rc, ref["status"])
    worst = {}
    for k in KINDS:
        assert got[k].shape == ref[k].shape, (label, k)
        d = float(np.max(np.abs(got[k] - ref[k]))) if ref[k].size else 0.0
        tol = TOL64 * (max(1.0, float(np.max(np.abs(ref[k])))) if scale_rel and ref[k].size else 1.0)
        worst[k] = d
        assert d <= tol, (label, k, d)
    _say(f"{label}: " + ", ".join(f"{k}={v:.1e}" for k, v in worst.items()))
    assert st["pair_points"] == ref["pair_points"]
    return got, ref


H2 = np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]])
TRI = np.array([[0.0, 0.0, 0.0], [1.4186, 0.0, 1.1082], [-1.4186, 0.0, 1.1082]])


def test_no_auxiliary_functions(ctx):
    basis = [[0, 1, 0, 0, 1.2], [1, 2, 1, 0, 0.9], [0, 2, 1, 1, 1.1]]
    got, _ = _check(ctx, MiniJob(TRI, [8, 1, 1], basis, np.zeros((0, 5)), Spec(5, 5, 4)), "no aux")
    assert got["PQ"].shape == (0, 0) and got["abP"].shape == (0, 3, 3)


def test_no_basis_functions(ctx):
    aux = [[0, 1, 0, 0, 2.0], [1, 2, 1, -1, 1.6], [2, 3, 2, 2, 2.2]]
    got, _ = _check(ctx, MiniJob(TRI, [8, 1, 1], np.zeros((0, 5)), aux, Spec(5, 5, 4)), "no basis")
    assert got["S"].shape == (0, 0) and got["abP"].shape == (3, 0, 0)


def test_single_function_each(ctx):
    _check(ctx, MiniJob(H2, [1, 1], [[1, 1, 0, 0, 1.0]], [[0, 1, 0, 0, 2.0]], Spec(6, 6, 4)), "one each")


def test_highest_quantum_numbers(ctx):
    """l = 6 and n = 12 (the largest the kernels support) on both sides of a diatomic; values of such
    functions reach a few hundred, so the bar is 1e-10 relative to each type's largest element."""
    basis = [[0, 7, 6, 6, 2.5], [0, 7, 6, -3, 2.5], [1, 12, 6, 0, 4.0], [1, 12, 0, 0, 5.0], [0, 1, 0, 0, 1.0]]
    aux = [[0, 7, 6, -6, 3.0], [1, 12, 5, 2, 6.0], [1, 1, 0, 0, 2.0]]
    _check(ctx, MiniJob(H2, [1, 1], basis, aux, Spec(10, 10, 8)), "l=6, n=12", scale_rel=True)


@pytest.mark.parametrize("q", [1, 16])
def test_extreme_points_per_cell(ctx, q):
    basis = [[0, 1, 0, 0, 1.3], [1, 2, 1, 1, 1.0], [2, 3, 2, -1, 0.9]]
    aux = [[0, 1, 0, 0, 2.6], [2, 2, 1, 0, 2.0]]
    spec = Spec(4, 3, 3, q, 2) if q == 16 else Spec(8, 8, 6, q, 3)
    _check(ctx, MiniJob(TRI, [8, 1, 1], basis, aux, spec), f"Q={q}")


def test_largest_third_centre_split(ctx):
    basis = [[0, 1, 0, 0, 1.3], [1, 2, 1, 1, 1.0], [2, 1, 0, 0, 1.1]]
    aux = [[0, 1, 0, 0, 2.6], [2, 2, 1, 0, 2.0]]
    _check(ctx, MiniJob(TRI, [8, 1, 1], basis, aux, Spec(6, 6, 4, 3, 8)), "N_SP=8")


def test_third_centre_on_the_pair_axis(ctx):
    """C on the line through A and B: its azimuth is undefined, the frame falls back to the global axis
    rule and only mu (nu = 0 or pi is a fixed line) can move."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.6], [0.0, 0.0, 3.5]])
    basis = [[0, 1, 0, 0, 1.2], [1, 2, 1, 0, 1.0], [2, 2, 1, 1, 0.9]]
    aux = [[0, 1, 0, 0, 2.4], [1, 1, 0, 0, 2.0], [2, 2, 1, -1, 1.8]]
    _check(ctx, MiniJob(xyz, [6, 1, 8], basis, aux, Spec(6, 6, 4)), "collinear")


def test_third_centre_beyond_the_grid(ctx):
    """C far outside the last mu line of the A-B grid: nothing moves or splits there."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.4], [60.0, 5.0, 0.0]])
    basis = [[0, 1, 0, 0, 1.2], [1, 1, 0, 0, 1.0], [2, 1, 0, 0, 1.5]]
    aux = [[0, 1, 0, 0, 2.4], [1, 1, 0, 0, 2.0], [2, 1, 0, 0, 3.0]]
    _check(ctx, MiniJob(xyz, [1, 1, 1], basis, aux, Spec(5, 5, 4)), "far third centre")


def test_equilateral_ties(ctx):
    """All distances equal: nearest atom and nearest-to-midpoint ties resolve to the lowest index on
    both sides."""
    s3 = np.sqrt(3.0)
    xyz = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [1.0, s3, 0.0]])
    basis = [[a, 1, 0, 0, 1.1] for a in range(3)] + [[a, 2, 1, 0, 0.9] for a in range(3)]
    aux = [[a, 1, 0, 0, 2.2] for a in range(3)]
    _check(ctx, MiniJob(xyz, [1, 1, 1], basis, aux, Spec(5, 5, 4)), "equilateral")
