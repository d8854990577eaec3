"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle, element by element.

FP64 path bar: 1e-10 absolute on every element (both sides compute the same quadrature; only the
rounding order and the evaluation formulas differ).
"""
import math
import sys

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle as O
from conftest import MiniJob, Spec
from paper_2510_15204_amd import psint
from paper_2510_15204_amd import workloads as W
import tile_shape_jobs as TS

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = psint.Context(0)
    yield c
    c.close()


def _compare(got, ref, tol, label):
    worst = {}
    for k in ("S", "T", "V", "PQ", "abP"):
        d = np.max(np.abs(got[k] - ref[k])) if ref[k].size else 0.0
        worst[k] = d
    _say(f"{label}: max abs diff " + ", ".join(f"{k}={v:.2e}" for k, v in worst.items()))
    for k, v in worst.items():
        assert v <= tol, (label, k, v)


# ---------------------------------------------------------------------------------------------
# Grid points and weights
# ---------------------------------------------------------------------------------------------

TRI = W.triatomic_geometry()


@pytest.mark.parametrize("A,B,C,spec", [
    (0, 1, -1, (5, 4, 3, 4, 3, 2.3, 0.25)),
    (0, 1, 2, (6, 5, 4, 3, 3, 2.3, 0.25)),
    (1, 2, 0, (7, 6, 5, 2, 2, 2.3, 0.25)),
    (0, 2, 1, (4, 4, 2, 5, 4, 2.3, 0.25)),
])
def test_grid_points_match_oracle(ctx, A, B, C, spec):
    _say(f"grid points A={A} B={B} C={C} spec={spec}")
    g = ctx.grid_points(TRI, A, B, C, Spec(*spec))
    x, y, z, w = O.grid_points(TRI, A, B, C, spec)
    assert g.shape[0] == x.size
    tree = cKDTree(np.stack([x, y, z], 1))
    d, idx = tree.query(g[:, :3])
    assert np.max(d) < 1e-12
    assert len(set(idx.tolist())) == x.size  # a bijection
    assert np.max(np.abs(g[:, 3] - w[idx]) / w[idx]) < 1e-12


# ---------------------------------------------------------------------------------------------
# Function values: chi, -1/2 lap chi, aux potential
# ---------------------------------------------------------------------------------------------

FUNCS = [(1, 0, 0, 1.3), (2, 1, -1, 0.7), (2, 1, 1, 2.5), (3, 2, 0, 1.1), (4, 3, -2, 1.9), (5, 4, 3, 0.9),
         (6, 5, -5, 1.5), (7, 6, 6, 2.2), (7, 6, -1, 0.6), (12, 3, 1, 1.4), (4, 0, 0, 3.5)]


@pytest.mark.parametrize("what", ["chi", "kin", "pot"])
def test_eval_function_matches_oracle(ctx, what):
    rng = np.random.default_rng(11)
    pts = rng.normal(size=(500, 3)) * rng.uniform(0.01, 6.0, size=(500, 1))
    center = np.array([0.3, -0.2, 0.1])
    for (n, l, m, z) in FUNCS:
        fn = [0, n, l, m, z]
        got = ctx.eval_function(what, fn, center, pts[:, 0] + center[0], pts[:, 1] + center[1],
                                pts[:, 2] + center[2])
        ref = O.eval_fn(what, fn, center, pts[:, 0] + center[0], pts[:, 1] + center[1], pts[:, 2] + center[2])
        scale = np.max(np.abs(ref)) + 1e-300
        err = np.max(np.abs(got - ref)) / scale
        assert err < 1e-13, (what, n, l, m, z, err)


# ---------------------------------------------------------------------------------------------
# Whole jobs against the oracle
# ---------------------------------------------------------------------------------------------

def test_diatomic_small_full_parity(ctx):
    job = W.diatomic_small()
    _say(f"job {job.name}: n_bf={job.n_bf} n_aux={job.n_aux}")
    got, st, rc = ctx.compute(job)
    ref = O.compute_full(job)
    assert rc == ref["status"] == 0
    _compare(got, ref, TOL64, job.name)
    assert np.max(np.abs(got["PQ_chol"] - ref["PQ_chol"])) < 1e-9
    assert st["pair_points"] == ref["pair_points"]


def _tri_tz(spec=(6, 5, 4, 4, 3, 2.3, 0.25)):
    rng = W.rng_for(1)
    Z = np.array([8.0, 1.0, 1.0])
    basis, aux = W.build_basis(rng, Z.astype(int), "TZ", "auxTZ", n_max=4)
    return MiniJob(TRI, Z, basis, aux, Spec(*spec))


def test_triatomic_tz_full_parity_several_tiles(ctx):
    """43 basis / 129 aux functions: the O x H pair block (225 rows) spans two 128-row tiles and the
    129 aux columns two 128-column tiles (ragged tails in both)."""
    job = _tri_tz()
    _say(f"triatomic TZ: n_bf={len(job.basis)} n_aux={len(job.aux)}")
    got, st, rc = ctx.compute(job)
    ref = O.compute_full(job)
    assert rc == ref["status"]
    _compare(got, ref, TOL64, "triatomic TZ")
    assert st["pair_points"] == ref["pair_points"]


def test_four_atoms_pair_and_third_centre_grids(ctx):
    """N = 4: grids G(A,B|C) that are not pair grids carry only V(nucleus C) and (ab|P on C)."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.2, 0.0], [-0.4, 1.8, 0.3], [0.6, -0.5, 2.0]])
    Z = [6.0, 1.0, 8.0, 1.0]
    rng = np.random.default_rng(3)
    basis = [[0, 1, 0, 0, 4.0], [0, 2, 1, 1, 1.2], [0, 3, 2, -2, 1.1], [1, 1, 0, 0, 1.3], [1, 2, 1, 0, 0.9],
             [2, 2, 0, 0, 1.7], [2, 2, 1, -1, 1.4], [3, 1, 0, 0, 1.0]]
    aux = [[0, 1, 0, 0, 5.0], [0, 2, 1, 0, 2.2], [1, 1, 0, 0, 2.5], [2, 3, 2, 1, 2.9], [2, 1, 0, 0, 3.3],
           [3, 2, 1, 1, 2.0]]
    job = MiniJob(xyz, Z, basis, aux, Spec(5, 4, 3, 3, 2))
    got, st, rc = ctx.compute(job)
    ref = O.compute_full(job)
    _compare(got, ref, TOL64, "four atoms")
    assert st["n_grids"] == 12
    assert st["pair_points"] == ref["pair_points"]


def test_pair_grid_overrides_and_unsorted_functions(ctx):
    """Per-pair grid specs, functions listed out of atom order, an atom without aux functions."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 1.7, 0.5], [1.5, -0.3, 0.2]])
    basis = [[2, 1, 0, 0, 1.1], [0, 2, 1, -1, 1.3], [1, 3, 2, 2, 0.8], [0, 1, 0, 0, 3.1], [2, 2, 1, 1, 1.0],
             [1, 1, 0, 0, 1.2]]
    aux = [[1, 2, 1, 0, 2.4], [0, 1, 0, 0, 4.1], [1, 1, 0, 0, 2.0]]
    pg = {(0, 2): Spec(6, 4, 3, 3, 3), (1, 2): Spec(4, 5, 4, 2, 2)}
    job = MiniJob(xyz, [7.0, 1.0, 1.0], basis, aux, Spec(5, 5, 3, 3, 3), pg)
    got, st, rc = ctx.compute(job)
    ref = O.compute_full(job)
    _compare(got, ref, TOL64, "overrides")
    assert st["pair_points"] == ref["pair_points"]


def test_device_outputs_equal_host_outputs(ctx):
    job = _tri_tz((4, 4, 3, 3, 2, 2.3, 0.25))
    host, _, _ = ctx.compute(job)
    dev, _, _ = ctx.compute(job, device=True)
    for k in psint.OUTPUTS:
        assert np.array_equal(host[k], dev[k].cpu().numpy()), k


def test_not_positive_definite_metric_reported(ctx):
    xyz = np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]])
    job = MiniJob(xyz, [1, 1], [[0, 1, 0, 0, 1.0], [1, 1, 0, 0, 1.0]], [[0, 1, 0, 0, 2.0], [0, 1, 0, 0, 2.0]],
                  Spec(6, 6, 4))
    got, st, rc = ctx.compute(job)
    assert rc == psint.PS_E_NOT_PD
    ref = O.compute_full(job)
    assert ref["status"] == -5
    _compare(got, ref, TOL64, "not PD")


def test_repeated_not_positive_definite_job_factors_every_time():
    """A job whose metric is not positive definite only in its second 32-column panel (35 auxiliary
    functions, the last a copy of the first), run three times on one context (the repeats reuse its
    plan and replay captured graphs): each run reports NOT_PD after factoring the first panel, so
    that panel equals the oracle's factor of the leading 32 x 32 block every time (a status left
    set by an earlier run would skip the factorisation and leave (P|Q) itself there)."""
    xyz = np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]])
    aux = []
    for a in range(2):
        aux += [[a, 1, 0, 0, z] for z in (1.0, 3.0)]
        aux += [[a, 2, 1, m, 1.5] for m in (-1, 0, 1)]
        aux += [[a, 3, 2, m, 2.0] for m in range(-2, 3)]
        aux += [[a, 4, 3, m, 2.2] for m in range(-3, 4)]
    aux.append(list(aux[0]))
    assert len(aux) == 35
    job = MiniJob(xyz, [1, 1], [[0, 1, 0, 0, 1.0], [1, 1, 0, 0, 1.0]], aux, Spec(10, 10, 6))
    c = psint.Context(0)
    try:
        runs = [c.compute(job) for _ in range(3)]
    finally:
        c.close()
    PQ = runs[0][0]["PQ"]
    L32 = np.linalg.cholesky(PQ[:32, :32])
    for got, st, rc in runs:
        assert rc == psint.PS_E_NOT_PD
        assert np.max(np.abs(got["PQ_chol"][:32, :32] - L32)) < 1e-12 * np.max(np.abs(L32))
        assert np.array_equal(got["PQ_chol"], runs[0][0]["PQ_chol"])
    assert runs[2][1]["graph_replay"] == 1


def _five_atoms():
    """Five atoms off every pair axis (third centres refine every grid), Q = 4: each pair has two grids
    G(A,B|C) besides its pair grid, so cross-third-centre reuse forms a shared segment per atom."""
    xyz = np.array([[0.0, 0.0, 0.0], [2.1, 0.3, 0.2], [-0.6, 1.9, -0.4], [0.5, -0.9, 1.95], [1.6, 1.7, 1.5]])
    basis, aux = [], []
    for a in range(5):
        basis += [[a, 1, 0, 0, 2.4 - 0.2 * a], [a, 2, 0, 0, 0.9], [a, 2, 1, -1, 1.3], [a, 2, 1, 0, 1.3],
                  [a, 2, 1, 1, 1.3], [a, 3, 2, -2, 1.1], [a, 3, 2, 1, 1.1]]
        aux += [[a, 1, 0, 0, 3.0], [a, 2, 1, 0, 2.2], [a, 3, 2, 2, 2.0]]
    return MiniJob(xyz, [6.0, 1.0, 8.0, 1.0, 1.0], basis, aux, Spec(10, 10, 6, 4, 3))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_third_centre_reuse_matches_per_grid_evaluation_and_oracle(prec):
    """Cross-third-centre reuse (ps_set_option PS_OPT_SHARE_THIRD_CENTRE): the shared evaluation does
    the per-grid evaluation's arithmetic for the shared cells, so every output equals the job without
    reuse to rounding (1e-13 of each type's largest element; FP32 values of the mixed job are rounded
    from the same FP64 values), and the FP64 job equals the oracle to 1e-10."""
    job = _five_atoms()
    c = psint.Context(0)
    try:
        c.set_option(psint.PS_OPT_SHARE_THIRD_CENTRE, 0)
        off, _, rc_off = c.compute(job, precision=prec)
        c.set_option(psint.PS_OPT_SHARE_THIRD_CENTRE, 1)
        on, _, rc_on = c.compute(job, precision=prec)
        c.set_option(psint.PS_OPT_SHARE_THIRD_CENTRE, -1)  # automatic: on for FP64 jobs
        auto, _, _ = c.compute(job, precision=prec)
    finally:
        c.close()
    for k in psint.OUTPUTS:
        assert np.array_equal(auto[k], on[k] if prec == "fp64" else off[k]), k
    assert rc_on == rc_off
    for k in ("S", "T", "V", "PQ", "abP"):
        scale = max(1.0, float(np.max(np.abs(off[k]))))
        d = float(np.max(np.abs(on[k] - off[k])))
        _say(f"{prec} {k}: |shared - per grid| = {d:.2e}, identical {np.array_equal(on[k], off[k])}")
        assert d <= 1e-13 * scale, (k, d)
    if prec == "fp64":
        ref = O.compute_full(job)
        _compare(on, ref, TOL64, "five atoms, shared evaluation")


def test_set_option_rejects_unknown():
    c = psint.Context(0)
    try:
        with pytest.raises(psint.PsError) as e:
            c.set_option(99, 1)
        assert e.value.status == psint.PS_E_INVALID
        with pytest.raises(psint.PsError):
            c.set_option(psint.PS_OPT_SHARE_THIRD_CENTRE, 2)
        c.set_option(psint.PS_OPT_SHARE_THIRD_CENTRE, -1)
    finally:
        c.close()


@pytest.mark.parametrize("bad", ["l_ge_n", "neg_zeta", "atom_index", "coincident", "spec", "too_high_l"])
def test_invalid_inputs_rejected(ctx, bad):
    xyz = np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]])
    basis = [[0, 1, 0, 0, 1.0], [1, 2, 1, 0, 1.0]]
    aux = [[0, 1, 0, 0, 2.0]]
    spec = Spec(6, 6, 4)
    expect = psint.PS_E_INVALID
    if bad == "l_ge_n":
        basis[1] = [1, 2, 2, 0, 1.0]
    elif bad == "neg_zeta":
        basis[0] = [0, 1, 0, 0, -1.0]
    elif bad == "atom_index":
        aux[0] = [5, 1, 0, 0, 2.0]
    elif bad == "coincident":
        xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1e-5]])
    elif bad == "spec":
        spec = Spec(1, 6, 4)
    elif bad == "too_high_l":
        basis[1] = [1, 9, 7, 0, 1.0]
        expect = psint.PS_E_UNSUPPORTED
    job = MiniJob(xyz, [1, 1], basis, aux, spec)
    with pytest.raises(psint.PsError) as e:
        ctx.compute(job)
    assert e.value.status == expect


@pytest.mark.parametrize("n_aux", sorted(TS.TALL_CASES))
def test_tall_and_short_row_tiles_match_oracle(ctx, n_aux):
    """Jobs whose plans use the 4 x 1 wave arrangement (128 rows x 16, 48, 80 or 112 columns, one per
    case), the 128-row shape and the 32-row shapes for short row tiles (tests/tile_shape_jobs.py; the
    CPU plan test checks that they do): FP64 against the oracle at 1e-10, mixed with (ab|P) within
    1e-7 of its largest element and the FP64 two-index outputs at 1e-10.  The factor of (P|Q) is not
    asked for: the larger auxiliary sets make the metric ill-conditioned (smallest to largest
    eigenvalue down to 1e-13), which is not what these jobs test."""
    job = TS.tall_job(n_aux)
    outs = ("S", "T", "V", "PQ", "abP")
    ref = O.compute_full(job, want=outs)
    got, _, rc = ctx.compute(job, outputs=outs)
    assert rc == psint.PS_OK
    _compare(got, ref, TOL64, f"tall shapes, {n_aux} auxiliaries on C")
    mix, _, _ = ctx.compute(job, outputs=outs, precision="mixed")
    for k in ("S", "T", "V", "PQ", "abP"):
        tol = 1e-7 * float(np.max(np.abs(ref[k]))) if k == "abP" else TOL64
        assert np.max(np.abs(mix[k] - ref[k])) <= tol, (n_aux, k)


@pytest.mark.parametrize("tiling", [(4, 4, 2), (4, 4, 1), (4, 2, 1), (2, 4, 2)])
def test_explicit_tilings_match_oracle(tiling):
    """Non-default tilings (ps_set_tiling) on a job with 128-row, tall and short row tiles: the merged
    launch of the 128-row shapes with the other stage size in each precision (FP64 32-point stages,
    FP32 16-point stages), a narrower main shape, and a 64-row main shape (no merged launch); FP64
    against the oracle at 1e-10, mixed with (ab|P) within 1e-7 of its largest element."""
    job = TS.tall_job(138)
    outs = ("S", "T", "V", "PQ", "abP")
    ref = O.compute_full(job, want=outs)
    c = psint.Context(0)
    try:
        c.set_tiling(*tiling, 0)
        got, _, rc = c.compute(job, outputs=outs)
        assert rc == psint.PS_OK
        _compare(got, ref, TOL64, f"tiling {tiling}")
        mix, _, _ = c.compute(job, outputs=outs, precision="mixed")
    finally:
        c.close()
    for k in outs:
        tol = 1e-7 * float(np.max(np.abs(ref[k]))) if k == "abP" else TOL64
        assert np.max(np.abs(mix[k] - ref[k])) <= tol, (tiling, k)


@pytest.mark.parametrize("ksplit", [1, 3, 17])
def test_explicit_k_splits_match_oracle(ksplit):
    """The same job with every contraction item split into 1, 3 or 17 point ranges (partial tiles
    summed in split order by the reduction, which reads whole lines of 16 columns): FP64 and mixed
    results against the oracle, and the FP64 results of different split counts agree to rounding."""
    job = _tri_tz()
    ref = O.compute_full(job)
    c = psint.Context(0)
    c.set_tiling(0, 0, 0, ksplit)
    got, _, rc = c.compute(job)
    assert rc == ref["status"]
    _compare(got, ref, TOL64, f"ksplit={ksplit}")
    mix, _, _ = c.compute(job, precision="mixed")
    for k in ("S", "T", "V", "PQ", "abP"):
        # S, T, V, (P|Q) contracted in FP64 inside the mixed job; (ab|P) on FP32 operands
        tol = 1e-7 * float(np.max(np.abs(ref[k]))) if k == "abP" else TOL64
        assert np.max(np.abs(mix[k] - ref[k])) <= tol, (ksplit, k)
    c.close()
