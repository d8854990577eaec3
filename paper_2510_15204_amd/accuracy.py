"""Grid-accuracy and geometry-scan harnesses (Section 3; eq. 13; Figs. 3-6 and S1; Table S3).

All integrals come from the library (libpsint through the C ABI); this module only chooses the
jobs, collects the outputs and reduces them.

* ``grid_ladder``  RMSE (eq. 13) of each integral type of a job on a sequence of grids against a
  large reference grid (Figs. 3-4; ladder of Table S3, left; reference 80 x 70 x 50 cells, Q = 4,
  N_SP = 3 as in Section 3).
* ``nsp_sweep``    RMSE of the nuclear-attraction matrix for N_SP = 1..4 along a ladder (Fig. 5,
  Table S3 right; the stretched-bond geometry of Fig. S1).
* ``geometry_scan``  two-centre Coulomb integrals between m = 0, zeta = 1 Slater functions as the
  second centre moves out along 16 directions (Fig. 6), run as one batch of jobs through the
  serving path; ``scan_deviation`` compares a scan with the same scan on a finer grid.

Integral types: overlap S, kinetic T, nuclear attraction V, two-centre Coulomb (P|Q) and
three-centre Coulomb (ab|P).  RMSE runs over every element of the matrix of a type.
"""
from __future__ import annotations

import time
from typing import Dict, Iterable, Sequence

import numpy as np

from . import psint
from .workloads import GridSpec, Job

# Table S3, left: N_mu, N_nu, N_phi (Figs. 3-4); the paper combines each radial size with each
# angular pair, the default ladder here walks the diagonal.
LADDER_S3 = [(26 + i, 20 + 2 * i, 8 + i) for i in range(12)]
# Table S3, right: the N_SP study (Fig. 5)
NSP_LADDER_S3 = [(13 + i, 20 + 2 * (i // 2), 8 + i // 2) for i in range(26)]
# the large reference grid of Section 3 (Table 1, Fig. 6)
REFERENCE = (80, 70, 50, 4, 3)

TYPES = {"overlap": "S", "kinetic": "T", "nuclear": "V", "coulomb2": "PQ", "coulomb3": "abP"}


def rmse(ref: np.ndarray, got: np.ndarray) -> float:
    """Root-mean-square error over all elements (eq. 13)."""
    ref = np.asarray(ref, dtype=np.float64).ravel()
    got = np.asarray(got, dtype=np.float64).ravel()
    return float(np.sqrt(np.mean((ref - got) ** 2)))


def _with_spec(job: Job, spec: Sequence) -> Job:
    t = tuple(spec)
    g = GridSpec(*t) if len(t) >= 5 else GridSpec(t[0], t[1], t[2], 4, 3)
    return Job(job.name, job.xyz, job.Z, job.basis, job.aux, g, {}, job.precision)


def _run(ctx: psint.Context, job: Job, precision: str):
    t0 = time.perf_counter()
    out, st, rc = ctx.compute(job, outputs=tuple(TYPES.values()), precision=precision)
    return out, st, (time.perf_counter() - t0) * 1e3


def grid_ladder(ctx: psint.Context, job: Job, specs: Iterable[Sequence], reference: Sequence = REFERENCE,
                precision: str = "fp64", types: Iterable[str] = tuple(TYPES)) -> Dict:
    """RMSE of each integral type on every grid of `specs` against the `reference` grid."""
    ref, st_ref, ms_ref = _run(ctx, _with_spec(job, reference), "fp64")
    rows = []
    for spec in specs:
        out, st, ms = _run(ctx, _with_spec(job, spec), precision)
        rows.append({"spec": list(spec), "points": int(st["n_points"]), "ms": ms,
                     "rmse": {t: rmse(ref[TYPES[t]], out[TYPES[t]]) for t in types}})
    return {"job": job.name, "reference": list(reference), "reference_points": int(st_ref["n_points"]),
            "reference_ms": ms_ref, "precision": precision, "rows": rows}


def nsp_sweep(ctx: psint.Context, job: Job, specs: Iterable[Sequence], nsps: Iterable[int] = (1, 2, 3, 4),
              reference: Sequence = REFERENCE, q: int = 4) -> Dict:
    """RMSE of the nuclear-attraction matrix V for each third-centre split N_SP along `specs`."""
    ref, _, _ = _run(ctx, _with_spec(job, reference), "fp64")
    table = {}
    for nsp in nsps:
        errs = []
        for spec in specs:
            out, _, _ = _run(ctx, _with_spec(job, (spec[0], spec[1], spec[2], q, nsp)), "fp64")
            errs.append(rmse(ref["V"], out["V"]))
        table[int(nsp)] = errs
    return {"job": job.name, "reference": list(reference), "specs": [list(s) for s in specs], "rmse_V": table}


# --------------------------------------------------------------------------------------------
# Geometry scan (Fig. 6)
# --------------------------------------------------------------------------------------------

def scan_directions() -> np.ndarray:
    """16 unit vectors: the 6 axis directions, the 8 cube diagonals and 2 generic directions."""
    d = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    d += [(sx, sy, sz) for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]
    d += [(1, 2, 3), (-3, 1, 2)]
    v = np.array(d, dtype=np.float64)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# (l on the fixed centre, l on the moving centre): the six profiles, up to an f-h pair
SCAN_PAIRS = [(0, 0), (1, 1), (2, 2), (0, 3), (2, 4), (3, 5)]


def scan_job(direction: Sequence[float], R: float, spec: Sequence = REFERENCE, pairs=SCAN_PAIRS) -> Job:
    """Two centres, the origin and R * direction; auxiliary functions n = l + 1, m = 0, zeta = 1 for
    every l in `pairs` on both; one 1s basis function per centre (the scan reads only (P|Q))."""
    ls = sorted({l for p in pairs for l in p})
    xyz = np.array([[0.0, 0.0, 0.0], list(R * np.asarray(direction, dtype=np.float64))])
    basis = np.array([[0, 1, 0, 0, 1.0], [1, 1, 0, 0, 1.0]])
    aux = np.array([[a, l + 1, l, 0, 1.0] for a in range(2) for l in ls])
    t = tuple(spec)
    return Job(f"scan_R{R:.3f}", xyz, np.array([1.0, 1.0]), basis, aux, GridSpec(*t))


def scan_values(out_pq: np.ndarray, pairs=SCAN_PAIRS) -> np.ndarray:
    """(P|Q) with P = (l1, fixed centre), Q = (l2, moving centre) for each pair."""
    ls = sorted({l for p in pairs for l in p})
    n = len(ls)
    return np.array([out_pq[ls.index(l1), n + ls.index(l2)] for l1, l2 in pairs])


def geometry_scan(ctx: psint.Context, distances: Sequence[float], directions=None, spec: Sequence = REFERENCE,
                  pairs=SCAN_PAIRS, precision: str = "fp64") -> Dict:
    """Submit every (direction, distance) job at once (continuous batching) and collect the scan
    values[direction][distance][pair]."""
    directions = scan_directions() if directions is None else np.asarray(directions, dtype=np.float64)
    t0 = time.perf_counter()
    handles = []
    for d in directions:
        for R in distances:
            handles.append(ctx.submit(scan_job(d, R, spec, pairs), outputs=("PQ",), precision=precision))
    vals = np.empty((len(directions), len(distances), len(pairs)))
    pp = 0.0
    for i, h in enumerate(handles):
        out, st, _ = ctx.wait(h)
        vals[i // len(distances), i % len(distances)] = scan_values(out["PQ"], pairs)
        pp += st["pair_points"]
    wall = time.perf_counter() - t0
    return {"directions": directions, "distances": np.asarray(distances, dtype=np.float64), "pairs": pairs,
            "values": vals, "jobs": len(handles), "wall_s": wall, "pair_points": pp}


def scan_deviation(values: np.ndarray, reference: np.ndarray) -> np.ndarray:
    """Largest |value - reference| along each path (per direction and pair), relative to the pair's
    largest reference magnitude over all paths (a profile that vanishes by symmetry along some
    direction is measured on the same scale as the others).  A grid artifact at any point of a path
    (a kink or jump, Fig. 6) shows up here, since the reference grid is many times finer."""
    values = np.asarray(values, dtype=np.float64)
    reference = np.asarray(reference, dtype=np.float64)
    scale = np.maximum(np.max(np.abs(reference), axis=(0, 1)), 1e-300)
    return np.max(np.abs(values - reference), axis=1) / scale
