"""CPU: invariants of the contraction plan (csrc/plan.cpp, built here with g++ into
tests/plan_check.cpp) on the benchmark workloads and under a small memory budget: every output
element of every task is covered by exactly one reduction item, each item's K splits tile its grid's
point chunks in order and evenly, every tile sits in a launch whose shape holds it, and the issued
FLOPs add up, and every pass's arrays and partial tiles lie in its own region (disjoint from the next
pass's when passes overlap); with cross-third-centre reuse, the shared segments and the cells their
members skip."""
import os
import subprocess

import pytest

from paper_2510_15204_amd import workloads as W
import tile_shape_jobs as TS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan_check")
    exe = str(d / "plan_check")
    csrc = os.path.join(ROOT, "paper_2510_15204_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", csrc, os.path.join(ROOT, "tests", "plan_check.cpp"),
                    os.path.join(csrc, "plan.cpp"), "-o", exe], check=True)
    return exe, d


def _write_job(job, path):
    lines = [str(len(job.xyz))]
    lines += [" ".join(repr(float(v)) for v in (*x, z)) for x, z in zip(job.xyz, job.Z)]
    for fns in (job.basis, job.aux):
        lines.append(str(len(fns)))
        lines += [f"{int(r[0])} {int(r[1])} {int(r[2])} {int(r[3])} {float(r[4])!r}" for r in fns]
    lines.append(" ".join(str(v) for v in job.grid.as_tuple()))
    lines.append(str(len(job.pair_grids)))
    lines += [f"{a} {b} " + " ".join(str(v) for v in s.as_tuple()) for (a, b), s in job.pair_grids.items()]
    path.write_text("\n".join(lines) + "\n")


@pytest.mark.parametrize("name,prec,budget_gb,share", [
    ("diatomic_small", 0, 200.0, ""),
    ("triatomic_qz", 0, 200.0, ""),
    ("triatomic_qz", 1, 200.0, ""),
    ("triatomic_qz", 0, 7.0, ""),       # one grid per memory pass, small workspace reservations
    ("hydrocarbon9", 0, 246.0, ""),     # 252 uneven grids, three passes
    ("hydrocarbon9", 1, 246.0, ""),
    ("hydrocarbon9", 0, 246.0, "share"),  # cross-third-centre reuse: shared segments, skip masks
    ("hydrocarbon9", 1, 246.0, "share"),
    ("hydrocarbon9", 0, 40.0, "share"),   # many passes: shares split by a pass boundary are dropped
    ("hydrocarbon9", 0, 246.0, "share,overlap"),  # overlapped passes: alternating disjoint regions
    ("hydrocarbon9", 1, 246.0, "overlap"),
    ("triatomic_qz", 0, 10.0, "overlap"),
    ("triatomic_qz", 0, 200.0, "overlap"),  # one pass: nothing to overlap
])
def test_plan_invariants(checker, name, prec, budget_gb, share):
    exe, d = checker
    job = getattr(W, name)()
    f = d / f"{name}.txt"
    _write_job(job, f)
    args = [exe, str(f), str(prec), "512", str(budget_gb)] + ([share] if share else [])
    out = subprocess.run(args, capture_output=True, text=True, timeout=300)
    print(out.stdout.strip())
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
    if "overlap" in share:
        assert ("overlapped" in out.stdout) == (budget_gb < 200.0 or name == "hydrocarbon9"), out.stdout


@pytest.mark.parametrize("n_aux", sorted(TS.TALL_CASES))
def test_tall_and_short_row_shapes_are_planned(checker, n_aux):
    """The GPU parity jobs of tests/tile_shape_jobs.py keep exercising what they are for: the 128-row
    shape, the tall last-column shape of their auxiliary count and a 32-row short row tile."""
    exe, d = checker
    f = d / f"tall_{n_aux}.txt"
    _write_job(TS.tall_job(n_aux), f)
    out = subprocess.run([exe, str(f), "0", "512", "200"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout
    shapes = out.stdout.split("shapes")[1].split()
    assert TS.TALL_CASES[n_aux] in shapes and any(s.startswith("1.") for s in shapes), shapes
    assert "merged" in shapes, shapes  # the 128-row shapes share one launch
