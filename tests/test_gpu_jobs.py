"""GPU: full-size sampled parity, mixed precision error bars, serving (continuous batching)."""
import sys
import time

import numpy as np
import pytest

import oracle as O
from conftest import MiniJob, Spec
from paper_2510_15204_amd import psint
from paper_2510_15204_amd import workloads as W

pytestmark = pytest.mark.gpu

KINDS = ("S", "T", "V", "PQ", "abP")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = psint.Context(0)
    yield c
    c.close()


def sample(job, n_abp, seed):
    rng = np.random.default_rng(seed)
    nb, na = job.n_bf, job.n_aux
    kinds, I, J, K = [], [], [], []
    for kind in range(4):
        lim = na if kind == 3 else nb
        for _ in range(8):
            a, b = sorted(rng.integers(0, lim, size=2))
            kinds.append(kind); I.append(a); J.append(b); K.append(0)
    # always include a diagonal and the largest-index corner
    kinds += [4, 4]; I += [0, nb - 1]; J += [0, nb - 1]; K += [0, na - 1]
    for _ in range(n_abp):
        a, b = sorted(rng.integers(0, nb, size=2))
        kinds.append(4); I.append(a); J.append(b); K.append(int(rng.integers(0, na)))
    return np.array(kinds), np.array(I), np.array(J), np.array(K)


def pick(out, kinds, I, J, K):
    return np.array([out["abP"][p, a, b] if kd == 4 else out[KINDS[kd]][a, b]
                     for kd, a, b, p in zip(kinds, I, J, K)])


def test_benchmark_workload_sampled_parity(ctx):
    """The triatomic QZ job at full size (three refined 96x96x48-point grids), default tiling as the
    benchmark runs it, device outputs: sampled elements of every kind within 1e-10 of the oracle."""
    job = W.triatomic_qz()
    _say(f"{job.name}: n_bf={job.n_bf} n_aux={job.n_aux}")
    got, st, rc = ctx.compute(job, device=True)
    host = {k: v.cpu().numpy() for k, v in got.items()}
    kinds, I, J, K = sample(job, 150, 7)
    ref, _ = O.compute_elements(job, kinds, I, J, K)
    err = np.abs(pick(host, kinds, I, J, K) - ref)
    _say("max abs err per kind: " + ", ".join(f"{KINDS[k]}={err[kinds == k].max():.2e}" for k in range(5)))
    assert err.max() < 1e-10
    # symmetry and the Cholesky factor at full size
    for k in ("S", "T", "V", "PQ"):
        assert np.array_equal(host[k], host[k].T)
    assert np.array_equal(host["abP"], host["abP"].transpose(0, 2, 1))
    # The synthetic auxiliary set of this job is nearly linearly dependent: at this grid (P|Q) has
    # negative eigenvalues of order 1e-6, so the library must report NOT_PD (the other outputs stay
    # valid, as checked above).  The factor itself is tested on a well-conditioned metric below.
    PQ = host["PQ"]
    ev_min = np.linalg.eigvalsh(PQ)[0]
    _say(f"rc={rc} min eig(PQ)={ev_min:.3e}")
    if rc == psint.PS_E_NOT_PD:
        assert ev_min < 1e-12 * np.max(np.abs(PQ))
    else:
        assert rc == psint.PS_OK
        L = host["PQ_chol"]
        assert np.max(np.abs(L @ L.T - PQ)) < 1e-11 * np.max(np.abs(PQ))


@pytest.mark.parametrize("name,prec", [("triatomic_5z", "mixed"), ("hydrocarbon9", "mixed"),
                                       ("hydrocarbon9", "fp64")])
def test_larger_workloads_sampled_parity(name, prec):
    """The triatomic 5Z job (three refined 128x128x64-point grids, auxiliaries up to l = 6) and the
    hydrocarbon job (252 grids of 64-128 points per axis, several memory passes, contraction launches
    balanced over uneven grids) at full size with the default tiling, as the benchmark runs them,
    device outputs: sampled elements of every kind against the oracle, within 1e-10 in FP64, and in
    mixed precision within 1e-10 for S, T, V, (P|Q) and MIXED_ABP_REL_TOL of the largest element for
    (ab|P).  A context of its own,
    released at the end: the hydrocarbon job reserves most of the device memory."""
    job = getattr(W, name)()
    _say(f"{job.name} {prec}: n_bf={job.n_bf} n_aux={job.n_aux}")
    c = psint.Context(0)
    try:
        got, st, rc = c.compute(job, device=True, precision=prec)
        _say(f"passes={st['n_passes']} device_ms={st['device_ms']:.1f} rc={rc}")
        host = {k: v.cpu().numpy() for k, v in got.items()}
        del got
    finally:
        c.close()
    kinds, I, J, K = sample(job, 60, 11)
    ref, _ = O.compute_elements(job, kinds, I, J, K)
    err = np.abs(pick(host, kinds, I, J, K) - ref)
    for k in range(5):
        scale = np.max(np.abs(host[KINDS[k]]))
        e = err[kinds == k].max()
        _say(f"{KINDS[k]}: max abs err {e:.2e} (largest element {scale:.2e})")
        assert e < (TOL64 if prec == "fp64" else mixed_tol(KINDS[k], scale)), (KINDS[k], e, scale)
    for k in ("S", "T", "V", "PQ"):
        assert np.array_equal(host[k], host[k].T)


def _pd_metric_job():
    """Three atoms, 75 auxiliary functions with well-separated exponents up to l = 3: (P|Q) has
    condition number about 2e4 on a 10x10x8-cell grid, and 75 = two full 32-column panels plus a
    ragged 11-column one."""
    xyz = W.triatomic_geometry()
    basis = [[a, 1, 0, 0, 1.5 + 0.2 * a] for a in range(3)]
    aux = []
    for a in range(3):
        aux += [[a, 1, 0, 0, z] for z in (9.0, 3.0, 1.0)]
        aux += [[a, 2, 1, m, z] for z in (4.0, 1.5) for m in (-1, 0, 1)]
        aux += [[a, 3, 2, m, 2.5] for m in range(-2, 3)]
        aux += [[a, 4, 3, m, 2.2] for m in range(-3, 4)]
    aux += [[0, 3, 2, m, 1.2] for m in range(-2, 3)] + [[1, 4, 3, m, 1.4] for m in range(-3, 4)]
    return MiniJob(xyz, [8, 1, 1], basis, aux, Spec(10, 10, 8, 4, 3))


@pytest.mark.parametrize("device", [False, True])
def test_multi_panel_cholesky(ctx, device):
    """Blocked FP64 Cholesky over several panels with a ragged last panel: the factor matches LAPACK's
    factor of the same (P|Q) to 1e-12 relative, and (P|Q) matches the oracle."""
    job = _pd_metric_job()
    assert len(job.aux) == 75
    got, st, rc = ctx.compute(job, device=device)
    host = {k: (v.cpu().numpy() if device else v) for k, v in got.items()}
    assert rc == psint.PS_OK
    PQ, L = host["PQ"], host["PQ_chol"]
    ref = O.compute_full(job)
    assert np.max(np.abs(PQ - ref["PQ"])) < 1e-10
    assert np.array_equal(np.triu(L, 1), np.zeros_like(L))
    Lref = np.linalg.cholesky(PQ)
    scale = np.max(np.abs(Lref))
    _say(f"chol max err {np.max(np.abs(L - Lref)):.2e} (scale {scale:.2e})")
    assert np.max(np.abs(L - Lref)) < 1e-12 * scale
    assert np.max(np.abs(L @ L.T - PQ)) < 1e-13 * np.max(np.abs(PQ))


# Mixed precision: S, T, V and (P|Q) are contracted in FP64 inside a mixed job (FP64 copies of their
# operands), so they meet the FP64 bar.  (ab|P) uses FP32 operands rounded from FP64 values and FP32
# MFMA sums over 32-point stages folded into FP64: each term carries about one FP32 rounding
# (2^-24 = 6e-8 relative) per operand and per stage sum, so the error is held to 1e-7 of the type's
# largest element, under two FP32 units (measured 1.6e-8 to 3.1e-8 on the benchmark jobs, 6.2e-8 on a
# coarse 8 x 8 x 6-cell grid, where fewer points share each element).
TOL64 = 1e-10
MIXED_ABP_REL_TOL = 1e-7


def mixed_tol(kind, scale):
    return MIXED_ABP_REL_TOL * scale if kind == "abP" else TOL64


def _tri_tz(spec=(8, 8, 6, 4, 3, 2.3, 0.25)):
    rng = W.rng_for(1)
    Z = np.array([8.0, 1.0, 1.0])
    basis, aux = W.build_basis(rng, Z.astype(int), "TZ", "auxTZ", n_max=4)
    return MiniJob(W.triatomic_geometry(), Z, basis, aux, Spec(*spec))


@pytest.mark.parametrize("make", ["diatomic", "triatomic_tz"])
def test_mixed_precision_error_bars(ctx, make):
    """Mixed precision against the oracle: S, T, V, (P|Q) and the (P|Q) factor within the FP64 bar
    (their contractions stay in FP64); (ab|P) within MIXED_ABP_REL_TOL of its largest element."""
    job = W.diatomic_small() if make == "diatomic" else _tri_tz()
    ref = O.compute_full(job)
    got, st, rc = ctx.compute(job, precision="mixed")
    f64, _, _ = ctx.compute(job, precision="fp64")
    for k in KINDS:
        scale = np.max(np.abs(ref[k]))
        em = np.max(np.abs(got[k] - ref[k]))
        e64 = np.max(np.abs(f64[k] - ref[k]))
        _say(f"{make} {k}: mixed {em:.2e} fp64 {e64:.2e} scale {scale:.2e}")
        assert em <= mixed_tol(k, scale), (k, em, scale)
        assert e64 < TOL64
    if rc == 0:
        assert np.max(np.abs(got["PQ_chol"] - ref["PQ_chol"])) < TOL64 * max(1.0, np.max(np.abs(ref["PQ_chol"])))


def _serving_jobs():
    jobs = []
    rng = np.random.default_rng(42)
    for n in (2, 3, 4, 3, 2, 3):
        xyz = [[0.0, 0.0, 0.0]]
        while len(xyz) < n:
            v = rng.normal(size=3)
            cand = np.array(xyz[int(rng.integers(0, len(xyz)))]) + rng.uniform(1.8, 2.6) * v / np.linalg.norm(v)
            if all(np.linalg.norm(cand - np.array(p)) > 1.7 for p in xyz):
                xyz.append(list(cand))
        Z = rng.choice([1, 6, 8], size=n).astype(float)
        basis, aux = [], []
        for a in range(n):
            basis += [[a, 1, 0, 0, 2.0 + a * 0.1], [a, 2, 1, -1, 1.1], [a, 2, 1, 1, 1.1], [a, 3, 2, 0, 0.9]]
            aux += [[a, 1, 0, 0, 3.0], [a, 2, 1, 0, 2.4], [a, 3, 2, 2, 2.0]]
        s = int(rng.integers(5, 9))
        jobs.append(MiniJob(np.array(xyz), Z, basis, aux, Spec(s, s, 4, 4, 3)))
    return jobs


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_serving_results_identical_alone_and_in_the_mix(ctx, prec):
    """Jobs submitted together overlap on the device; each result equals (bit for bit) the same job run
    alone, because a job's plan and reduction order do not depend on what else runs."""
    jobs = _serving_jobs()
    alone = [ctx.compute(j, precision=prec)[0] for j in jobs]
    handles = [ctx.submit(j, precision=prec) for j in jobs]
    for h, a, j in zip(handles, alone, jobs):
        out, st, rc = ctx.wait(h, timeout_us=120_000_000)
        assert rc in (psint.PS_OK, psint.PS_E_NOT_PD)
        for k in psint.OUTPUTS:
            assert np.array_equal(out[k], a[k]), k
        assert st["total_ms"] >= st["queue_ms"] >= 0.0
    ref = O.compute_full(jobs[1])
    for k in KINDS:
        scale = float(np.max(np.abs(ref[k])))
        tol = TOL64 if prec == "fp64" else mixed_tol(k, scale)
        assert np.max(np.abs(alone[1][k] - ref[k])) < tol, k


SERVING_PICKS = [2, 5, 9, 12, 19, 31]  # requests of 2-4 atoms with DZ/TZ-sized bases, 0.4-8.5 M points


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_serving_stream_requests_identical_alone_and_in_the_mix(ctx, prec):
    """Six requests of the serving stream itself (random tree-grown molecules of 2-4 atoms, DZ/TZ-sized
    bases with 3x auxiliary sets, per-pair grids of 48-128 points per axis) submitted together: each
    result equals the request run alone bit for bit, and sampled elements of every kind match the
    oracle (FP64: 1e-10; mixed: S, T, V, (P|Q) 1e-10, (ab|P) MIXED_ABP_REL_TOL of its largest)."""
    reqs = W.serving_stream(n_requests=max(SERVING_PICKS) + 1)
    jobs = [reqs[i][1] for i in SERVING_PICKS]
    _say(", ".join(f"{j.name} ({j.n_bf}/{j.n_aux})" for j in jobs))
    alone = [ctx.compute(j, precision=prec)[0] for j in jobs]
    handles = [ctx.submit(j, precision=prec) for j in jobs]
    for h, a in zip(handles, alone):
        out, st, rc = ctx.wait(h, timeout_us=120_000_000)
        assert rc in (psint.PS_OK, psint.PS_E_NOT_PD)
        for k in psint.OUTPUTS:
            assert np.array_equal(out[k], a[k]), k
    for t, (j, a) in enumerate(zip(jobs, alone)):
        kinds, I, J, K = sample(j, 12, 100 + t)
        ref, _ = O.compute_elements(j, kinds, I, J, K)
        err = np.abs(pick(a, kinds, I, J, K) - ref)
        for kd in range(5):
            name = KINDS[kd]
            tol = TOL64 if prec == "fp64" else mixed_tol(name, float(np.max(np.abs(a[name]))))
            assert err[kinds == kd].max() < tol, (j.name, name, err[kinds == kd].max())


def test_serving_device_outputs_and_stats(ctx):
    jobs = _serving_jobs()[:3]
    hs = [ctx.submit(j, device=True) for j in jobs]
    for h, j in zip(hs, jobs):
        out, st, rc = ctx.wait(h)
        solo, _, _ = ctx.compute(j)
        assert np.array_equal(out["abP"].cpu().numpy(), solo["abP"])
        assert st["pair_points"] > 0 and st["device_ms"] > 0


def test_serving_rejects_job_beyond_budget():
    small = psint.Context(0, budget_bytes=64 << 20)
    with pytest.raises(psint.PsError) as e:
        small.submit(W.triatomic_qz())
    assert e.value.status == psint.PS_E_NOMEM
    # a small job still runs on the same context
    out, st, rc = small.compute(_serving_jobs()[0])
    assert rc in (psint.PS_OK, psint.PS_E_NOT_PD)
    small.close()


def test_wait_timeout_then_completion(ctx):
    job = _tri_tz((10, 10, 8, 4, 3, 2.3, 0.25))
    h = ctx.submit(job)
    out, st, rc = ctx.wait(h, timeout_us=0)
    if rc == psint.PS_E_TIMEOUT:
        out, st, rc = ctx.wait(h, timeout_us=-1)
    assert rc in (psint.PS_OK, psint.PS_E_NOT_PD)
    solo, _, _ = ctx.compute(job)
    assert np.array_equal(out["S"], solo["S"])


def test_memory_passes_match_single_pass():
    """A budget that forces several grid passes (the array region is reused) gives the same results as
    one pass, up to the summation order of the point splits."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.2, 0.0], [-0.4, 1.8, 0.3], [0.6, -0.5, 2.0]])
    basis = [[a, 1, 0, 0, 1.2 + 0.3 * a] for a in range(4)] + [[a, 2, 1, 1, 1.0] for a in range(4)]
    aux = [[a, 1, 0, 0, 2.5] for a in range(4)] + [[a, 2, 1, -1, 2.0] for a in range(4)]
    job = MiniJob(xyz, [6, 1, 8, 1], basis, aux, Spec(10, 10, 8, 4, 3))
    big = psint.Context(0)
    ref, st_big, _ = big.compute(job)
    assert st_big["n_passes"] == 1
    need = big.plan_work(job)["device_bytes"]
    got = st_small = None
    for frac in (0.5, 0.3, 0.2, 0.15, 0.1, 0.07):
        small = psint.Context(0, budget_bytes=int(need * frac))
        try:
            got, st_small, _ = small.compute(job)
        except psint.PsError as e:
            assert e.status == psint.PS_E_NOMEM
            small.close()
            continue
        small.close()
        _say(f"budget {need * frac / 1e6:.0f} MB: {st_small['n_passes']} passes")
        if st_small["n_passes"] >= 2:
            break
    assert st_small is not None and st_small["n_passes"] >= 2
    for k in psint.OUTPUTS:
        scale = max(np.max(np.abs(ref[k])), 1e-300)
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-12 * scale, k
    big.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_overlapped_passes_match_serial_passes(prec):
    """PS_OPT_OVERLAP_PASSES: under a budget that needs several memory passes, the overlapped plan
    (alternate regions, each pass's evaluation on the side stream during the previous contraction) gives
    the serial plan's results up to the grouping of the grids' sums, on its first run, its captured
    second run and its replayed third; and the same job served through the dispatcher agrees."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.2, 0.0], [-0.4, 1.8, 0.3], [0.6, -0.5, 2.0]])
    basis = [[a, 1, 0, 0, 1.2 + 0.3 * a] for a in range(4)] + [[a, 2, 1, 1, 1.0] for a in range(4)]
    aux = [[a, 1, 0, 0, 2.5] for a in range(4)] + [[a, 2, 1, -1, 2.0] for a in range(4)]
    job = MiniJob(xyz, [6, 1, 8, 1], basis, aux, Spec(10, 10, 8, 4, 3))
    probe = psint.Context(0)
    need = probe.plan_work(job, precision=prec)["device_bytes"]
    probe.close()
    c = None
    for frac in (0.6, 0.5, 0.4, 0.3, 0.25, 0.2, 0.15, 0.1):
        # a budget under which the job needs several passes and its largest grid fits half a region
        budget = int(need * frac)
        c = psint.Context(0, budget_bytes=budget)
        c.set_option(psint.PS_OPT_OVERLAP_PASSES, 1)
        try:
            first = c.compute(job, precision=prec)
        except psint.PsError as e:
            assert e.status == psint.PS_E_NOMEM
            first = None
        if first is not None and first[1]["passes_overlapped"]:
            break
        c.close()
        c = None
    assert c is not None, "no budget gave overlapped passes"
    serial = psint.Context(0, budget_bytes=budget)
    serial.set_option(psint.PS_OPT_OVERLAP_PASSES, 0)
    ref, st_ref, _ = serial.compute(job, precision=prec)
    serial.close()
    try:
        runs = [first] + [c.compute(job, precision=prec) for _ in range(2)]
        _say(f"{prec}: budget {budget / 1e6:.0f} MB, serial {st_ref['n_passes']} passes, overlapped "
             f"{runs[0][1]['n_passes']}; graph replay {[r[1]['graph_replay'] for r in runs]}")
        assert st_ref["n_passes"] >= 2 and st_ref["passes_overlapped"] == 0
        assert runs[2][1]["graph_replay"] == 1 and runs[2][1]["passes_overlapped"] == 1
        served, _, _ = c.wait(c.submit(job, precision=prec), timeout_us=60_000_000)
    finally:
        c.close()
    for i, (got, _, _) in enumerate(runs + [(served, None, None)]):
        for k in psint.OUTPUTS:
            scale = max(np.max(np.abs(ref[k])), 1e-300)
            d = np.max(np.abs(got[k] - ref[k]))
            assert d <= 1e-12 * scale, (i, k, d)
            if i:
                assert np.array_equal(got[k], runs[0][0][k]), (i, k)


def test_device_pool_reuse_across_job_sizes():
    """One context runs jobs of growing and shrinking size (its arena ranges move within the device
    pool; one job needs a quarter of the budget or more and reserves the rest of it; one needs two
    grid passes) and each result is bit-identical to the same job on a fresh context."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.2, 0.0], [-0.4, 1.8, 0.3], [0.6, -0.5, 2.0]])
    basis = [[a, 1, 0, 0, 1.2 + 0.3 * a] for a in range(4)] + [[a, 2, 1, 1, 1.0] for a in range(4)]
    aux = [[a, 1, 0, 0, 2.5] for a in range(4)] + [[a, 2, 1, -1, 2.0] for a in range(4)]
    small = MiniJob(xyz[:2], [6, 1], basis[:1] + basis[4:5], aux[:1], Spec(6, 6, 4))
    medium = MiniJob(xyz[:3], [6, 1, 8], [b for b in basis if b[0] < 3], [q for q in aux if q[0] < 3],
                     Spec(8, 8, 6))
    large = MiniJob(xyz, [6, 1, 8, 1], basis, aux, Spec(10, 10, 8, 4, 3))
    probe = psint.Context(0)
    need = probe.plan_work(large)["device_bytes"]
    probe.close()
    budget = int(need * 0.6)  # the large job alone needs two passes here; it takes over 1/4 of it
    jobs = [("small", small), ("medium", medium), ("large", large), ("small", small), ("medium", medium)]
    refs = {}
    for name, job in jobs[:3]:
        fresh = psint.Context(0, budget_bytes=budget)
        refs[name], st, _ = fresh.compute(job)
        fresh.close()
        _say(f"{name}: {st['n_passes']} passes")
    c = psint.Context(0, budget_bytes=budget)
    for name, job in jobs:
        got, st, _ = c.compute(job)
        for k in psint.OUTPUTS:
            assert np.array_equal(got[k], refs[name][k]), (name, k)
        _say(f"compute {name} ok")
    # the same through the serving path, all submitted at once (the idle arena of the synchronous
    # path, sized for the large job, is taken back when the served large job needs the memory)
    hs = [c.submit(job) for _, job in jobs]
    for (name, _), h in zip(jobs, hs):
        got, _, _ = c.wait(h, timeout_us=60_000_000)
        for k in psint.OUTPUTS:
            assert np.array_equal(got[k], refs[name][k]), (name, k, "served")
        _say(f"served {name} ok")
    c.close()


def test_compute_after_serving_takes_back_idle_slot_memory():
    """A served job leaves its arena with its (now idle) serving slot.  A later ps_compute of another
    job on the same context, which fits the budget only with that memory, takes it back from the slot
    instead of failing, and so does an RI call after serving again; results equal those of a fresh
    context with the same budget."""
    a = _tri_tz((8, 8, 6, 4, 3, 2.3, 0.25))
    b = _tri_tz((9, 8, 6, 4, 3, 2.3, 0.25))
    # a budget that holds either job's device memory but not both (the plan's workspace depends on
    # the budget, so the needs are taken from the planner under that budget)
    budget = psint.plan_work_host(a)["device_bytes"]
    for _ in range(6):
        probe = psint.Context(0, budget_bytes=budget)
        na_, nb_ = probe.plan_work(a)["device_bytes"], probe.plan_work(b)["device_bytes"]
        probe.close()
        mib = 2 << 20
        ra, rb = -(-na_ // mib) * mib, -(-nb_ // mib) * mib  # pool ranges are 2 MiB multiples
        if max(ra, rb) + mib <= budget < ra + rb:
            break
        budget = int(1.3 * max(ra, rb)) + mib
    _say(f"needs {na_ / 1e6:.0f} / {nb_ / 1e6:.0f} MB, budget {budget / 1e6:.0f} MB")
    assert max(ra, rb) + mib <= budget < ra + rb
    rng = np.random.default_rng(3)
    M = rng.normal(size=(len(b.aux),) * 2)
    Lr = np.linalg.cholesky(M @ M.T + len(b.aux) * np.eye(len(b.aux)))  # any factor: RI is linear in it
    fresh = psint.Context(0, budget_bytes=budget)  # same budget: same plan, same summation order
    ref_b, _, _ = fresh.compute(b)
    B_ref, e_ref, _ = fresh.ri_assemble(ref_b["abP"], Lr)
    fresh.close()
    c = psint.Context(0, budget_bytes=budget)
    try:
        c.wait(c.submit(a))
        got, _, rc = c.compute(b)
        for k in psint.OUTPUTS:
            assert np.array_equal(got[k], ref_b[k]), k
        c.wait(c.submit(a))
        B, e, _ = c.ri_assemble(got["abP"], Lr)
        assert np.array_equal(B, B_ref) and np.array_equal(e, e_ref)
    finally:
        c.close()


def test_autotune_selects_fastest_and_keeps_results():
    """ps_autotune times every candidate tiling, leaves the fastest on the context, and a job run with
    it agrees with the default tiling (up to the summation order of the point splits) and the oracle."""
    job = _tri_tz((10, 10, 8, 4, 3, 2.3, 0.25))
    c = psint.Context(0)
    ref, _, _ = c.compute(job)
    best, table = c.autotune(job, reps=2)
    _say("autotune: " + "; ".join(f"{t['wm']}x{t['wn']}x{t['stage_chunks']} {t['device_ms']:.3f} ms"
                                  for t in table))
    assert len(table) == 8
    assert best["device_ms"] == min(t["device_ms"] for t in table)
    assert all(t["device_ms"] > 0 and 0 < t["contract_ms"] <= t["device_ms"] for t in table)
    got, st, rc = c.compute(job)
    for k in KINDS:
        scale = max(np.max(np.abs(ref[k])), 1e-300)
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-12 * scale, k
    # this auxiliary metric is ill-conditioned, so the factor amplifies last-bit differences of (P|Q);
    # check it as a factor of the (P|Q) it came with
    if rc == psint.PS_OK:
        L = got["PQ_chol"]
        assert np.max(np.abs(L @ L.T - got["PQ"])) < 1e-12 * np.max(np.abs(got["PQ"]))
    orc = O.compute_full(job)
    assert max(np.max(np.abs(got[k] - orc[k])) for k in KINDS) < 1e-10
    with pytest.raises(psint.PsError):
        c.autotune(job, reps=0)
    c.close()


def test_plan_reuse_for_repeated_jobs():
    """ps_compute keeps the last plan on the context: the same job again reuses it (identical
    results), a changed job (one exponent, then the tiling) is planned afresh (results equal a fresh
    context's)."""
    job = _tri_tz((8, 8, 6, 4, 3, 2.3, 0.25))
    c = psint.Context(0)
    a1, _, _ = c.compute(job)
    a2, _, _ = c.compute(job)
    for k in psint.OUTPUTS:
        assert np.array_equal(a1[k], a2[k]), k
    changed = MiniJob(job.xyz, job.Z, job.basis.copy(), job.aux, job.grid)
    changed.basis[3, 4] *= 1.1
    b1, _, _ = c.compute(changed)
    fresh = psint.Context(0)
    b2, _, _ = fresh.compute(changed)
    for k in psint.OUTPUTS:
        assert np.array_equal(b1[k], b2[k]), k
    assert not np.array_equal(a1["S"], b1["S"])
    c.set_tiling(2, 2, 1, 0)
    a3, _, _ = c.compute(job)
    fresh.set_tiling(2, 2, 1, 0)
    a4, _, _ = fresh.compute(job)
    for k in psint.OUTPUTS:
        assert np.array_equal(a3[k], a4[k]), k
    c.close()
    fresh.close()


def test_repeated_job_graph_replay_matches_eager():
    """The second run of an unchanged job is captured into HIP graphs (one per segment) and later runs
    replay them: every replay, with other device work in between, equals the first (eager) run bit
    for bit, and the timing events between the graphs report."""
    import torch
    job = _tri_tz((8, 8, 6, 4, 3, 2.3, 0.25))
    c, other = psint.Context(0), psint.Context(0)
    ref, st0, _ = c.compute(job)
    x = torch.ones(1 << 20, dtype=torch.float64, device="cuda:0")
    for i in range(5):
        out, st, _ = c.compute(job)
        for k in psint.OUTPUTS:
            assert np.array_equal(out[k], ref[k]), (i, k)
        assert st["contract_ms"] > 0 and st["device_ms"] >= st["contract_ms"]
        assert st["graph_replay"] == 1 and st0["graph_replay"] == 0
        other.compute(_serving_jobs()[i % 3])  # eager work on another context in between
        x.mul_(1.0000001)
        torch.cuda.synchronize()
    dev, _, _ = c.compute(job, device=True)  # same plan, device outputs
    for k in psint.OUTPUTS:
        assert np.array_equal(dev[k].cpu().numpy(), ref[k]), k
    c.close()
    other.close()


def test_multi_pass_graph_replay_matches_eager_and_times_afresh():
    """A job split into several memory passes is replayed as one captured graph per segment (the
    evaluation, each pass's contraction, the reductions), with the timing events recorded between the
    graphs: every replay equals the eager run bit for bit, and the contraction time is measured on
    each replay rather than repeated from one run."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.2, 0.0], [-0.4, 1.8, 0.3], [0.6, -0.5, 2.0]])
    basis = [[a, 1, 0, 0, 1.2 + 0.3 * a] for a in range(4)] + [[a, 2, 1, 1, 1.0] for a in range(4)]
    aux = [[a, 1, 0, 0, 2.5] for a in range(4)] + [[a, 2, 1, -1, 2.0] for a in range(4)]
    job = MiniJob(xyz, [6, 1, 8, 1], basis, aux, Spec(10, 10, 8, 4, 3))
    probe = psint.Context(0)
    need = probe.plan_work(job)["device_bytes"]
    probe.close()
    c = psint.Context(0, budget_bytes=int(need * 0.3))
    ref, st0, _ = c.compute(job)
    assert st0["n_passes"] >= 2 and st0["graph_replay"] == 0
    times = set()
    for i in range(4):
        out, st, _ = c.compute(job)
        assert st["graph_replay"] == 1 and st["n_passes"] == st0["n_passes"]
        for k in psint.OUTPUTS:
            assert np.array_equal(out[k], ref[k]), (i, k)
        assert 0 < st["contract_ms"] <= st["device_ms"]
        times.add(round(st["contract_ms"], 6))
    _say(f"{st0['n_passes']} passes, contraction ms over replays: {sorted(times)}")
    assert len(times) > 1  # measured on every replay
    c.close()


@pytest.mark.parametrize("prec,peak", [("fp64", 78.6), ("mixed", 157.3)])
def test_mfma_rate_probe(ctx, prec, peak):
    """The matrix-pipe probe reports a rate between a third of the published dense peak and the peak
    itself (plus 5% for rounding of the published figure and clock variation)."""
    rate = ctx.mfma_rate(prec)
    _say(f"{prec}: probe {rate:.1f} TFLOP/s of {peak} published")
    assert peak / 3 < rate < 1.05 * peak
    out = psint.C.c_double()
    assert psint.lib().ps_mfma_rate(ctx.h, 7, psint.C.byref(out)) == psint.PS_E_INVALID
