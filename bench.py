#!/usr/bin/env python3
"""Benchmark: S/T/V/(ab|P) quadrature throughput (pair-points per second) on one MI355X.

One step = one ps_compute of the whole job (grid generation, function and potential evaluation,
every contraction, reductions, symmetrisation and the (P|Q) Cholesky) with outputs left in HBM.
The default workload is the largest single-GPU configuration: the 9-atom hydrocarbon with the
quadruple-zeta-sized basis on its 252 grids G(A,B|C) of 64-128 points per axis (uneven blocks,
several memory passes), in FP64 (--workload and --precision pick others).  Prints one JSON line.

  latency_ms    p50 / p99 / max of the timed steps and every step's time.
  roofline      the contraction kernel (the dominant kernel): algorithmic FLOPs per launch
                (2 per pair-point) over the launch's mean duration, measured with HIP events the
                library records around it on its own stream, against the MI355X FP64 (or FP32 for
                the mixed path) dense peak.
  mixed         (FP64 runs) the same job in mixed precision after the timed steps: throughput,
                contraction rate and the max-abs error of every output element against the FP64 run.
  cpu_baseline  the FP64 CPU oracle timed on a seeded sample of elements confined to a few of the
                job's grids, all host cores and one core; the same sample gives the stated max-abs
                error of the GPU outputs against the oracle.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "mixed": 157.3e12}  # MI355X dense FP64 / FP32 matrix peaks, FLOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="hydrocarbon9",
                    choices=["triatomic_qz", "triatomic_5z", "diatomic_small", "hydrocarbon9", "serving_stream",
                             "grid_ladder", "nsp_sweep", "geometry_scan"])
    ap.add_argument("--autotune", action="store_true",
                    help="choose the contraction tiling with ps_autotune before the timed steps")
    ap.add_argument("--requests", type=int, default=40, help="serving_stream: measured requests")
    ap.add_argument("--warmup-requests", type=int, default=3, help="serving_stream: untimed requests")
    ap.add_argument("--rate", type=float, default=50.0, help="serving_stream: Poisson arrival rate, 1/s")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default fp64 (serving_stream: mixed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg of an FP64 run")
    ap.add_argument("--cpu-pair-points", type=float, default=3e11,
                    help="largest (ab|P on C) block, in pair-points, the oracle sample may pick")
    ap.add_argument("--tiling", default="0,0,0,0", help="wm,wn,stage_chunks,ksplit (0 = library default)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "contract_traffic.json"))
    ap.add_argument("--no-ri", action="store_true", help="skip the RI-assembly measurement after the steps")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter calibration)")
    return ap.parse_args()


def kernel_source_hash():
    """Hash of the sources that decide the contraction's memory traffic: the contraction kernels (the
    part of kernels.hip from their section header to the reduction's) and the tile planner."""
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2510_15204_amd/csrc/kernels.hip"), encoding="utf-8") as fh:
        k = fh.read()
    i, j = k.find("// Contraction kernels."), k.find("// Sum the splits of each reduction item")
    h.update(k[i:j].encode() if 0 <= i < j else k.encode())
    with open(os.path.join(ROOT, "paper_2510_15204_amd/csrc/plan.cpp"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def tiling_is_default(args, tuning):
    return tuning is None and all(int(x) == 0 for x in args.tiling.split(","))


def third_atom_blocks(job):
    """The (ab|P on C) blocks of the job, one per grid G(A,B|C): (A, B, C, points, pair-points).
    These are the job's dominant work; the point count follows the grid spec (refined at C)."""
    bat = job.basis[:, 0].astype(int)
    xat = job.aux[:, 0].astype(int)
    out = []
    for A in range(job.n_atoms):
        for B in range(A + 1, job.n_atoms):
            sp = job.spec_for(A, B)
            pts = (sp.n_mu * sp.n_nu * sp.n_phi + 8 * (sp.n_sp ** 3 - 1)) * sp.q ** 3
            for C in range(job.n_atoms):
                if C in (A, B):
                    continue
                el = int(np.sum(bat == A)) * int(np.sum(bat == B)) * int(np.sum(xat == C))
                if el:
                    out.append((A, B, C, pts, float(el) * pts))
    return out


def oracle_sample(job, rng, max_pp, n_aux_per_block=None):
    """Seeded oracle sample: every (ab|P on C) element of one grid G(A,B|C) chosen at random among the
    blocks of at most max_pp pair-points (the smallest block if none is), or only n_aux_per_block of
    its P; plus 4 S, T, V and (P|Q) elements of the same atom pair (its other grids).
    Returns (kinds, I, J, K, description)."""
    blocks = third_atom_blocks(job)
    fit = [b for b in blocks if b[4] <= max_pp] or [min(blocks, key=lambda b: b[4])]
    A, B, C, pts, _ = fit[int(rng.integers(len(fit)))]
    bat = job.basis[:, 0].astype(int)
    xat = job.aux[:, 0].astype(int)
    fa, fb, pc = np.flatnonzero(bat == A), np.flatnonzero(bat == B), np.flatnonzero(xat == C)
    if n_aux_per_block:
        pc = np.sort(rng.choice(pc, size=min(n_aux_per_block, pc.size), replace=False))
    kinds, I, J, K = [], [], [], []
    for P in pc:
        for a in fa:
            for b in fb:
                kinds.append(4); I.append(int(a)); J.append(int(b)); K.append(int(P))
    pa, pb = np.flatnonzero(xat == A), np.flatnonzero(xat == B)
    for kd in range(4):
        for _ in range(4):
            if kd == 3:
                if not (pa.size and pb.size):
                    continue
                kinds.append(3); I.append(int(rng.choice(pa))); J.append(int(rng.choice(pb)))
            else:
                kinds.append(kd); I.append(int(rng.choice(fa))); J.append(int(rng.choice(fb)))
            K.append(0)
    desc = (f"(ab|P on C) block of G({A},{B}|{C}) ({pts} points): {fa.size}x{fb.size}x{pc.size} elements, "
            f"plus S/T/V/(P|Q) elements of atoms {A},{B}")
    return np.array(kinds), np.array(I), np.array(J), np.array(K), desc


def cpu_baseline_leg(job, outs, args, pair_points_job):
    """The FP64 oracle on a seeded grid-confined sample of the job (all host cores; then one core on a
    smaller sample), scaled to pair-points/s; max-abs error of the GPU outputs on the sample."""
    import oracle as O
    kinds, I, J, K, desc = oracle_sample(job, np.random.default_rng(15204), args.cpu_pair_points)
    cores = O.set_threads(0)
    c0 = time.perf_counter()
    vals, wpp = O.compute_elements(job, kinds, I, J, K)
    cdt = time.perf_counter() - c0
    host = {k: v.cpu().numpy() for k, v in outs.items()}
    got = np.array([host["abP"][p, a, b] if kd == 4 else host[("S", "T", "V", "PQ")[kd]][a, b]
                    for kd, a, b, p in zip(kinds, I, J, K)])
    err = {name: float(np.max(np.abs(got[kinds == kd] - vals[kinds == kd]))) if np.any(kinds == kd) else None
           for kd, name in enumerate(("S", "T", "V", "PQ", "abP"))}
    rate = wpp / cdt
    # one core: the smallest block, a few of its auxiliary functions
    k1, i1, j1, p1, desc1 = oracle_sample(job, np.random.default_rng(15205), 0.0, n_aux_per_block=30)
    O.set_threads(1)
    c1 = time.perf_counter()
    _, wpp1 = O.compute_elements(job, k1, i1, j1, p1)
    cdt1 = time.perf_counter() - c1
    O.set_threads(cores)
    base = {"value": rate, "unit": "pair·points/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"{len(kinds)} seeded elements: {desc}; {wpp:.3e} pair-points in {cdt:.1f} s; the whole "
                       f"job ({pair_points_job:.3e} pair-points) would take {pair_points_job / rate:.0f} s at "
                       f"this rate"),
            "single_thread": {"value": wpp1 / cdt1, "unit": "pair·points/s", "cores": 1,
                              "sample": f"{len(k1)} seeded elements: {desc1}; {wpp1:.3e} pair-points in "
                                        f"{cdt1:.1f} s"}}
    return base, err


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the library has no multi-GPU path "
                                   "(whole grids would be spread over GPUs by their cost, each GPU running "
                                   "the single-GPU path)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}), flush=True)
        return
    from paper_2510_15204_amd import psint
    from paper_2510_15204_amd import workloads as W

    if args.workload == "serving_stream":
        return serve_bench(args, torch, psint, W)
    if args.workload in ("grid_ladder", "nsp_sweep", "geometry_scan"):
        return accuracy_bench(args, psint, W)
    job = W.WORKLOADS[args.workload]()
    prec = args.precision or "fp64"
    ctx = psint.Context(0)
    wm, wn, sc, ks = (int(x) for x in args.tiling.split(","))
    if wm or wn or sc or ks:
        ctx.set_tiling(wm, wn, sc, ks)
    tuning = None
    if args.autotune:
        best, table = ctx.autotune(job, precision=prec, reps=1)
        tuning = {"chosen": [best["wm"], best["wn"], best["stage_chunks"], best["ksplit"]],
                  "device_ms": {f"{t['wm']}x{t['wn']}x{t['stage_chunks']}": round(t["device_ms"], 3)
                                for t in table}}
        print(f"[bench] autotune: {tuning}", flush=True)
    nb, na = job.n_bf, job.n_aux
    outs = device_outputs(torch, nb, na)
    print(f"[bench] workload={job.name} precision={prec} n_bf={nb} n_aux={na}", flush=True)
    run = timed_steps(ctx, job, prec, outs, args.steps, args.warmup, torch)
    lat, stats, rc, elapsed = run["lat"], run["stats"], run["rc"], run["elapsed"]
    pp = stats["pair_points"]
    value = pp * args.steps / elapsed
    flops = stats["contract_flops"]
    mean_contract_s = float(np.mean(run["contract_ms"])) / 1e3
    achieved = flops / mean_contract_s
    traffic = None
    if os.path.exists(args.traffic_json):
        # counters taken on this workload and precision with the current kernel and planner sources
        try:
            tj = json.load(open(args.traffic_json))
            if (tj.get("workload") == job.name and tj.get("precision") == prec
                    and tj.get("source_hash") == kernel_source_hash() and tiling_is_default(args, tuning)):
                traffic = tj.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK[prec], "traffic": traffic,
                "kernel": ("contract_mixed" if prec == "mixed" else "contract_f64") + " (all launches)",
                "flops_per_launch": flops, "mean_launch_ms": mean_contract_s * 1e3}
    # what this device's matrix pipe sustains in the path's precision (a probe kernel of independent
    # MFMAs, after the timed steps), beside the published peak that `frac` uses
    probe = ctx.mfma_rate(prec) * 1e12
    roofline["probe_peak"] = probe / 1e12
    roofline["frac_of_probe"] = achieved / probe
    out = {"metric": "S/T/V/(ab|P) quadrature pair·points/s at stated error vs FP64; p99 job latency",
           "value": value, "unit": "pair·points/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": job.name, "atoms": job.n_atoms, "n_bf": nb, "n_aux": na,
                      "grids": int(stats["n_grids"]), "points": int(stats["n_points"]),
                      "pair_points_per_step": pp, "precision": prec, "passes": int(stats["n_passes"]),
                      "graph_replay": bool(stats["graph_replay"]),
                      "tiling": tuning["chosen"] if tuning else args.tiling},
           "latency_ms": latency_summary(lat),
           "roofline": roofline}
    if tuning:
        out["autotune"] = tuning
    PQ = outs["PQ"].cpu().numpy()
    out["metric_min_eigenvalue"] = {"PQ": float(np.linalg.eigvalsh(PQ)[0]), "PQ_max": float(np.max(np.diag(PQ))),
                                    "cholesky_status": int(rc)}
    if prec == "fp64" and not args.no_mixed:
        out["mixed"] = mixed_leg(ctx, job, outs, torch, max(2, args.steps // 4))
    elif prec == "mixed":
        # every element of the mixed result against one FP64 run of the same job on the device (the
        # FP64 path equals the oracle to ~1e-12, checked by the sampled oracle comparison and tests)
        ref, _, _ = ctx.compute(job, precision="fp64")
        out["error_vs_fp64_full"] = full_error({k: v.cpu().numpy() for k, v in outs.items()}, ref)
    if not args.no_ri:
        out["ri_assembly"] = ri_leg(ctx, outs, rc, psint)
    if not args.no_cpu_baseline:
        print("[bench] oracle sample on the host cores", flush=True)
        out["cpu_baseline"], out["error_vs_fp64_oracle"] = cpu_baseline_leg(job, outs, args, pp)
    print(json.dumps(out), flush=True)


def device_outputs(torch, nb, na):
    """Device output tensors, allocated once; the job's inputs are a few KB of host structs."""
    dev = torch.device("cuda:0")
    return {"S": torch.empty((nb, nb), dtype=torch.float64, device=dev),
            "T": torch.empty((nb, nb), dtype=torch.float64, device=dev),
            "V": torch.empty((nb, nb), dtype=torch.float64, device=dev),
            "PQ": torch.empty((na, na), dtype=torch.float64, device=dev),
            "PQ_chol": torch.empty((na, na), dtype=torch.float64, device=dev),
            "abP": torch.empty((na, nb, nb), dtype=torch.float64, device=dev)}


def timed_steps(ctx, job, prec, outs, steps, warmup, torch):
    """warmup untimed jobs, then `steps` timed ones bracketed by device synchronisation."""
    for i in range(warmup):
        ctx.compute(job, precision=prec, device=True, out_tensors=outs)
        print(f"[bench] {prec} warmup {i + 1}/{warmup} done", flush=True)
    torch.cuda.synchronize()
    lat, contract_ms, stats, rc = [], [], None, None
    t0 = time.perf_counter()
    for i in range(steps):
        s0 = time.perf_counter()
        _, stats, rc = ctx.compute(job, precision=prec, device=True, out_tensors=outs)
        lat.append((time.perf_counter() - s0) * 1e3)
        contract_ms.append(stats["contract_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] {prec}: {steps} steps in {elapsed:.3f}s", flush=True)
    return {"lat": lat, "contract_ms": contract_ms, "stats": stats, "rc": rc, "elapsed": elapsed}


def latency_summary(lat):
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "max": float(np.max(lat)), "steps": [round(float(x), 3) for x in lat]}


def full_error(got, ref):
    """Max-abs error of every element per output type, and over that type's largest element."""
    err = {}
    for k in ("S", "T", "V", "PQ", "abP"):
        d = float(np.max(np.abs(got[k] - ref[k]))) if ref[k].size else 0.0
        scale = float(np.max(np.abs(ref[k]))) if ref[k].size else 0.0
        err[k] = {"max_abs": d, "max_abs_over_max_element": d / scale if scale else 0.0}
    return err


def mixed_leg(ctx, job, outs64, torch, steps):
    """The same job in mixed precision after the FP64 steps: throughput, contraction rate against the
    FP32 peak, and every output element against the FP64 run."""
    outs = device_outputs(torch, job.n_bf, job.n_aux)
    run = timed_steps(ctx, job, "mixed", outs, steps, 1, torch)
    st = run["stats"]
    achieved = st["contract_flops"] / (float(np.mean(run["contract_ms"])) / 1e3)
    res = {"value": st["pair_points"] * steps / run["elapsed"], "unit": "pair·points/s", "steps": steps,
           "ms_per_step": run["elapsed"] * 1e3 / steps, "passes": int(st["n_passes"]),
           "latency_ms": latency_summary(run["lat"]),
           "contract_tflops": achieved / 1e12, "contract_frac_fp32_peak": achieved / PEAK["mixed"],
           "error_vs_fp64_full": full_error({k: v.cpu().numpy() for k, v in outs.items()},
                                            {k: v.cpu().numpy() for k, v in outs64.items()})}
    del outs
    torch.cuda.empty_cache()
    return res


def ri_leg(ctx, outs, rc, psint, reps=3):
    """RI assembly (eq. 14) on the job's (ab|P) and (P|Q) factor, after the timed steps.  When the
    synthetic auxiliary metric is not positive definite at this grid, the factor of (P|Q) + eps I
    (eps = 1e-5 of its largest diagonal element) stands in; the kernels' work does not depend on it."""
    import torch
    abP, L = outs["abP"], outs["PQ_chol"]
    note = "factor of the job's (P|Q)"
    if rc != psint.PS_OK:
        PQ = outs["PQ"].cpu().numpy()
        eps = 1e-5 * float(np.max(np.diag(PQ)))
        L = torch.from_numpy(np.linalg.cholesky(PQ + eps * np.eye(PQ.shape[0]))).to(abP.device)
        note = f"(P|Q) not positive definite at this grid; factor of (P|Q) + {eps:.2e} I"
    na, nb = abP.shape[0], abP.shape[1]
    npair = nb * (nb + 1) // 2
    ctx.ri_assemble(abP, L)  # warm-up (allocates the scratch)
    ms = [ctx.ri_assemble(abP, L)[2] for _ in range(reps)]
    syrk = float(npair) * (npair + 1) * na  # 2 FLOPs per multiply-add over the upper triangle
    trsm = float(na) * na * npair
    t = float(np.mean(ms)) / 1e3
    return {"inputs": note, "n_pair": npair, "n_aux": na, "ms": t * 1e3, "flops": syrk + trsm,
            "achieved_tflops": (syrk + trsm) / t / 1e12, "frac_fp64_peak": (syrk + trsm) / t / PEAK["fp64"]}


def accuracy_bench(args, psint, W):
    """The grid-accuracy and geometry-scan harnesses at the paper's sizes: Table S3 ladders against
    the 80 x 70 x 50-cell reference grid (eq. 13), N_SP = 1..4 on the OF2 shape and its stretched
    variant, and the 16-direction two-centre Coulomb scan on the reference grid."""
    from paper_2510_15204_amd import accuracy as A
    ctx = psint.Context(0)
    t0 = time.perf_counter()
    if args.workload == "grid_ladder":
        res = [A.grid_ladder(ctx, job, A.LADDER_S3) for job in (W.clf_tz(), W.of2_tz())]
        body = {job["job"]: {"reference_points": job["reference_points"],
                             "rows": [{"spec": r["spec"], "points": r["points"],
                                       "rmse": {k: float(f"{v:.3e}") for k, v in r["rmse"].items()}}
                                      for r in job["rows"]]} for job in res}
    elif args.workload == "nsp_sweep":
        res = [A.nsp_sweep(ctx, job, A.NSP_LADDER_S3) for job in (W.of2_tz(), W.of2_tz(long_bond=True))]
        body = {r["job"]: {str(k): [float(f"{x:.3e}") for x in v] for k, v in r["rmse_V"].items()} for r in res}
    else:
        dist = [1.0 + 0.25 * i for i in range(21)]
        scan = A.geometry_scan(ctx, dist)
        fine_ok = {"jobs": scan["jobs"], "wall_s": scan["wall_s"], "pair_points": scan["pair_points"],
                   "pairs": scan["pairs"], "distances": dist,
                   "values_dir0": np.round(scan["values"][0], 10).tolist(),
                   "values_dir15": np.round(scan["values"][15], 10).tolist()}
        body = fine_ok
    wall = time.perf_counter() - t0
    print(json.dumps({"metric": f"{args.workload} (eq. 13 RMSE / Fig. 6 scan)", "value": wall, "unit": "s",
                      "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": args.workload}, "result": body}), flush=True)


def serve_bench(args, torch, psint, W):
    """Continuous-batching run of the Poisson serving stream: requests are submitted at their arrival
    times from this thread while a second thread waits for them in order; latency = completion -
    arrival.  The first requests run alone (untimed) to warm up."""
    import threading
    n_warm, n_meas = args.warmup_requests, args.requests
    reqs = W.serving_stream(n_requests=n_warm + n_meas, rate_per_s=args.rate)
    prec = args.precision or "mixed"
    ctx = psint.Context(0)
    for i in range(n_warm):  # through the serving path, so no synchronous arena stays allocated
        ctx.wait(ctx.submit(reqs[i][1], outputs=("S", "T", "V", "PQ", "abP"), precision=prec, device=True))
        print(f"[bench] warmup request {i + 1}/{n_warm} done", flush=True)
    torch.cuda.synchronize()
    meas = reqs[n_warm:]
    t_first = meas[0][0]
    handles = [None] * n_meas
    done = [None] * n_meas
    ready = threading.Semaphore(0)

    def waiter():
        for i in range(n_meas):
            ready.acquire()
            if handles[i] is None:  # rejected at submission
                continue
            try:
                _, st, rc = ctx.wait(handles[i])
            except psint.PsError as e:
                st, rc = None, e.status
                print(f"[bench] request {i} failed: {e}", flush=True)
            done[i] = (time.perf_counter(), st, rc)
            handles[i] = None  # release the device outputs
            if (i + 1) % 10 == 0:
                print(f"[bench] {i + 1}/{n_meas} requests complete", flush=True)

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    arrivals = []
    for i, (ta, job) in enumerate(meas):
        due = t0 + (ta - t_first)
        now = time.perf_counter()
        if due > now:
            time.sleep(due - now)
        arrivals.append(due)
        try:
            handles[i] = ctx.submit(job, outputs=("S", "T", "V", "PQ", "abP"), precision=prec, device=True)
        except psint.PsError as e:
            handles[i] = None
            print(f"[bench] request {i} rejected: {e}", flush=True)
        ready.release()
    th.join()
    torch.cuda.synchronize()
    ok = [(d, a) for d, a in zip(done, arrivals) if d is not None and d[1] is not None]
    rejected = n_meas - len(ok)
    t_end = max(d[0] for d, _ in ok)
    makespan = t_end - t0
    lat = np.array([(d[0] - a) * 1e3 for d, a in ok])
    pp = sum(d[1]["pair_points"] for d, _ in ok)
    # in service = admitted on the device -> results ready; busy = union of those intervals
    spans = sorted((a + d[1]["queue_ms"] / 1e3, a + d[1]["total_ms"] / 1e3) for d, a in ok)
    busy, cur0, cur1 = 0.0, None, None
    for b0, b1 in spans:
        if cur1 is None or b0 > cur1:
            if cur1 is not None:
                busy += cur1 - cur0
            cur0, cur1 = b0, b1
        else:
            cur1 = max(cur1, b1)
    if cur1 is not None:
        busy += cur1 - cur0
    service_ms = [d[1]["total_ms"] - d[1]["queue_ms"] for d, _ in ok]
    done = [d for d, _ in ok]
    atoms = [job.n_atoms for _, job in meas]
    out = {"metric": "S/T/V/(ab|P) quadrature pair·points/s at stated error vs FP64; p99 job latency",
           "value": pp / makespan, "unit": "pair·points/s", "n_gpus": 1, "steps": n_meas,
           "warmup": n_warm, "ms_per_step": makespan * 1e3 / n_meas, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": "serving_stream", "requests": n_meas, "rate_per_s": args.rate,
                      "atoms_min_max": [min(atoms), max(atoms)], "precision": prec,
                      "pair_points_total": pp},
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                          "max": float(lat.max())},
           "serving": {"makespan_s": makespan, "completed_requests_per_s": n_meas / makespan,
                       "mean_queue_ms": float(np.mean([d[1]["queue_ms"] for d in done])),
                       "mean_service_ms": float(np.mean(service_ms)),
                       "utilisation_rho": args.rate * float(np.mean(service_ms)) / 1e3,
                       "device_busy_fraction": busy / makespan,
                       "latency_ms_each": [round(float(x), 1) for x in lat],
                       "not_pd": int(sum(d[2] == psint.PS_E_NOT_PD for d in done)), "rejected": rejected}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
