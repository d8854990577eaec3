#!/usr/bin/env python3
"""Benchmark: S/T/V/(ab|P) quadrature throughput (pair-points per second) on one MI355X.

One step = one ps_compute of the whole job (grid generation, function and potential evaluation,
every contraction, reductions, symmetrisation and the (P|Q) Cholesky) with outputs left in HBM.
The workload is the bent triatomic with the quadruple-zeta-sized basis on three refined
96x96x48-point grids in FP64 (--workload picks another).  Prints one JSON line.

  roofline      the contraction kernel (the dominant kernel): algorithmic FLOPs per launch
                (2 per pair-point) over the launch's mean duration, measured with HIP events the
                library records around it on its own stream, against the MI355X FP64 (or FP32 for
                the mixed path) dense peak.
  cpu_baseline  the FP64 CPU oracle timed on a seeded sample of the same job's output elements;
                the same sample gives the stated max-abs error of the GPU outputs.
  error_vs_fp64_full  (mixed precision) max-abs error of every output element against an FP64
                run of the same job, absolute and over the type's largest element.
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
    ap.add_argument("--workload", default="triatomic_qz",
                    choices=["triatomic_qz", "triatomic_5z", "diatomic_small", "hydrocarbon9", "serving_stream",
                             "grid_ladder", "nsp_sweep", "geometry_scan"])
    ap.add_argument("--autotune", action="store_true",
                    help="choose the contraction tiling with ps_autotune before the timed steps")
    ap.add_argument("--requests", type=int, default=40, help="serving_stream: measured requests")
    ap.add_argument("--warmup-requests", type=int, default=3, help="serving_stream: untimed requests")
    ap.add_argument("--rate", type=float, default=50.0, help="serving_stream: Poisson arrival rate, 1/s")
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=200000, help="abP elements in the oracle sample")
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


def sample_elements(job, n_abp, rng):
    """Seeded sample of output elements of every kind (S, T, V, PQ, abP)."""
    nb, na = job.n_bf, job.n_aux
    kinds, I, J, K = [], [], [], []
    for kind, n in ((0, 6), (1, 6), (2, 6), (3, 6)):
        lim = na if kind == 3 else nb
        for _ in range(n):
            a, b = sorted(rng.integers(0, lim, size=2))
            kinds.append(kind); I.append(a); J.append(b); K.append(0)
    for _ in range(n_abp):
        a, b = sorted(rng.integers(0, nb, size=2))
        kinds.append(4); I.append(a); J.append(b); K.append(int(rng.integers(0, na)))
    return np.array(kinds), np.array(I), np.array(J), np.array(K)


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
    prec = args.precision or job.precision
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
    # device outputs allocated once; the job's inputs are a few KB of host structs
    dev = torch.device("cuda:0")
    nb, na = job.n_bf, job.n_aux
    outs = {"S": torch.empty((nb, nb), dtype=torch.float64, device=dev),
            "T": torch.empty((nb, nb), dtype=torch.float64, device=dev),
            "V": torch.empty((nb, nb), dtype=torch.float64, device=dev),
            "PQ": torch.empty((na, na), dtype=torch.float64, device=dev),
            "PQ_chol": torch.empty((na, na), dtype=torch.float64, device=dev),
            "abP": torch.empty((na, nb, nb), dtype=torch.float64, device=dev)}
    print(f"[bench] workload={job.name} precision={prec} n_bf={nb} n_aux={na}", flush=True)
    for i in range(args.warmup):
        ctx.compute(job, precision=prec, device=True, out_tensors=outs)
        print(f"[bench] warmup {i + 1}/{args.warmup} done", flush=True)
    torch.cuda.synchronize()
    lat, contract_ms, stats = [], [], None
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        _, stats, rc = ctx.compute(job, precision=prec, device=True, out_tensors=outs)
        lat.append((time.perf_counter() - s0) * 1e3)
        contract_ms.append(stats["contract_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s", flush=True)
    pp = stats["pair_points"]
    value = pp * args.steps / elapsed
    flops = stats["contract_flops"]
    mean_contract_s = float(np.mean(contract_ms)) / 1e3
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
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
           "roofline": roofline}
    if tuning:
        out["autotune"] = tuning
    if prec == "mixed":
        # every element of the mixed result against one FP64 run of the same job on the device (the
        # FP64 path equals the oracle to ~1e-12, checked by the sampled oracle comparison and tests)
        ref, _, _ = ctx.compute(job, precision="fp64")
        err = {}
        for k in ("S", "T", "V", "PQ", "abP"):
            got = outs[k].cpu().numpy()
            d = float(np.max(np.abs(got - ref[k]))) if ref[k].size else 0.0
            scale = float(np.max(np.abs(ref[k]))) if ref[k].size else 0.0
            err[k] = {"max_abs": d, "max_abs_over_max_element": d / scale if scale else 0.0}
        out["error_vs_fp64_full"] = err
    if not args.no_ri:
        out["ri_assembly"] = ri_leg(ctx, outs, rc, psint)
    if not args.no_cpu_baseline:
        import oracle as O
        rng = np.random.default_rng(15204)
        kinds, I, J, K = sample_elements(job, args.cpu_sample, rng)
        cores = O.set_threads(0)
        c0 = time.perf_counter()
        vals, wpp = O.compute_elements(job, kinds, I, J, K)
        cdt = time.perf_counter() - c0
        host = {k: v.cpu().numpy() for k, v in outs.items()}
        got = np.empty(len(kinds))
        for e, (kd, a, b, p) in enumerate(zip(kinds, I, J, K)):
            got[e] = host["abP"][p, a, b] if kd == 4 else host[("S", "T", "V", "PQ")[kd]][a, b]
        err = {name: float(np.max(np.abs(got[kinds == kd] - vals[kinds == kd])))
               for kd, name in enumerate(("S", "T", "V", "PQ", "abP"))}
        out["cpu_baseline"] = {"value": wpp / cdt, "unit": "pair·points/s", "cores": int(cores),
                               "kind": "oracle",
                               "sample": f"{len(kinds)} seeded elements (6 each of S/T/V/PQ, "
                                         f"{args.cpu_sample} of (ab|P)) of the same job, "
                                         f"{wpp:.3e} pair-points in {cdt:.1f} s"}
        out["error_vs_fp64_oracle"] = err
    print(json.dumps(out), flush=True)


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
           "serving": {"makespan_s": makespan, "capacity_requests_per_s": n_meas / makespan,
                       "offered_load": args.rate * makespan / n_meas,
                       "mean_queue_ms": float(np.mean([d[1]["queue_ms"] for d in done])),
                       "not_pd": int(sum(d[2] == psint.PS_E_NOT_PD for d in done)), "rejected": rejected}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
