"""Benchmark: Anderson-accelerated Lloyd K-Means solves on one MI355X.

One step = one complete solve (Algorithm 1: every assignment, update,
Anderson and controller step until convergence) of the Gaussian-mixture
workload N=1,000,000, d=32, K=256 (float32), m_max=10, tol=1e-6, from a
seeded random-sample initialisation (step s uses init seed s), with the
row bounds of the paper's assignment method (Hamerly's lower bound; --bounds 0
assigns every row through the distance GEMM).  X stays resident in HBM; the
timed region holds K steps between two device synchronisations.  Prints one
JSON line.

    python bench.py [--gpus 1] [--steps 100] [--warmup 2] [--no-cpu-baseline | --cpu-full-solve] [--bounds 0|1]
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

FP32_MFMA_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
HBM_PEAK_GBS = 8000.0

WORKLOAD = dict(N=1_000_000, d=32, K=256, m_max=10, tol=1e-6, max_iter=500)

# HBM bytes per launch of the assignment kernels from rocprofv3 FETCH_SIZE and
# WRITE_SIZE, each scaled by its reading for a plain copy of known size
# (profiles/assign_f32_N1M_d32_K256_traffic.md): the dense pass (every row
# through the GEMM) and the mean over the candidate launches of a solve with
# row bounds.  Set to None when the kernel changes until it is measured again.
TRAFFIC_BYTES_PER_LAUNCH = 137474245
TRAFFIC_BYTES_PER_LAUNCH_BND = 181306566


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="solves timed (default workload: one seed each, seed = step index)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full-solve", nargs="?", const="f64", choices=["f64", "f32"], default=None,
                    help="default workload: the CPU baseline is one complete oracle solve from the first "
                         "timed seed's starting centroids (minutes) instead of one timed oracle pass; f32: "
                         "the oracle stores its iterates in float32 as the GPU does")
    ap.add_argument("--bounds", type=int, choices=[0, 1], default=1,
                    help="default workload: keep row bounds (Hamerly's lower bound, the assignment method of "
                         "the paper's experiments; KM_FLAG_BOUNDS) and skip the distance GEMM for rows they "
                         "prove (1, default), or assign every row through the GEMM (0)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU time budget of the oracle baseline sample")
    ap.add_argument("--workload", choices=["plain", "small", "precision", "batched", "served", "studies",
                                           "update"],
                    default="plain",
                    help="plain: N=1e6 d=32 K=256 float32 (default line); small: N=1e4 d=2 K=10 over "
                         "100 seeds, Lloyd and Anderson, p50/p99 latency beside the oracle on the host; precision: "
                         "N=4e6 d=128 K=1024 bfloat16-stored X, float32 vs bfloat16 GEMM; batched: "
                         "512 uneven instances in one engine vs one at a time; served: Poisson arrivals "
                         "(200 jobs/s) through the continuous-batching engine vs a FIFO loop; studies: fixed vs "
                         "dynamic m and Lloyd vs Anderson on synthetic mixtures; update: the update step "
                         "against the HBM roofline at N=1e7 d=16 K=256 and N=1e6 d=32 K=256")
    ap.add_argument("--seeds", type=int, default=100, help="small: number of seeds")
    ap.add_argument("--instances", type=int, default=512, help="batched: number of instances")
    ap.add_argument("--duration", type=float, default=60.0, help="served: seconds of arrivals")
    ap.add_argument("--rate", type=float, default=200.0, help="served: arrivals per second")
    ap.add_argument("--engines", type=int, choices=[1, 2], default=1,
                    help="served: one engine for all jobs, or one per size class (large jobs on "
                         "3/4 of the assignment workgroups)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def cpu_baseline(X, C0, passes_per_solve, budget_s):
    """Time the FP64 oracle's G pass on a bounded sample of rows."""
    from oracle import kmeans_oracle as ko
    n = X.shape[0]
    chunk = 32768
    rows = 0
    t0 = time.perf_counter()
    while rows < n and time.perf_counter() - t0 < budget_s:
        ko.g(X[rows:rows + chunk], C0)
        rows += min(chunk, n - rows)
    dt = time.perf_counter() - t0
    pass_s = dt * n / rows
    solves_per_s = 1.0 / (pass_s * passes_per_solve)
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        threads = os.cpu_count()
    return {
        "value": solves_per_s,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"extrapolated, not a timed solve: one oracle G pass (float64 direct differences, "
                   f"assignment+update+energy) timed on the first {rows} of {n} rows in {dt:.1f} s, "
                   f"scaled to a full pass ({pass_s:.2f} s/pass) times the GPU's mean of "
                   f"{passes_per_solve:.1f} assignment passes per solve (a full oracle solve would take "
                   f"about {pass_s * passes_per_solve / 60:.0f} min); single-threaded NumPy on a host with "
                   f"{threads} visible cores"),
        "dist_evals_per_s": rows * C0.shape[0] / dt,
    }


def cpu_full_solve(X, C0, w, seed, gpu_iters, gpu_passes, gpu_E, stored32=False):
    """Time one complete solve of the FP64 oracle (Algorithm 1) from the
    starting centroids of one timed GPU solve; one progress line per
    iteration on stderr.  stored32: the oracle keeps its iterates (the
    fall-back G and every candidate) as float32 values, as the GPU stores
    them; its arithmetic stays float64."""
    from oracle import kmeans_oracle as ko
    t0 = time.perf_counter()

    def progress(t):   # called at the start of each iteration; keeps the oracle's own iterate
        print(f"oracle solve, seed {seed}: iteration {t} at {time.perf_counter() - t0:.0f} s",
              file=sys.stderr, flush=True)
        return None

    f32 = (lambda A: A.astype(np.float32).astype(np.float64)) if stored32 else None
    r = ko.solve(X.astype(np.float64), C0.astype(np.float64), m_max=w["m_max"], tol=w["tol"],
                 max_iter=w["max_iter"], replay=progress, stored=f32, stored_cand=f32)
    dt = time.perf_counter() - t0
    return {
        "value": 1.0 / dt,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one complete oracle solve (float64 direct differences, single-threaded NumPy"
                   f"{', iterates stored as float32' if stored32 else ''}) from the "
                   f"starting centroids of seed {seed}: {r.iters} iterations, {r.assign_passes} assignment "
                   f"passes in {dt:.1f} s; the GPU's solve of the same seed: {gpu_iters} iterations, "
                   f"{gpu_passes} passes"),
        "oracle_iters": r.iters,
        "oracle_passes": r.assign_passes,
        "gpu_iters": gpu_iters,
        "gpu_passes": gpu_passes,
        "energy_rel_diff": abs(gpu_E - r.E) / abs(r.E) if r.E else None,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solver runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "copies": 3}))
        return
    import paper_1805_10638_amd as km
    from paper_1805_10638_amd import synth
    if args.workload == "small":
        small_workload(args, km, synth, torch)
        return
    if args.workload == "precision":
        precision_workload(args, km, synth, torch)
        return
    if args.workload == "batched":
        batched_workload(args, km, synth, torch)
        return
    if args.workload == "served":
        served_workload(args, km, synth, torch)
        return
    if args.workload == "studies":
        studies_workload(args, km, synth, torch)
        return
    if args.workload == "update":
        update_workload(args, km, synth, torch)
        return

    w = WORKLOAD
    X, _ = synth.plain_large(rep=0, n=w["N"], d=w["d"], k=w["K"])
    Xd = torch.from_numpy(X).to("cuda")
    seeds = list(range(args.warmup + args.steps))
    inits = [torch.from_numpy(synth.init_centroids(X, w["K"], s)).to("cuda") for s in seeds]
    Cout = torch.empty((w["K"], w["d"]), dtype=torch.float32, device="cuda")
    rho = torch.empty(w["N"], dtype=torch.int32, device="cuda")
    ctx = km.Context(0)

    def solve(C0):
        return km.kmeans_solve(Xd, C0, m_max=w["m_max"], tol=w["tol"], max_iter=w["max_iter"],
                               ctx=ctx, out=(Cout, rho), bounds=bool(args.bounds))

    for s in range(args.warmup):
        solve(inits[s])
    ctx.set_timing(True)
    torch.cuda.synchronize()
    lat, iters, passes, acc, rej, flagged, assign_ms, assign_n = [], [], [], [], [], [], 0.0, 0
    gemm_rows = []
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        ts = time.perf_counter()
        _, _, E, it, st = solve(inits[s])
        lat.append(time.perf_counter() - ts)
        if s == args.warmup:
            first = (it, st.assign_passes, E)
        iters.append(it)
        passes.append(st.assign_passes)
        acc.append(st.accepted)
        rej.append(st.rejected)
        flagged.append(st.recheck_rows)
        gemm_rows.append(st.gemm_rows)
        assign_ms += st.assign_ms
        assign_n += st.assign_launches
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # With row bounds the candidate launches mostly filter rows; beside them,
    # outside the timed region, a few solves without bounds give the dense
    # pass (all N rows through the MFMA GEMM) its own roofline.
    dense = None
    if args.bounds:
        d_ms, d_n = 0.0, 0
        for s in range(args.warmup, args.warmup + min(3, args.steps)):
            st = km.kmeans_solve(Xd, inits[s], m_max=w["m_max"], tol=w["tol"], max_iter=w["max_iter"],
                                 ctx=ctx, out=(Cout, rho), bounds=False)[4]
            d_ms += st.assign_ms
            d_n += st.assign_launches
        torch.cuda.synchronize()
        d_s = (d_ms / 1e3) / max(d_n, 1)
        d_flops = 2.0 * w["N"] * w["K"] * w["d"]
        dense = {"kernel": "assignment without bounds (all rows through the GEMM, candidate role)",
                 "bound": "mfma", "achieved": d_flops / d_s / 1e12, "peak": FP32_MFMA_PEAK_TFLOPS,
                 "unit": "TFLOP/s", "frac": d_flops / d_s / 1e12 / FP32_MFMA_PEAK_TFLOPS,
                 "traffic": TRAFFIC_BYTES_PER_LAUNCH, "avg_launch_us": d_s * 1e6, "launches": d_n,
                 "flop_per_launch": d_flops}
    ctx.set_timing(False)

    N, d, K = w["N"], w["d"], w["K"]
    solves_per_s = args.steps / elapsed
    dist_evals = sum(passes) * N * K
    avg_assign_s = (assign_ms / 1e3) / max(assign_n, 1)
    # rows through the distance GEMM per pass (N without bounds; with bounds
    # the mean over the passes after the first, which always assigns all rows)
    rows_per_pass = (sum(gemm_rows) - N * len(gemm_rows)) / max(sum(passes) - len(passes), 1)
    flops = 2.0 * rows_per_pass * K * d
    achieved = flops / avg_assign_s / 1e12
    lat_ms = sorted(x * 1e3 for x in lat)

    def pct(p):
        i = min(len(lat_ms) - 1, max(0, int(round(p / 100.0 * (len(lat_ms) - 1)))))
        return lat_ms[i]

    out = {
        "metric": "Lloyd+AA solves/s, p50/p99 latency; dist-evals/s & % roofline vs FP32",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "gaussian-mixture N=1000000 d=32 K=256 float32, random-sample init "
                        "(seed = step index), m_max=10 tol=1e-6 max_iter=500",
            "N": N, "d": d, "K": K, "m_max": w["m_max"], "tol": w["tol"],
            "gemm": "f32 MFMA", "parallelism": "single GPU", "row_bounds": bool(args.bounds),
        },
        "p50_ms": pct(50),
        "p99_ms": pct(99),
        "dist_evals_per_s": dist_evals / elapsed,
        "iters_mean": statistics.mean(iters),
        "assign_passes_mean": statistics.mean(passes),
        "accepted_mean": statistics.mean(acc),
        "rejected_mean": statistics.mean(rej),
        "recheck_rows_per_pass": sum(flagged) / max(sum(passes), 1),
        "roofline": {
            "kernel": ("assignment with row bounds (k_assign_bnd, candidate role; GEMM rows only count)"
                       if args.bounds else "assignment (k_assign, candidate role)"),
            "bound": "mfma",
            "achieved": achieved,
            "peak": FP32_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_MFMA_PEAK_TFLOPS,
            "traffic": TRAFFIC_BYTES_PER_LAUNCH_BND if args.bounds else TRAFFIC_BYTES_PER_LAUNCH,
            "avg_launch_us": avg_assign_s * 1e6,
            "launches": assign_n,
            "flop_per_launch": flops,
            "gemm_rows_per_pass": rows_per_pass,
        },
    }
    if dense is not None:
        out["roofline_dense"] = dense
    if args.cpu_full_solve:
        out["cpu_baseline"] = cpu_full_solve(X, synth.init_centroids(X, K, args.warmup), w, args.warmup, *first,
                                             stored32=args.cpu_full_solve == "f32")
    elif not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, synth.init_centroids(X, K, 0),
                                           statistics.mean(passes), args.cpu_seconds)
    print(json.dumps(out), flush=True)


BF16_MFMA_PEAK_TFLOPS = 2516.6   # MI355X dense bf16 matrix peak


def _pct(v, p):
    v = sorted(v)
    return v[min(len(v) - 1, max(0, int(round(p / 100.0 * (len(v) - 1)))))] if v else None


def small_workload(args, km, synth, torch):
    """Many small solves: N=10,000, d=2, K=10 (the plain small mixture), one
    instance per seed s (data rep s, init seed s), Lloyd (m_max=0) and
    Anderson (m_max=10, m_init=2), tol=1e-6, max_iter=500.  Each GPU solve is
    timed on the host around the call (X and C0 already on the device), so the
    latency includes the binding and the final copies.  Beside it the float64
    oracle solves the same inputs on the host CPU, each timed the same way;
    every GPU result is compared with the oracle's (iterations, accepted
    count, energy to 1e-6 relative)."""
    from oracle import kmeans_oracle as ko
    seeds = list(range(args.seeds))
    K = 10
    host = [synth.plain_small(rep=s)[0] for s in seeds]
    inits = [synth.init_centroids(x, K, s) for s, x in zip(seeds, host)]
    Xd = [torch.from_numpy(x).to("cuda") for x in host]
    Cd = [torch.from_numpy(c).to("cuda") for c in inits]
    ctx = km.Context(0)
    for j in range(3):                                   # warm-up (code objects, workspace)
        km.kmeans_solve(Xd[j], Cd[j], m_max=10, tol=1e-6, ctx=ctx)
    torch.cuda.synchronize()
    res = {}
    for mode, m_max in (("lloyd", 0), ("aa", 10)):
        lat, its, Es, acc = [], [], [], []
        t0 = time.perf_counter()
        for j in range(len(seeds)):
            ts = time.perf_counter()
            _, _, E, it, st = km.kmeans_solve(Xd[j], Cd[j], m_max=m_max, tol=1e-6, ctx=ctx)
            lat.append((time.perf_counter() - ts) * 1e3)
            its.append(it)
            Es.append(E)
            acc.append(st.accepted)
        wall = time.perf_counter() - t0
        clat, cits, mism, differ = [], [], 0, []
        ct0 = time.perf_counter()
        for j in range(len(seeds)):
            ts = time.perf_counter()
            r = ko.solve(host[j].astype(np.float64), inits[j].astype(np.float64), m_max=m_max, tol=1e-6)
            clat.append((time.perf_counter() - ts) * 1e3)
            cits.append(r.iters)
            if r.iters != its[j] or r.accepted != acc[j] or abs(r.E - Es[j]) > 1e-6 * abs(r.E):
                mism += 1
                differ.append(j)
        cwall = time.perf_counter() - ct0
        # seeds that differ again, with the oracle storing its iterates in
        # float32 as the GPU does (decisions near a threshold, e.g. the
        # tol = 1e-6 stop, can flip on float32 rounding of the centroids)
        f32 = lambda A: A.astype(np.float32).astype(np.float64)   # noqa: E731
        mism32, e_rel = 0, 0.0
        for j in differ:
            r = ko.solve(host[j].astype(np.float64), inits[j].astype(np.float64), m_max=m_max, tol=1e-6,
                         stored=f32, stored_cand=f32)
            e_rel = max(e_rel, abs(r.E - Es[j]) / abs(r.E))
            if r.iters != its[j] or r.accepted != acc[j] or abs(r.E - Es[j]) > 1e-6 * abs(r.E):
                mism32 += 1
        res[mode] = {"solves_per_s": len(seeds) / wall, "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
                     "iters_mean": statistics.mean(its),
                     "oracle_cpu": {"solves_per_s": len(seeds) / cwall, "p50_ms": _pct(clat, 50),
                                    "p99_ms": _pct(clat, 99), "iters_mean": statistics.mean(cits),
                                    "cores": 1},
                     "seeds_differing_from_oracle": mism,
                     "seeds_differing_from_oracle_with_float32_iterates": mism32,
                     "max_E_rel_diff_of_those": e_rel}
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        threads = os.cpu_count()
    print(json.dumps({
        "metric": "small solves: solves/s and p50/p99 latency, Lloyd and Anderson, GPU vs float64 oracle on CPU",
        "value": res["aa"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "data": "synthetic",
        "config": {"workload": f"gaussian-mixture N=10000 d=2 K=10 (10 unit-variance components, centres "
                               f"U[-10,10]^2), {len(seeds)} seeds, random-sample init, tol=1e-6 max_iter=500; "
                               "Lloyd = m_max 0, Anderson = m_max 10 m_init 2",
                   "N": 10000, "d": 2, "K": K, "seeds": len(seeds)},
        "results": res,
        "oracle_note": f"single-threaded NumPy float64 (direct differences, no BLAS) on a host with "
                       f"{threads} visible cores",
    }), flush=True)


def update_workload(args, km, synth, torch):
    """The update step (Eq. (4): cluster sums and sizes, means) against the
    HBM roofline.  kmeans_g at N=1e7, d=16, K=256 (X is 640 MB, more than the
    256 MB last-level cache) and at N=1e6, d=32, K=256, each applied
    repeatedly at the centroids of one Lloyd step from a seeded random-sample
    start; device time of the update from HIP events (both shapes take the
    fixed-point sums; the one pass over X that bounds |x| is computed once per
    X and is not part of the update).
    Algorithmic bytes per update, the least any update moves: N*d*4 (X read
    once) + 4*N (labels read once) + 4*K*d (float32 means written)."""
    res = {}
    reps = max(3, args.steps)
    for N, d, K in ((10_000_000, 16, 256), (1_000_000, 32, 256)):
        X, C0 = synth.device_instance(N, d, K, seed=0)
        ctx = km.Context(0)
        ctx.set_timing(True)
        _, C, _, _ = km.kmeans_g(X, C0, ctx=ctx)
        upd, asg = [], []
        for _ in range(reps):
            _, _, _, st = km.kmeans_g(X, C, ctx=ctx)
            upd.append(st.update_ms)
            asg.append(st.assign_ms)
        u_ms = statistics.median(upd)
        nbytes = N * d * 4 + 4 * N + 4 * K * d
        gbs = nbytes / (u_ms / 1e3) / 1e9
        res[f"N{N}_d{d}_K{K}"] = {"update_ms": u_ms, "assign_ms": statistics.median(asg),
                                  "algorithmic_bytes": nbytes, "achieved_GBs": gbs,
                                  "peak_GBs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS, "reps": reps}
        del X, C0, C, ctx
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "update step: algorithmic bytes per second vs HBM peak", "unit": "GB/s",
                      "data": "synthetic", "dtype": "i64 fixed-point sums of f32 rows",
                      "config": {"workload": "kmeans_g on gaussian mixtures (centres N(0,25I), std U[0.5,2], "
                                             "Dirichlet(1) weights), random-sample init, one Lloyd step, then "
                                             "repeated G at those centroids"},
                      "results": res}), flush=True)


def precision_workload(args, km, synth, torch):
    """N=4,000,000, d=128, K=1024 with X stored as bfloat16: time to converge
    with the float32 and the bfloat16 distance GEMM from the same C0, the
    assignment kernel against its roofline, and the error of each result
    against the float64 oracle:
      * labels: the result's labels against the oracle's assignment at the
        result's centroids on 20,000 sampled rows (mismatches outside oracle
        near ties, and the near ties);
      * energy: |E - E_oracle| / E_oracle with E_oracle the float64 energy of
        the result's labels at its centroids over all N rows;
      * centroids: one more kmeans_g at the result's centroids (same GEMM)
        against the oracle's means of its labels, max over all K centroids of
        ||dc_j|| / max(||c_j||, s_X) (s_X the RMS spread of X), and its
        energy against the oracle's;
      * flagged (re-checked) rows per assignment pass."""
    from oracle import kmeans_oracle as ko
    N, d, K = 4_000_000, 128, 1024
    Xb, _ = synth.precision(rep=0, n=N, d=d, k=K)
    Xd = torch.from_numpy(Xb.view(np.int16)).to("cuda")
    steps = max(1, min(args.steps, 3))
    inits = [torch.from_numpy(synth.init_centroids(Xb, K, s)).to("cuda") for s in range(steps + 1)]
    ctx = km.Context(0)
    rows = np.sort(np.random.default_rng(7).choice(N, 20000, replace=False))
    X64 = synth.bf16_bits_to_f32(Xb).astype(np.float64)
    sX = float(np.sqrt(((X64 - X64.mean(axis=0)) ** 2).sum(axis=1).mean()))

    def energy_all(lab, C):
        tot = 0.0
        for a in range(0, N, 500_000):
            tot += ko.energy(X64[a:a + 500_000], lab[a:a + 500_000], C)
        return tot

    res = {}
    for prec, peak in (("f32", FP32_MFMA_PEAK_TFLOPS), ("bf16", BF16_MFMA_PEAK_TFLOPS)):
        km.kmeans_solve(Xd, inits[0], m_max=10, tol=1e-6, prec=prec, ctx=ctx, max_iter=3)  # warm-up
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = []
        for s in range(1, steps + 1):
            outs.append(km.kmeans_solve(Xd, inits[s], m_max=10, tol=1e-6, prec=prec, ctx=ctx))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.set_timing(False)
        C, rho, E, it, st = outs[-1]
        print(f"[precision] {prec}: {steps} solves in {el:.2f} s; oracle checks", file=sys.stderr, flush=True)
        a_ms = sum(o[4].assign_ms for o in outs) / max(1, sum(o[4].assign_launches for o in outs))
        ach = 2.0 * N * K * d / (a_ms / 1e3) / 1e12
        Cn = C.cpu().numpy().astype(np.float64)
        lab_all = rho.cpu().numpy().astype(np.int64)
        a = ko.assign(X64[rows], Cn)
        lab = lab_all[rows]
        mism = int(((a.rho != lab) & ~a.near_tie).sum())
        E_or = energy_all(lab_all, Cn)
        # G at the result: labels, means and energy against the oracle
        rho_g, C_g, E_g, gst = km.kmeans_g(Xd, C, prec=prec, ctx=ctx)
        lab_g = rho_g.cpu().numpy().astype(np.int64)
        Co, _ = ko.update(X64, lab_g, Cn)
        cerr = np.linalg.norm(C_g.cpu().numpy().astype(np.float64) - Co, axis=1) / \
            np.maximum(np.linalg.norm(Co, axis=1), sX)
        E_or_g = energy_all(lab_g, Cn)
        res[prec] = {"solves_per_s": steps / el, "time_to_converge_ms": el * 1e3 / steps,
                     "iters": it, "assign_passes": st.assign_passes, "E": E,
                     "assign_avg_us": a_ms * 1e3, "assign_tflops": ach, "peak_tflops": peak,
                     "frac": ach / peak, "recheck_rows_per_pass": st.recheck_rows / st.assign_passes,
                     "oracle_errors": {
                         "label_mismatch_outside_near_ties_sampled": mism,
                         "label_near_ties_sampled": int(a.near_tie.sum()),
                         "label_sample_rows": int(rows.size),
                         "energy_rel_err": abs(E - E_or) / E_or,
                         "g_labels_equal_result": bool((lab_g == lab_all).all()),
                         "g_energy_rel_err": abs(E_g - E_or_g) / E_or_g,
                         "g_max_rel_centroid_err": float(cerr.max()),
                         "g_recheck_rows": gst.recheck_rows, "g_near_tie_rows": gst.near_tie_rows}}
    ef, eb = res["f32"]["E"], res["bf16"]["E"]
    print(json.dumps({"metric": "precision mode: time to converge, f32 vs bf16 distance GEMM",
                      "config": {"workload": "gaussian-mixture N=4000000 d=128 K=1024, 5% outliers, "
                                             "X stored bfloat16, m_max=10 tol=1e-6",
                                 "N": N, "d": d, "K": K},
                      "steps": steps, "results": res,
                      "bf16_speedup": res["bf16"]["solves_per_s"] / res["f32"]["solves_per_s"],
                      "energy_rel_diff_bf16_vs_f32": abs(eb - ef) / ef}), flush=True)


def batched_workload(args, km, synth, torch):
    """Many uneven instances (N log-uniform in [2e3, 2e5], d in {3, 16, 64},
    K log-uniform in [8, 512], float32, per-instance seeded init) solved by
    one batched engine run, against the same instances solved one at a time
    with kmeans_solve.  Both use the tuned tile shapes."""
    n_inst = args.instances
    sizes = synth.instance_sizes(n_inst, rep=0)
    probs = [synth.device_instance(n, d, k, seed=i) for i, (n, d, k) in enumerate(sizes)]
    torch.cuda.synchronize()
    ctx = km.Context(0)
    kw = dict(m_max=10, tol=1e-6, max_iter=500)
    km.kmeans_solve_batch(probs[:8], ctx=ctx, **kw)          # warm-up (code objects, pools)
    for X, C0 in probs[:8]:
        km.kmeans_solve(X, C0, ctx=ctx, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = km.kmeans_solve_batch(probs, ctx=ctx, **kw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    solo = []
    for X, C0 in probs:
        _, _, E, it, st = km.kmeans_solve(X, C0, ctx=ctx, **kw)
        solo.append((E, it, st.assign_passes))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    flops = sum(2.0 * n * k * d * r[2].assign_passes for (n, d, k), r in zip(sizes, out))
    dist = sum(float(n) * k * r[2].assign_passes for (n, d, k), r in zip(sizes, out))
    it_mismatch = sum(int(r[2].iters != s[1]) for r, s in zip(out, solo))
    e_rel = max(abs(r[2].E - s[0]) / max(abs(s[0]), 1e-300) for r, s in zip(out, solo))
    ach = flops / t_batch / 1e12
    print(json.dumps({
        "metric": "batched: instances solved per second, one engine vs one at a time",
        "value": n_inst / t_batch, "unit": "solves/s", "n_gpus": 1, "data": "synthetic",
        "config": {"workload": f"{n_inst} gaussian-mixture instances, N log-uniform [2e3,2e5], "
                               "d in {3,16,64}, K log-uniform [8,512], float32, m_max=10 tol=1e-6",
                   "total_rows": int(sum(n for n, _, _ in sizes)),
                   "tuned_shape_entries": ctx.tuned_entries},
        "batched_s": t_batch, "one_at_a_time_s": t_seq, "one_at_a_time_solves_per_s": n_inst / t_seq,
        "speedup": t_seq / t_batch,
        "iters_mean": statistics.mean(r[2].iters for r in out),
        "iters_mismatch_vs_solo": it_mismatch, "max_E_rel_diff_vs_solo": e_rel,
        "assign_flop": flops, "dist_evals_per_s": dist / t_batch,
        "assignment_tflops_over_run": ach, "frac_fp32_mfma_peak_over_run": ach / FP32_MFMA_PEAK_TFLOPS,
    }), flush=True)


def served_workload(args, km, synth, torch):
    """Poisson arrivals (rate per second, for `duration` seconds) of jobs
    sized like the batched mix, plus 2 % large jobs (N=2e6, d=96, K=2048,
    bfloat16 X, bfloat16 GEMM).  Each job's data is generated on the device
    when it arrives (excluded from its latency); the engine (or, with
    --engines 2, one per size class, large jobs on at most 3/4 of the
    assignment workgroups) admits jobs under a 200 GB workspace budget while
    others run, stepped without blocking from one host loop.  The baseline runs
    the same jobs through a FIFO loop of float32 kmeans_solve calls, one at
    a time, with latency = finish - arrival."""
    rng = np.random.default_rng([180510638, 5, 0])
    arrivals = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / args.rate)
        if t > args.duration:
            break
        arrivals.append(t)
    n = len(arrivals)
    small = synth.instance_sizes(n, rep=0, cfg=5)
    large = rng.random(n) < 0.02
    spec = [((2_000_000, 96, 2048, True) if large[i] else (*small[i], False)) for i in range(n)]

    def make(i):
        nn, d, k, bf = spec[i]
        return synth.device_instance(nn, d, k, seed=10_000 + i, bf16=bf)

    ctx = km.Context(0)
    kw = dict(m_max=10, tol=1e-6, max_iter=500)
    # two size classes, each its own engine and stream: large bfloat16 jobs
    # take at most 3/4 of the assignment workgroups so small jobs keep moving
    budget = 200 * 10**9
    if args.engines == 2:
        eng_s = km.Engine(hbm_budget=budget // 4, graphs=False, ctx=ctx, **kw)
        eng_l = km.Engine(hbm_budget=budget - budget // 4, graphs=False, ctx=ctx, prec="bf16", **kw)
        eng_l.set_share(0.75)
        engines = (eng_s, eng_l)
    else:
        eng_s = eng_l = km.Engine(hbm_budget=budget, graphs=False, ctx=ctx, **kw)
        engines = (eng_s,)

    def route(i):
        return eng_l if spec[i][3] else eng_s

    warm = 0                                        # warm-up jobs, not timed
    for i in range(n):
        if warm == 3:
            break
        if i < 2 or spec[i][3]:
            X, C0 = make(i)
            route(i).submit(X, C0, prec="bf16" if spec[i][3] else "f32")
            warm += 1
    while warm > 0:
        for e in engines:
            e.step()
            warm -= len(e.poll())

    lat, lag, lat_large, lat_small = [], [], [], []
    t_sub = {}
    fin_at = [0.0] * n                               # finish time of each job (s after the start)
    keep = {}                                        # sampled small jobs kept for the oracle check
    sample = set(j for j in range(n) if not spec[j][3] and spec[j][0] * spec[j][1] * spec[j][2] <= 5e7)
    sample = set(sorted(sample)[len(sample) // 4::max(1, len(sample) // 3)][:3])
    backlog_at_end = None
    t_start = time.perf_counter()
    i = done = 0
    next_note = 10.0
    while done < n:
        now = time.perf_counter() - t_start
        while i < n and arrivals[i] <= now:
            X, C0 = make(i)
            e = route(i)
            tk = e.submit(X, C0, prec="bf16" if spec[i][3] else "f32")
            t_sub[(id(e), tk)] = (i, time.perf_counter())
            lag.append(time.perf_counter() - t_start - arrivals[i])
            i += 1
        busy = 0
        for e in engines:
            a, q, _ = e.step(wait=False)
            busy += a + q
            for tk, C, rho, res in e.poll():
                j, ts = t_sub.pop((id(e), tk))
                dt = (time.perf_counter() - ts) * 1e3
                lat.append(dt)
                (lat_large if spec[j][3] else lat_small).append(dt)
                fin_at[j] = time.perf_counter() - t_start
                if j in sample:
                    keep[j] = (C.cpu().numpy(), rho.cpu().numpy(), res)
                done += 1
        if backlog_at_end is None and i == n:
            backlog_at_end = n - done
        if now >= next_note:
            print(f"served: t={now:.0f} s, {i} arrived, {done} done", file=sys.stderr, flush=True)
            next_note += 10.0
        if busy == 0 and i < n:
            time.sleep(max(0.0, min(0.002, arrivals[i] - (time.perf_counter() - t_start))))
    t_served = time.perf_counter() - t_start
    print(f"served: {n} jobs in {t_served:.1f} s", file=sys.stderr, flush=True)
    for e in engines:
        e.close()
    # served results against the float64 oracle (a few small jobs; their data
    # is regenerated from the same seeded device generator)
    from oracle import kmeans_oracle as ko
    o_mism = 0
    for j, (Cj, rj, res) in sorted(keep.items()):
        X, C0 = make(j)
        r = ko.solve(X.cpu().numpy().astype(np.float64), C0.cpu().numpy().astype(np.float64), m_max=10, tol=1e-6)
        if r.iters != res.iters or abs(r.E - res.E) > 1e-6 * abs(r.E) or \
                np.abs(Cj.astype(np.float64) - r.C).max() > 1e-4 * max(1.0, np.abs(r.C).max()):
            o_mism += 1
        del X, C0

    # FIFO baseline: float32 GEMM, one job at a time, in arrival order
    fin = 0.0
    base_lat = []
    busy = 0.0
    print(f"served: {len(keep)} results checked against the oracle, {o_mism} mismatched; "
          "FIFO baseline next", file=sys.stderr, flush=True)
    for j in range(n):
        if j % 2000 == 0:
            print(f"FIFO baseline: job {j} of {n}", file=sys.stderr, flush=True)
        X, C0 = make(j)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        km.kmeans_solve(X, C0, ctx=ctx, prec="f32", **kw)
        torch.cuda.synchronize()
        dur = time.perf_counter() - t0
        busy += dur
        start = max(arrivals[j], fin)
        fin = start + dur
        base_lat.append((fin - arrivals[j]) * 1e3)
        del X, C0

    def pct(v, p):
        v = sorted(v)
        return v[min(len(v) - 1, max(0, int(round(p / 100.0 * (len(v) - 1)))))] if v else None

    print(json.dumps({
        "metric": "served: p50/p99 latency and solves/s, continuous batching vs FIFO float32",
        "value": n / t_served, "unit": "solves/s", "n_gpus": 1, "data": "synthetic",
        "config": {"workload": f"Poisson {args.rate:g} jobs/s for {args.duration:g} s; sizes as the batched "
                               "mix, 2% large (N=2e6 d=96 K=2048 bfloat16 X, bfloat16 GEMM); HBM budget 200 GB",
                   "jobs": n, "large_jobs": int(large.sum()), "engines": args.engines},
        "served": {"solves_per_s": n / t_served, "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                   "small_p50_ms": pct(lat_small, 50), "small_p99_ms": pct(lat_small, 99),
                   "large_p50_ms": pct(lat_large, 50), "large_p99_ms": pct(lat_large, 99),
                   "mean_submit_lag_ms": 1e3 * statistics.mean(lag),
                   "arrival_rate": n / args.duration, "keeps_up": n / t_served >= 0.98 * n / args.duration,
                   "unfinished_when_arrivals_end": backlog_at_end,
                   "drain_after_arrivals_s": t_served - args.duration,
                   "oracle_checked_jobs": len(keep), "oracle_mismatches": o_mism},
        "fifo_f32": {"solves_per_s": n / fin, "p50_ms": pct(base_lat, 50), "p99_ms": pct(base_lat, 99),
                     "busy_s": busy},
    }), flush=True)


STUDY_SETS = [  # (name, N, d, mixture components)
    ("mix2d", 200_000, 2, 50), ("mix8d", 1_000_000, 8, 128), ("mix16d", 200_000, 16, 64),
    ("mix32d", 500_000, 32, 256), ("mix64d", 200_000, 64, 32), ("mix128d", 200_000, 128, 64),
]


def studies_workload(args, km, synth, torch):
    """Synthetic analogues of the paper's two experiments (its datasets are
    not available): (1) fixed m vs dynamic m with m initialised to 2 and 5,
    m_max = 30, eps1 = 0.02, eps2 = 0.5 (Sec. 3.1), reporting time and
    accepted/total iterations; (2) Lloyd vs Anderson (dynamic m) for K = 10,
    100, 1000 from the same random-sample initialisation, reporting
    iterations, time and final mean squared error (Sec. 3.2).  Both run to
    convergence (tol = 0: no assignment changes, as the paper does) and with
    the benchmark's stopping rule (tol = 1e-6 relative energy change).
    Times are whole GPU solves (median of 3)."""
    for tol in (0.0, 1e-6):
        _studies(args, km, synth, torch, tol)


def _studies(args, km, synth, torch, tol):
    ctx = km.Context(0)
    data = [(name, *synth.device_instance(n, d, comps, seed=7 + i)) for i, (name, n, d, comps) in
            enumerate(STUDY_SETS)]
    torch.cuda.synchronize()

    def run(X, C0, **kw):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, E, it, st = km.kmeans_solve(X, C0, ctx=ctx, max_iter=500, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return {"ms": 1e3 * statistics.median(ts), "iters": it, "accepted": st.accepted, "E": E}

    km.kmeans_solve(data[0][1], data[0][1][:10].contiguous(), ctx=ctx, max_iter=5)   # warm-up
    m_rows = []
    for i, (name, X, _) in enumerate(data):
        K = STUDY_SETS[i][3]
        C0 = X[torch.from_numpy(synth.init_indices(X.shape[0], K, 11 + i)).to(X.device)].contiguous()
        row = {"set": name, "N": X.shape[0], "d": X.shape[1], "K": K}
        for m0 in (2, 5):
            row[f"fixed_m{m0}"] = run(X, C0, m_max=30, m_init=m0, fixed_m=True, tol=tol)
            row[f"dynamic_m{m0}"] = run(X, C0, m_max=30, m_init=m0, tol=tol)
        m_rows.append(row)
        print(json.dumps({"study": "fixed_vs_dynamic_m", "tol": tol, **row}), flush=True)
    k_rows = []
    for i, (name, X, _) in enumerate(data):
        for K in (10, 100, 1000):
            C0 = X[torch.from_numpy(synth.init_indices(X.shape[0], K, 31 + i)).to(X.device)].contiguous()
            lloyd = run(X, C0, m_max=0, tol=tol)
            aa = run(X, C0, m_max=30, m_init=2, tol=tol)
            # the printed return: stop as soon as any candidate repeats the assignment
            lit = run(X, C0, m_max=30, m_init=2, tol=tol, literal_return=True)
            n = X.shape[0]
            row = {"set": name, "N": n, "d": X.shape[1], "K": K,
                   "lloyd": {**lloyd, "mse": lloyd["E"] / n}, "aa": {**aa, "mse": aa["E"] / n},
                   "aa_printed_return": {**lit, "mse": lit["E"] / n},
                   "time_ratio": aa["ms"] / lloyd["ms"], "time_ratio_printed_return": lit["ms"] / lloyd["ms"]}
            k_rows.append(row)
            print(json.dumps({"study": "lloyd_vs_aa", "tol": tol, **row}), flush=True)
    wins = sum(1 for r in k_rows if r["time_ratio"] < 1.0)
    wins_lit = sum(1 for r in k_rows if r["time_ratio_printed_return"] < 1.0)
    dyn_better = sum(1 for r in m_rows for m0 in (2, 5) if r[f"dynamic_m{m0}"]["ms"] < r[f"fixed_m{m0}"]["ms"])
    print(json.dumps({"study": "summary", "tol": tol, "aa_faster_than_lloyd": f"{wins}/{len(k_rows)}",
                      "aa_printed_return_faster_than_lloyd": f"{wins_lit}/{len(k_rows)}",
                      "mean_time_ratio_aa_over_lloyd": statistics.mean(r["time_ratio"] for r in k_rows),
                      "dynamic_faster_than_fixed": f"{dyn_better}/{2 * len(m_rows)}"}), flush=True)


if __name__ == "__main__":
    main()
