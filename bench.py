#!/usr/bin/env python3
"""Benchmark: t-SVT/s of TNN-C completion at 256 x 256 x 31 on one MI355X.

One step = one iteration of Algorithm 1 (ADMM) on the multispectral-shaped
workload: Z = X - M/beta, forward DCT along tubes, one-sided Jacobi SVD of all
31 transformed slices, soft-threshold, rebuild, inverse DCT, X- and M-updates.
Each step performs exactly one t-SVT, so steps/s = t-SVT/s.

Workload (synthetic, seeded): tubal-rank-10 DCT t-product of N(0,1) factors
256x10x31 and 10x256x31, min-max scaled to [0,1]; 30% of entries observed
(Bernoulli mask); tau decays geometrically from 10 to 0.1 over the 100
iterations of the run, beta_l = 1/tau_l.  Inputs are resident in HBM before
timing starts; the library's own t-product builds the tensor on the GPU.

`value` is the mixed-precision path (BF16 hi+lo transforms, FP32 Jacobi
sweeps with FP64 angles, one FP64 sweep); the plain FP64 path is reported
beside it.  Also reported: cold single t-SVT rates, the uneven 64-tensor batch
and the serving stream (p50/p99 latency at a fixed request rate).

Prints one JSON line (progress goes to stderr).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N1, N2, N3, RANK, SR, L_FULL = 256, 256, 31, 10, 0.3, 100
PEAK = {"fp64_alu": 78.6, "fp32_alu": 157.3, "hbm_GBs": 8000.0}


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paths", default="mixed,fp64")
    ap.add_argument("--no-extras", action="store_true", help="skip cold t-SVT, batch and serving measurements")
    ap.add_argument("--serving-requests", type=int, default=60)
    ap.add_argument("--serving-loads", default="0.5,0.8", help="fractions of the measured saturation throughput")
    ap.add_argument("--warm-period", type=int, default=-1,
                    help="completion warm start: -1 automatic, 0 cold starts, N: reset every N iterations")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (hardware-counter scale for profiling runs)")
    return ap.parse_args()


def gpu_tprod_factory(tm, torch):
    def gpu_tprod(F1, F2):
        a = torch.from_numpy(np.asfortranarray(F1)).to("cuda:0")
        b = torch.from_numpy(np.asfortranarray(F2)).to("cuda:0")
        z = tm.tprod_dct(a, b)
        torch.cuda.synchronize()
        return np.asfortranarray(z.cpu().numpy())
    return gpu_tprod


def run_completion(tm, torch, case, prec, steps, warmup, profile, warm_period=-1):
    dt = torch.float64 if prec == tm.FP64 else torch.float32
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_WARM_START, warm_period)
    B = torch.from_numpy(case.B).to(dt).to("cuda:0")
    mask = torch.from_numpy(case.mask).to("cuda:0")
    taus = list(case.taus) + [case.taus[-1]] * max(0, steps + warmup + 1 - len(case.taus))
    if warmup > 0:
        tm.complete_tensor(B, mask, max_iter=warmup, tol=0.0, tau_schedule=taus, prec=prec, ctx=ctx)
    torch.cuda.synchronize()
    ctx.set_option(tm.OPT_PROFILE, int(profile))  # 0 off, 1 every phase, 2 Jacobi launches only
    ctx.stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, info, M = tm.complete_tensor(B, mask, max_iter=steps, tol=0.0, tau_schedule=taus, prec=prec, ctx=ctx,
                                    return_M=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ctx.stats(reset=True)
    with_v = ctx.get_option(tm.OPT_WARM_START) != 0
    tile = dict(ctx.tile(prec, N1, N2, N3, with_v=with_v), with_v=with_v)
    Xn = X.detach().cpu().to(torch.float64).numpy()
    # the next iteration's t-SVT input, Z = X - M / beta (Algorithm 1, first step)
    beta = 1.0 / taus[steps]
    Zn = (X - M / beta).detach().cpu().to(torch.float64).numpy()
    ctx.close()
    return {"seconds": t1 - t0, "info": info, "stats": st, "X": Xn, "Z_next": Zn, "tau_next": taus[steps], "tile": tile}


def jacobi_roofline(res, prec_name):
    st = res["stats"]
    m, p = max(N1, N2), min(N1, N2)
    # one-sided Jacobi, norms tracked: per column pair one inner product (2m
    # flops) and the rotation of two length-m columns (6m flops), plus the
    # rotation of the two length-p columns of V when the warm start carries V
    # (6p); p(p-1)/2 pairs per sweep.  Units: slice-sweeps (counted on the device).
    with_v = res["tile"].get("with_v", False)
    flops_per_slice_sweep = (8.0 * m + (6.0 * p if with_v else 0.0)) * p * (p - 1) / 2.0
    launches = max(1, st["launches"]["jacobi"])
    avg_ms = st["ms"]["jacobi"] / launches
    flops_per_launch = flops_per_slice_sweep * st["slice_sweeps"] / launches
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    peak = PEAK["fp64_alu"] if prec_name == "fp64" else PEAK["fp32_alu"]
    return {"kernel": "k_jacobi_team", "bound": "alu", "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic_for("jacobi", prec_name),
            "avg_launch_ms": round(avg_ms, 4), "sweeps_per_slice": round(st["slice_sweeps"] / (launches * N3), 2),
            "flops_per_launch": flops_per_launch}


def dct_roofline(res, prec_name):
    # forward transform with the completion prologue: reads X and M, writes
    # Zbar (3 N n3 elements); algorithmic bytes per launch
    st = res["stats"]
    es = 8 if prec_name == "fp64" else 4
    launches = max(1, st["launches"]["forward_transform"])
    avg_ms = st["ms"]["forward_transform"] / launches
    nbytes = 3.0 * N1 * N2 * N3 * es
    achieved = nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"kernel": "k_tube_mfma", "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK["hbm_GBs"],
            "unit": "GB/s", "frac": round(achieved / PEAK["hbm_GBs"], 4), "avg_launch_ms": round(avg_ms, 5),
            "bytes_per_launch": nbytes}


def kernel_source_md5():
    """Hash of the Jacobi kernel's sources (the counters are tied to them)."""
    h = hashlib.md5()
    for f in ("jacobi.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_1902_03070_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(kernel, prec_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken with the kernel sources that are built now; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_completion_256x256x31.json")
    try:
        with open(path) as f:
            t = json.load(f)
        ent = t.get("%s_%s" % (kernel, prec_name))
        if ent and ent.get("kernel_src_md5") == kernel_source_md5():
            return ent["bytes_per_launch"]
    except (OSError, ValueError):
        pass
    return None


def isolated_tsvt(tm, torch, Zh, tau, prec, reps=5):
    """tsvt_dct calls one after another on one resident input."""
    dt = torch.float64 if prec == tm.FP64 else torch.float32
    Z = torch.from_numpy(np.asfortranarray(Zh)).to(dt).to("cuda:0")
    ctx = tm.Context(0)
    tm.tsvt_dct(Z, float(tau), prec=prec, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tm.tsvt_dct(Z, float(tau), prec=prec, ctx=ctx)
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / reps
    ctx.close()
    return {"t_svt_per_s": round(1.0 / dt_s, 2), "ms": round(1e3 * dt_s, 3)}


def batched(tm, torch, tprod):
    import synth

    shapes = synth.batch_shapes(64, synth.SEED_BASE + 4)
    Zs, taus = [], []
    for s in shapes:
        Zs.append(torch.from_numpy(synth.tsvt_case(tprod, s.n1, s.n2, s.n3, s.r, 0.01, s.tau, s.seed).Z)
                  .float().to("cuda:0"))
        taus.append(s.tau)
    ctx = tm.Context(0)
    tm.tsvt_dct_batched(Zs, taus, prec=tm.FP32, ctx=ctx)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tm.tsvt_dct_batched(Zs, taus, prec=tm.FP32, ctx=ctx)
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    ctx.close()
    slices = sum(s.n3 for s in shapes)
    return {"tensors": len(shapes), "slices": slices, "makespan_ms": round(1e3 * dt_s, 2),
            "t_svt_per_s": round(len(shapes) / dt_s, 2), "dtype": "f32",
            "recipe": "n1,n2 ~ U{32..512}, n3 ~ U{8..128}, rank min(n1,n2)/10, t-product + N(0,0.01)"}


def serving(tm, torch, tprod, nreq, loads):
    import synth

    g = np.random.default_rng(synth.SEED_BASE + 5)
    shapes = synth.batch_shapes(nreq, synth.SEED_BASE + 5, cfg_index=5)
    reqs = []
    for j, s in enumerate(shapes):
        if j % 2 == 0:
            Z = synth.tsvt_case(tprod, s.n1, s.n2, s.n3, s.r, 0.01, s.tau, s.seed).Z.astype(np.float32)
            reqs.append(("tsvt", Z, s.tau))
        else:
            cc = synth.completion_case(tprod, s.n1, s.n2, s.n3, s.r, 0.3, 50, s.seed)
            reqs.append(("complete", cc.B.astype(np.float32), cc.mask))
    budget = 64 << 30

    def submit(srv, r):
        if r[0] == "tsvt":
            return srv.submit_tsvt(r[1], r[2])
        return srv.submit_complete(r[1], r[2], 50, 10.0, 0.1)

    def drain(srv, ids):
        got = {}
        while len(got) < len(ids):
            for i in ids:
                if i not in got:
                    r = srv.poll(i)
                    if r is not None:
                        got[i] = r[1]
            time.sleep(0.0005)
        return got

    # saturation: all requests submitted at once
    srv = tm.Server(budget_bytes=budget, max_active=16)
    t0 = time.perf_counter()
    ids = [submit(srv, r) for r in reqs]
    drain(srv, ids)
    sat = len(reqs) / (time.perf_counter() - t0)
    srv.close()
    log("serving saturation %.2f req/s" % sat)
    out = {"requests": len(reqs), "mix": "50% t-SVT / 50% completion (50 iterations, tau 10->0.1), 30% observed",
           "shapes": "n1,n2 ~ U{32..512}, n3 ~ U{8..128}", "saturation_req_per_s": round(sat, 3),
           "budget_bytes": budget, "max_active": 16, "loads": {}}
    # fixed request rates: Poisson arrivals at a fraction of saturation
    for load in loads:
        qps = load * sat
        arrivals = synth.poisson_arrivals(g, qps, len(reqs))
        srv = tm.Server(budget_bytes=budget, max_active=16)
        t0 = time.perf_counter()
        ids = []
        for a, r in zip(arrivals, reqs):
            while time.perf_counter() - t0 < a:
                time.sleep(0.0002)
            ids.append(submit(srv, r))
        got = drain(srv, ids)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat = np.array([got[i][2] - got[i][0] for i in ids]) * 1e3
        kinds = [r[0] for r in reqs]
        lt = np.array([lat[k] for k in range(len(ids)) if kinds[k] == "tsvt"])
        lc = np.array([lat[k] for k in range(len(ids)) if kinds[k] == "complete"])
        pc = lambda a, q: round(float(np.percentile(a, q)), 2)  # noqa: E731
        out["loads"][str(load)] = {
            "qps": round(qps, 3), "p50_ms": pc(lat, 50), "p99_ms": pc(lat, 99),
            "p50_ms_tsvt": pc(lt, 50), "p99_ms_tsvt": pc(lt, 99),
            "p50_ms_complete": pc(lc, 50), "p99_ms_complete": pc(lc, 99),
            "throughput_req_per_s": round(len(ids) / wall, 3), "ticks": st["ticks"], "peak_bytes": st["peak_bytes"]}
        log("serving load %.2f: %s" % (load, out["loads"][str(load)]))
    return out


def video_shaped(tm, torch, tprod, steps):
    """Mixed-precision completion at 144x176x100 (rank 15, 20% observed), with
    its relative difference from the FP64 GPU path on the same input."""
    import synth

    cc = synth.completion_case(tprod, 144, 176, 100, 15, 0.2, 100, synth.SEED_BASE + 3)
    out = {}
    for name, prec in (("mixed", tm.MIXED), ("fp64", tm.FP64)):
        r = run_completion(tm, torch, cc, prec, steps, 2, profile=False)
        out[name] = r
    X64, Xm = out["fp64"]["X"], out["mixed"]["X"]
    return {"shape": [144, 176, 100], "rank": 15, "observed": 0.2, "iterations": steps,
            "t_svt_per_s_mixed": round(steps / out["mixed"]["seconds"], 2),
            "t_svt_per_s_fp64": round(steps / out["fp64"]["seconds"], 2),
            "mixed_rel_err_vs_fp64_gpu": float(np.linalg.norm(Xm - X64) / np.linalg.norm(X64)),
            "recovery_rel_err_mixed": float(np.linalg.norm(Xm - cc.T) / np.linalg.norm(cc.T))}


def cpu_baseline(case):
    import oracle

    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.tsvt_dct(case.B, float(case.taus[0]))
    dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 5), "unit": "t-SVT/s", "cores": 1, "kind": "oracle",
            "sample": "one FP64 oracle t-SVT of the first completion iterate (Z = B, tau = 10) at 256x256x31, "
                      "single thread, %.1f s" % dt}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1902_03070_amd as tm
    import synth

    assert torch.cuda.is_available(), "needs a ROCm GPU"
    tprod = gpu_tprod_factory(tm, torch)
    case = synth.completion_case(tprod, N1, N2, N3, RANK, SR, L_FULL, synth.SEED_BASE + 2)
    paths = args.paths.split(",")
    precs = {"fp64": tm.FP64, "fp32": tm.FP32, "mixed": tm.MIXED}
    results = {}
    for name in paths:
        # events around the Jacobi launches only (each event pair costs a few us of GPU time)
        r = run_completion(tm, torch, case, precs[name], args.steps, args.warmup, profile=2,
                           warm_period=args.warm_period)
        results[name] = r
        log("%s: %.3f s for %d steps (%.3f ms/step), jacobi %.3f ms/launch, slice-sweeps %d" % (
            name, r["seconds"], args.steps, 1e3 * r["seconds"] / args.steps,
            r["stats"]["ms"]["jacobi"] / max(1, r["stats"]["launches"]["jacobi"]), r["stats"]["slice_sweeps"]))
    head = paths[0]
    r = results[head]
    # the phase split comes from a second run of the same workload with events around every phase
    ph = run_completion(tm, torch, case, precs[head], args.steps, args.warmup, profile=1,
                        warm_period=args.warm_period)
    log("%s with events around every phase: %.3f ms/step" % (head, 1e3 * ph["seconds"] / args.steps))
    # the same run replayed as a captured HIP graph (no per-kernel events)
    g = run_completion(tm, torch, case, precs[head], args.steps, 0, profile=False, warm_period=args.warm_period)
    log("%s graph replay: %.3f ms/step" % (head, 1e3 * g["seconds"] / args.steps))
    # the same completion with every Jacobi SVD started cold, for comparison
    cold = run_completion(tm, torch, case, precs[head], args.steps, 1, profile=False, warm_period=0)
    log("%s cold-start SVDs: %.3f ms/step" % (head, 1e3 * cold["seconds"] / args.steps))
    out = {
        "metric": "t-SVT/s at 256x256x31 (mixed vs plain FP64) + p50/p99 latency at fixed QPS",
        "value": round(args.steps / r["seconds"], 3),
        "unit": "t-SVT/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["seconds"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": "TNN-C completion (Algorithm 1), 256x256x31, tubal rank 10, 30%% observed, "
                               "tau 10->0.1 over 100 iterations, path=%s" % head,
                   "n1": N1, "n2": N2, "n3": N3, "rank": RANK, "observed": SR, "iterations": args.steps},
        "roofline": jacobi_roofline(r, head),
        "dct_roofline": dct_roofline(ph, head),
        "phase_ms_per_step": {k: round(v / args.steps, 4) for k, v in ph["stats"]["ms"].items()},
        "phase_run_ms_per_step": round(1e3 * ph["seconds"] / args.steps, 4),
        "graph_replay_ms_per_step": round(1e3 * g["seconds"] / args.steps, 4),
        "jacobi_start": ("warm: V of the previous iteration, reset every %d iterations" % (
            64 if args.warm_period < 0 else args.warm_period)) if args.warm_period != 0 else "cold",
        "cold_start_t_svt_per_s": round(args.steps / cold["seconds"], 3),
    }
    T = case.T
    for name, rr in results.items():
        out.setdefault("paths", {})[name] = {
            "t_svt_per_s": round(args.steps / rr["seconds"], 3),
            "ms_per_step": round(1e3 * rr["seconds"] / args.steps, 4),
            "jacobi_roofline": jacobi_roofline(rr, name),
            "recovery_rel_err": float(np.linalg.norm(rr["X"] - T) / np.linalg.norm(T)),
            "status": rr["info"]["status"], "max_sweeps": rr["info"]["max_sweeps"], "jacobi_tile": rr["tile"],
        }
    if "fp64" in results and head != "fp64":
        X64 = results["fp64"]["X"]
        out["paths"][head]["rel_err_vs_fp64_gpu"] = float(np.linalg.norm(r["X"] - X64) / np.linalg.norm(X64))
        out["speedup_vs_fp64"] = round(results["fp64"]["seconds"] / r["seconds"], 3)
    if not args.no_extras:
        # isolated t-SVTs on the first iterate (Z = B, tau = 10) and on the
        # iterate after the timed run (tau at its end), each path on its own iterate
        iso = {}
        for name in paths:
            iso[name] = {"first_iterate": isolated_tsvt(tm, torch, case.B, case.taus[0], precs[name]),
                         "last_iterate": isolated_tsvt(tm, torch, results[name]["Z_next"], results[name]["tau_next"],
                                                       precs[name])}
        out["isolated_tsvt"] = iso
        log("isolated t-SVT:", iso)
        out["video_shaped"] = video_shaped(tm, torch, tprod, 100)
        log("video-shaped:", out["video_shaped"])
        out["batched"] = batched(tm, torch, tprod)
        log("batched:", out["batched"])
        out["serving"] = serving(tm, torch, tprod, args.serving_requests,
                                 [float(x) for x in args.serving_loads.split(",")])
        log("serving:", out["serving"])
    if args.copy_calibration:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = a.clone()
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
