#!/usr/bin/env python3
"""Benchmark: t-SVT/s at 256 x 256 x 31 on one MI355X.

One step = one t-SVT (Theorem 5: forward DCT along tubes, one-sided Jacobi SVD
of all 31 transformed slices, soft threshold, rebuild, inverse DCT) of an
iterate of the multispectral-shaped completion workload.  The steps alternate
between two fixed inputs, so the work per step does not depend on --steps:
  * Z_0  = B (Algorithm 1's first iterate), tau = 10 (start of the schedule);
  * Z_99 = X_99 - M_99 / beta_99, the input of the schedule's last iteration
    (tau = 0.1), captured once, untimed, from a 99-iteration FP64 completion
    on the GPU.
Every SVD starts cold (no warm start).  Workload (synthetic, seeded):
tubal-rank-10 DCT t-product of N(0,1) factors 256x10x31 and 10x256x31,
min-max scaled to [0,1]; 30% of entries observed (Bernoulli mask); tau decays
geometrically from 10 to 0.1 over 100 iterations, beta_l = 1/tau_l.  Inputs
are resident in HBM before timing starts.

`value` is the mixed-precision path (BF16 hi+lo transforms, FP32 Jacobi
sweeps with FP64 angles, one FP64 sweep); the plain FP64 path is timed the
same way beside it.  Also reported: the whole 100-iteration completion in
situ (warm-started SVDs), the video-shaped completion, the uneven 64-tensor
batch, the serving stream (p50/p99 latency at fixed request rates), and the
FP64 oracle on the host's threads (cpu_baseline).

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
WORKLOAD = ("isolated t-SVT (Theorem 5), 256x256x31, cold Jacobi SVDs, steps alternating between the first "
            "(Z_0 = B, tau 10) and last (Z_99, tau 0.1) iterates of the tubal-rank-10, 30%-observed completion "
            "workload (tau 10->0.1 over 100 iterations)")


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paths", default="mixed,fp64")
    ap.add_argument("--no-extras", action="store_true", help="skip completion, batch and serving measurements")
    ap.add_argument("--serving-requests", type=int, default=60)
    ap.add_argument("--serving-loads", default="0.5,0.8", help="fractions of the measured saturation throughput")
    ap.add_argument("--serving-stream", type=int, default=0,
                    help="only the long serving stream: this many requests per load after the warm-up")
    ap.add_argument("--serving-warmup", type=int, default=200)
    ap.add_argument("--serving-pool", type=int, default=200, help="distinct requests the stream cycles through")
    ap.add_argument("--serving-saturation", type=float, default=0.0,
                    help="saturation throughput (req/s) for the stream's loads; 0 measures it on the pool")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (hardware-counter scale for profiling runs)")
    return ap.parse_args()


def gpu_tprod_factory(tm, torch):
    def gpu_tprod(F1, F2):
        ctx = tm.Context(0)
        a = torch.from_numpy(np.asfortranarray(F1)).to("cuda:0")
        b = torch.from_numpy(np.asfortranarray(F2)).to("cuda:0")
        z = tm.tprod_dct(a, b, ctx=ctx)
        torch.cuda.synchronize()
        out = np.asfortranarray(z.cpu().numpy())
        ctx.close()
        return out
    return gpu_tprod


def capture_last_iterate(tm, torch, case):
    """Z_99 = X_99 - M_99 / beta_99: the t-SVT input of the schedule's last
    iteration, from 99 FP64 iterations of Algorithm 1 on the GPU (untimed)."""
    ctx = tm.Context(0)
    B = torch.from_numpy(case.B).to("cuda:0")
    mask = torch.from_numpy(case.mask).to("cuda:0")
    X, info, M = tm.complete_tensor(B, mask, max_iter=L_FULL - 1, tol=0.0, tau_schedule=list(case.taus), ctx=ctx,
                                    return_M=True)
    Z = (X - M * float(case.taus[L_FULL - 1])).contiguous()
    torch.cuda.synchronize()
    ctx.close()
    return tm.fortran(Z.permute(2, 1, 0).contiguous().permute(2, 1, 0)), info


def jacobi_roofline(st, prec_name, with_v, n3_total):
    """Roofline of the Jacobi kernel from the device's counts and the HIP
    events around its launches.  One-sided Jacobi with tracked norms: per
    column pair an inner product (2m flops) and the rotation of two length-m
    columns (6m), plus the rotation of two length-p columns of V when V is
    carried (6p).  The full iteration takes p(p-1)/2 pairs per sweep; the
    kept-column mode counts the pairs it evaluates (the others cost no flop)."""
    m, p = max(N1, N2), min(N1, N2)
    flops_per_pair = 8.0 * m + (6.0 * p if with_v else 0.0)
    flops_per_slice_sweep = flops_per_pair * p * (p - 1) / 2.0
    launches = max(1, st["launches"]["jacobi"])
    avg_ms = st["ms"]["jacobi"] / launches
    pairs = st.get("pairs", 0)
    if pairs > 0:
        flops_per_launch = flops_per_pair * pairs / launches
    else:
        flops_per_launch = flops_per_slice_sweep * st["slice_sweeps"] / launches
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    peak = PEAK["fp64_alu"] if prec_name == "fp64" else PEAK["fp32_alu"]
    return {"kernel": "k_jacobi_team", "bound": "alu", "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": traffic_for("jacobi_tsvt" if not with_v else "jacobi", prec_name),
            "avg_launch_ms": round(avg_ms, 4), "launches": launches,
            "slice_sweeps": st["slice_sweeps"], "sweeps_per_slice": round(st["slice_sweeps"] / (launches * n3_total), 3),
            "pairs_per_launch": round(pairs / launches, 1), "fallback_slices": st.get("fallback_slices", 0),
            "flops_per_pair": flops_per_pair, "flops_per_slice_sweep": flops_per_slice_sweep,
            "flops_per_launch": flops_per_launch}


def dct_roofline(st, prec_name, launches_per_step=1):
    """Forward transform with the completion prologue: reads X and M, writes
    Zbar (3 N n3 elements per launch, the algorithmic bytes)."""
    es = 8 if prec_name == "fp64" else 4
    launches = max(1, st["launches"]["forward_transform"])
    avg_ms = st["ms"]["forward_transform"] / launches
    nbytes = 3.0 * N1 * N2 * N3 * es
    achieved = nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"kernel": "k_tube_mfma", "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK["hbm_GBs"],
            "unit": "GB/s", "frac": round(achieved / PEAK["hbm_GBs"], 4), "avg_launch_ms": round(avg_ms, 5),
            "bytes_per_launch": nbytes}


def kernel_source_md5():
    """Hash of the Jacobi kernel's sources, jacobi.hip then jacobi.h (the
    counters are tied to them)."""
    h = hashlib.md5()
    for f in ("jacobi.hip", "jacobi.h"):
        with open(os.path.join(ROOT, "paper_1902_03070_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(kernel, prec_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken with the kernel sources that are built now; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_bench_256x256x31.json")
    try:
        with open(path) as f:
            t = json.load(f)
        ent = t.get("%s_%s" % (kernel, prec_name))
        if ent and ent.get("kernel_src_md5") == kernel_source_md5():
            return ent["bytes_per_launch"]
    except (OSError, ValueError):
        pass
    return None


def timed_tsvt(tm, torch, inputs, prec, steps, warmup, kept=1, phases=True):
    """The timed loop: `steps` cold t-SVTs, step i on inputs[i % len(inputs)],
    asynchronous calls on one stream with HIP events around the Jacobi
    launches (the device status is checked after the loop).  kept: the
    kept-column Jacobi with its threshold certificate (1, the library's
    default) or the full iteration (0)."""
    dt = torch.float64 if prec == tm.FP64 else torch.float32
    Zs = [(Z.to(dt), float(tau)) for Z, tau in inputs]
    Zs = [(tm.fortran(Z.permute(2, 1, 0).contiguous().permute(2, 1, 0)), tau) for Z, tau in Zs]
    Ys = [tm.empty_f(N1, N2, N3, dt, "cuda:0") for _ in Zs]
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_KEPT_COLUMNS, kept)
    for i in range(max(warmup, len(Zs))):  # the first calls tune the Jacobi tile
        Z, tau = Zs[i % len(Zs)]
        tm.tsvt_dct(Z, tau, Y=Ys[i % len(Zs)], prec=prec, ctx=ctx)
    torch.cuda.synchronize()
    ctx.set_option(tm.OPT_SYNC_STATUS, 0)
    ctx.set_option(tm.OPT_PROFILE, 2)
    ctx.stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        Z, tau = Zs[i % len(Zs)]
        tm.tsvt_dct(Z, tau, Y=Ys[i % len(Zs)], prec=prec, ctx=ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    status, max_sweeps = ctx.sync_status()
    st = ctx.stats(reset=True)
    tile = ctx.tile(prec, N1, N2, N3)
    # each input alone (per-input time, same context and tile)
    ctx.set_option(tm.OPT_PROFILE, 0)
    per = []
    for Z, tau in Zs:
        reps = 5
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            tm.tsvt_dct(Z, tau, Y=Ys[0], prec=prec, ctx=ctx)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - a) / reps)
    ctx.sync_status()
    phase_ms = None
    if phases:
        # events around every phase (they add a few microseconds each): where a step goes
        ctx.set_option(tm.OPT_PROFILE, 1)
        ctx.stats(reset=True)
        reps = 2 * len(Zs) * 5
        for i in range(reps):
            Z, tau = Zs[i % len(Zs)]
            tm.tsvt_dct(Z, tau, Y=Ys[i % len(Zs)], prec=prec, ctx=ctx)
        ph = ctx.stats(reset=True)
        phase_ms = {k: round(v / reps, 4) for k, v in ph["ms"].items()}
        ctx.set_option(tm.OPT_PROFILE, 0)
    ctx.sync_status()
    ctx.close()
    return {"seconds": t1 - t0, "stats": st, "status": status, "max_sweeps": max_sweeps, "tile": tile,
            "per_input_ms": [round(1e3 * x, 4) for x in per], "phase_ms_per_step": phase_ms}


def run_completion(tm, torch, case, prec, steps, warmup, profile, warm_period=-1):
    """Algorithm 1 in situ: `steps` iterations of the schedule (after an untimed
    warm-up run that tunes the tile), warm-started SVDs by default."""
    dt = torch.float64 if prec == tm.FP64 else torch.float32
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_WARM_START, warm_period)
    B = torch.from_numpy(case.B).to(dt).to("cuda:0")
    mask = torch.from_numpy(case.mask).to("cuda:0")
    taus = list(case.taus)
    if warmup > 0:
        tm.complete_tensor(B, mask, max_iter=warmup, tol=0.0, tau_schedule=taus, prec=prec, ctx=ctx)
    torch.cuda.synchronize()
    ctx.set_option(tm.OPT_PROFILE, int(profile))  # 0 off, 1 every phase, 2 Jacobi launches only
    ctx.stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, info = tm.complete_tensor(B, mask, max_iter=steps, tol=0.0, tau_schedule=taus, prec=prec, ctx=ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ctx.stats(reset=True)
    with_v = ctx.get_option(tm.OPT_WARM_START) != 0
    tile = dict(ctx.tile(prec, N1, N2, N3, with_v=with_v), with_v=with_v)
    Xn = X.detach().cpu().to(torch.float64).numpy()
    ctx.close()
    return {"seconds": t1 - t0, "info": info, "stats": st, "X": Xn, "tile": tile}


def psnr(X, T):
    """Peak signal-to-noise ratio in dB of X against the ground truth T in [0, 1]."""
    mse = float(np.mean((np.clip(X, 0.0, 1.0) - T) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(1.0 / mse)


def completion_in_situ(tm, torch, case):
    out = {}
    for name, prec in (("mixed", tm.MIXED), ("fp64", tm.FP64)):
        r = run_completion(tm, torch, case, prec, L_FULL, 3, profile=2)
        ph = run_completion(tm, torch, case, prec, L_FULL, 0, profile=1) if name == "mixed" else None
        X = r["X"]
        out[name] = {
            "t_svt_per_s": round(L_FULL / r["seconds"], 2), "ms_per_iteration": round(1e3 * r["seconds"] / L_FULL, 4),
            "jacobi_roofline": jacobi_roofline(r["stats"], name, True, N3),
            "recovery_rel_err": float(np.linalg.norm(X - case.T) / np.linalg.norm(case.T)),
            "psnr_db": round(psnr(X, case.T), 3), "status": r["info"]["status"],
            "max_sweeps": r["info"]["max_sweeps"], "jacobi_tile": r["tile"], "X": X}
        if ph is not None:
            out[name]["phase_ms_per_iteration"] = {k: round(v / L_FULL, 4) for k, v in ph["stats"]["ms"].items()}
            out[name]["dct_roofline"] = dct_roofline(ph["stats"], name)
        log("completion %s: %.3f ms/iteration" % (name, 1e3 * r["seconds"] / L_FULL))
    out["mixed"]["rel_err_vs_fp64_gpu"] = float(np.linalg.norm(out["mixed"]["X"] - out["fp64"]["X"]) /
                                                 np.linalg.norm(out["fp64"]["X"]))
    for v in out.values():
        v.pop("X")
    out["iterations"] = L_FULL
    out["warm_start"] = "V of the previous iteration, reset every 64 iterations"
    return out


def beta_sweep(tm, torch, case):
    """Parameter study of Algorithm 1's fixed penalty beta (tau = 1/beta), at
    the paper's experimental settings otherwise (at most 500 iterations,
    tolerance 1e-8): recovery error and PSNR against beta, MIXED path."""
    rows = []
    B = torch.from_numpy(case.B).float().to("cuda:0")
    mask = torch.from_numpy(case.mask).to("cuda:0")
    ctx = tm.Context(0)
    for beta in (1e-3, 3e-3, 1e-2, 3e-2, 1e-1, 3e-1):
        t0 = time.perf_counter()
        X, info = tm.complete_tensor(B, mask, max_iter=500, tol=1e-8, beta=beta, check_every=10, prec=tm.MIXED,
                                     ctx=ctx)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        Xh = X.detach().cpu().double().numpy()
        rows.append({"beta": beta, "iters": info["iters"], "seconds": round(sec, 3),
                     "recovery_rel_err": float(np.linalg.norm(Xh - case.T) / np.linalg.norm(case.T)),
                     "psnr_db": round(psnr(Xh, case.T), 3)})
        log("beta sweep:", rows[-1])
    ctx.close()
    return rows


def batched(tm, torch, tprod):
    import synth

    shapes = synth.batch_shapes(64, synth.SEED_BASE + 4)
    Zs, taus = [], []
    for s in shapes:
        Zs.append(torch.from_numpy(synth.tsvt_case(tprod, s.n1, s.n2, s.n3, s.r, 0.01, s.tau, s.seed).Z)
                  .float().to("cuda:0"))
        taus.append(s.tau)
    ctx = tm.Context(0)
    tm.tsvt_dct_batched(Zs, taus, prec=tm.FP32, ctx=ctx)  # warm (tunes the batched tiles)
    torch.cuda.synchronize()
    ctx.set_option(tm.OPT_PROFILE, 1)
    ctx.stats(reset=True)
    t0 = time.perf_counter()
    _, status = tm.tsvt_dct_batched(Zs, taus, prec=tm.FP32, ctx=ctx, return_status=True)
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    st = ctx.stats(reset=True)
    ctx.close()
    # algorithmic Jacobi flops of the batch: per slice-sweep 8 m p(p-1)/2, summed
    # over the batch with each tensor's executed sweeps unknown individually;
    # the device counts slice-sweeps in total, so use the mean per slice-sweep
    slices = sum(s.n3 for s in shapes)
    f_mean = sum(8.0 * max(s.n1, s.n2) * min(s.n1, s.n2) * (min(s.n1, s.n2) - 1) / 2.0 * s.n3
                 for s in shapes) / slices
    jac_ms = st["ms"]["jacobi"]
    flops = f_mean * st["slice_sweeps"]
    return {"tensors": len(shapes), "slices": slices, "makespan_ms": round(1e3 * dt_s, 2),
            "t_svt_per_s": round(len(shapes) / dt_s, 2), "dtype": "f32", "statuses_ok": all(v == 0 for v in status),
            "phase_ms": {k: round(v, 3) for k, v in st["ms"].items()},
            "jacobi_roofline": {"bound": "alu", "slice_sweeps": st["slice_sweeps"],
                                "sweeps_per_slice": round(st["slice_sweeps"] / slices, 3),
                                "achieved": round(flops / (jac_ms * 1e-3) / 1e12, 3) if jac_ms > 0 else None,
                                "peak": PEAK["fp32_alu"], "unit": "TFLOP/s",
                                "frac": round(flops / (jac_ms * 1e-3) / 1e12 / PEAK["fp32_alu"], 4) if jac_ms > 0
                                else None,
                                "note": "flops from the slice-weighted mean per slice-sweep"},
            "recipe": "n1,n2 ~ U{32..512}, n3 ~ U{8..128}, rank min(n1,n2)/10, t-product + N(0,0.01)"}


def serving_requests(tprod, n, seed_offset=5):
    """n requests of the serving mix: shapes as the batch configuration,
    alternately a t-SVT and a 50-iteration completion (30% observed)."""
    import synth

    shapes = synth.batch_shapes(n, synth.SEED_BASE + seed_offset, cfg_index=5)
    reqs = []
    for j, s in enumerate(shapes):
        if j % 2 == 0:
            Z = synth.tsvt_case(tprod, s.n1, s.n2, s.n3, s.r, 0.01, s.tau, s.seed).Z.astype(np.float32)
            reqs.append(("tsvt", Z, s.tau))
        else:
            cc = synth.completion_case(tprod, s.n1, s.n2, s.n3, s.r, 0.3, 50, s.seed)
            reqs.append(("complete", cc.B.astype(np.float32), cc.mask))
    return reqs


def _submit(srv, r):
    if r[0] == "tsvt":
        return srv.submit_tsvt(r[1], r[2])
    return srv.submit_complete(r[1], r[2], 50, 10.0, 0.1)


def _drain(srv, ids):
    got = {}
    while len(got) < len(ids):
        for i in ids:
            if i not in got:
                r = srv.poll(i)
                if r is not None:
                    got[i] = r[1]
        time.sleep(0.0005)
    return got


def serving_saturation(tm, reqs, budget, max_active=16):
    """Requests per second with every request submitted at once."""
    srv = tm.Server(budget_bytes=budget, max_active=max_active)
    t0 = time.perf_counter()
    _drain(srv, [_submit(srv, r) for r in reqs])
    sat = len(reqs) / (time.perf_counter() - t0)
    srv.close()
    return sat


def serving_load(tm, reqs, kinds, qps, g, budget, skip=0, max_active=16):
    """Poisson arrivals at qps; latency percentiles over the requests after the
    first `skip` (warm-up).  reqs[k] is submitted as request k."""
    import synth

    arrivals = synth.poisson_arrivals(g, qps, len(reqs))
    srv = tm.Server(budget_bytes=budget, max_active=max_active)
    t0 = time.perf_counter()
    ids = []
    for a, r in zip(arrivals, reqs):
        while time.perf_counter() - t0 < a:
            time.sleep(0.0002)
        ids.append(_submit(srv, r))
        if len(ids) % 200 == 0:
            log("serving: %d of %d requests submitted, %.0f s" % (len(ids), len(reqs), time.perf_counter() - t0))
    got = _drain(srv, ids)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = np.array([got[i][2] - got[i][0] for i in ids]) * 1e3
    keep = range(skip, len(ids))
    la = np.array([lat[k] for k in keep])
    lt = np.array([lat[k] for k in keep if kinds[k] == "tsvt"])
    lc = np.array([lat[k] for k in keep if kinds[k] == "complete"])
    pc = lambda a, q: round(float(np.percentile(a, q)), 2)  # noqa: E731
    return {"qps": round(qps, 3), "p50_ms": pc(la, 50), "p99_ms": pc(la, 99),
            "p50_ms_tsvt": pc(lt, 50), "p99_ms_tsvt": pc(lt, 99),
            "p50_ms_complete": pc(lc, 50), "p99_ms_complete": pc(lc, 99),
            "throughput_req_per_s": round(len(ids) / wall, 3), "ticks": st["ticks"], "peak_bytes": st["peak_bytes"]}


SERVING_MIX = "50% t-SVT / 50% completion (50 iterations, tau 10->0.1), 30% observed"
SERVING_SHAPES = "n1,n2 ~ U{32..512}, n3 ~ U{8..128}"


def serving(tm, torch, tprod, nreq, loads):
    import synth

    g = np.random.default_rng(synth.SEED_BASE + 5)
    reqs = serving_requests(tprod, nreq)
    kinds = [r[0] for r in reqs]
    budget = 64 << 30
    sat = serving_saturation(tm, reqs, budget)
    log("serving saturation %.2f req/s" % sat)
    out = {"requests": len(reqs), "mix": SERVING_MIX, "shapes": SERVING_SHAPES, "saturation_req_per_s": round(sat, 3),
           "budget_bytes": budget, "max_active": 16, "loads": {}}
    # fixed request rates: Poisson arrivals at a fraction of saturation
    for load in loads:
        out["loads"][str(load)] = serving_load(tm, reqs, kinds, load * sat, g, budget)
        log("serving load %.2f: %s" % (load, out["loads"][str(load)]))
    return out


def serving_stream(tm, torch, tprod, nreq, warmup, loads, pool, saturation):
    """The long serving stream: warmup + nreq requests per load, drawn in turn
    from a pool of `pool` generated requests (request k is pool[k mod pool]);
    percentiles over the nreq requests after the warm-up.  Saturation is
    given, or measured on the pool."""
    import synth

    g = np.random.default_rng(synth.SEED_BASE + 8)
    base = serving_requests(tprod, pool)
    budget = 64 << 30
    sat = saturation if saturation > 0 else serving_saturation(tm, base, budget)
    total = warmup + nreq
    reqs = [base[k % pool] for k in range(total)]
    kinds = [r[0] for r in reqs]
    out = {"requests": nreq, "warmup_requests": warmup, "pool": pool, "mix": SERVING_MIX, "shapes": SERVING_SHAPES,
           "saturation_req_per_s": round(sat, 3), "saturation_given": saturation > 0, "budget_bytes": budget,
           "max_active": 16, "loads": {}}
    for load in loads:
        out["loads"][str(load)] = serving_load(tm, reqs, kinds, load * sat, g, budget, skip=warmup)
        log("serving stream load %.2f: %s" % (load, out["loads"][str(load)]))
    return out


def video_shaped(tm, torch, tprod, steps):
    """Mixed-precision completion at 144x176x100 (rank 15, 20% observed), with
    its relative difference from the FP64 GPU path on the same input."""
    import synth

    cc = synth.completion_case(tprod, 144, 176, 100, 15, 0.2, 100, synth.SEED_BASE + 3)
    out = {}
    for name, prec in (("mixed", tm.MIXED), ("fp64", tm.FP64)):
        r = run_completion(tm, torch, cc, prec, steps, 2, profile=0)
        out[name] = r
    X64, Xm = out["fp64"]["X"], out["mixed"]["X"]
    return {"shape": [144, 176, 100], "rank": 15, "observed": 0.2, "iterations": steps,
            "t_svt_per_s_mixed": round(steps / out["mixed"]["seconds"], 2),
            "t_svt_per_s_fp64": round(steps / out["fp64"]["seconds"], 2),
            "mixed_rel_err_vs_fp64_gpu": float(np.linalg.norm(Xm - X64) / np.linalg.norm(X64)),
            "recovery_rel_err_mixed": float(np.linalg.norm(Xm - cc.T) / np.linalg.norm(cc.T))}


def dct_vs_dft(tm, torch, reps=3):
    """Table 2's comparison on MI355X: the DCT and DFT paths on random N(0,1)
    tensors of the table's four shapes, FP64.  tnn_* is the t-SVD work (tube
    transform and slice SVDs, then the singular-value sum), tsvt_* the whole
    t-SVT (also the threshold, rebuild and inverse transform).  The DFT path
    thresholds complex slices through their 2 n1 x 2 n2 real forms, so shapes
    with more than 256 rows or columns are beyond it."""
    rows = []
    g = np.random.default_rng(synth_seed(6))
    for n1, n2, n3 in ((100, 100, 100), (100, 100, 400), (200, 200, 100), (400, 400, 100)):
        X = torch.from_numpy(np.asfortranarray(g.standard_normal((n1, n2, n3)))).to("cuda:0")
        X = tm.fortran(X.permute(2, 1, 0).contiguous().permute(2, 1, 0))
        ctx = tm.Context(0)
        row = {"shape": [n1, n2, n3]}
        tau = 0.5 * (np.sqrt(n1) + np.sqrt(n2))
        calls = {"tnn_c": lambda: tm.tnn_c(X, ctx=ctx), "tsvt_dct": lambda: tm.tsvt_dct(X, tau, ctx=ctx)}
        if max(n1, n2) <= 256:
            calls["tnn_f"] = lambda: tm.tnn_f(X, ctx=ctx)
            calls["tsvt_dft"] = lambda: tm.tsvt_dft(X, tau * np.sqrt(n3), ctx=ctx)
        for name, fn in calls.items():
            fn()  # tunes the tiles of the shape
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            row[name + "_ms"] = round(1e3 * (time.perf_counter() - t0) / reps, 3)
        if "tnn_f_ms" in row:
            row["dft_over_dct_tnn"] = round(row["tnn_f_ms"] / row["tnn_c_ms"], 3)
            row["dft_over_dct_tsvt"] = round(row["tsvt_dft_ms"] / row["tsvt_dct_ms"], 3)
        else:
            row["dft"] = "beyond the DFT path (real forms of 800 rows)"
        ctx.close()
        rows.append(row)
        log("dct vs dft:", row)
    return {"rows": rows, "dtype": "f64", "data": "random N(0,1) tensors (Table 2's shapes)",
            "paper_table2_s": {"100x100x100": [0.0859, 0.0481], "100x100x400": [0.3425, 0.1799],
                               "200x200x100": [0.3817, 0.2140], "400x400x100": [1.9668, 0.9523],
                               "note": "original (DFT) and DCT t-SVD in seconds, MATLAB on the paper's CPU"}}


def other_transforms(tm, torch, Z0, tau, reps=10):
    """The t-SVT under caller-given transforms (the concluding remarks' other
    transforms) against the DCT one on the same input (Z_0 at 256x256x31):
    a random orthogonal L and a random well-conditioned non-orthogonal L
    (I + 0.2 N(0,1)/sqrt(n3)), same kernels, host-given matrices."""
    g = np.random.default_rng(synth_seed(9))
    n3 = Z0.shape[2]
    Lo, _ = np.linalg.qr(g.standard_normal((n3, n3)))
    Lg = np.eye(n3) + 0.2 * g.standard_normal((n3, n3)) / np.sqrt(n3)
    rows = []
    for name, prec in (("mixed", tm.MIXED), ("fp64", tm.FP64)):
        dt = torch.float64 if prec == tm.FP64 else torch.float32
        Z = tm.fortran(Z0.to(dt).permute(2, 1, 0).contiguous().permute(2, 1, 0))
        ctx = tm.Context(0)
        calls = {"dct": lambda: tm.tsvt_dct(Z, tau, prec=prec, ctx=ctx),
                 "orthogonal_L": lambda: tm.tsvt_transform(Z, tau, Lo, prec=prec, ctx=ctx),
                 "general_L": lambda: tm.tsvt_transform(Z, tau, Lg, prec=prec, ctx=ctx)}
        row = {"path": name}
        for k, fn in calls.items():
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            row[k + "_ms"] = round(1e3 * (time.perf_counter() - t0) / reps, 4)
        ctx.close()
        rows.append(row)
        log("other transforms:", row)
    return {"shape": list(Z0.shape), "tau": float(tau), "rows": rows,
            "note": "cold t-SVTs of Z_0; the transform matrix changes the slices, so sweeps differ"}


def long_tubes(tm, torch, reps=5):
    """Tubes longer than 128: the fast O(n3 log n3) transform (Bluestein's chirp
    with register FFTs) against the dense vector-ALU product, forward-transform
    launch time from the HIP events of a profiled t-SVT on N(0,1) tensors.
    Roofline of the fast kernel: algorithmic bytes = read and write every
    element once (2 N n3 es)."""
    rows = []
    g = np.random.default_rng(synth_seed(7))
    for n1, n2, n3 in ((256, 256, 200), (256, 256, 400)):
        for name, prec in (("mixed", tm.MIXED), ("fp64", tm.FP64)):
            dt = torch.float64 if prec == tm.FP64 else torch.float32
            X = torch.from_numpy(np.asfortranarray(g.standard_normal((n1, n2, n3)))).to(dt).to("cuda:0")
            X = tm.fortran(X.permute(2, 1, 0).contiguous().permute(2, 1, 0))
            row = {"shape": [n1, n2, n3], "path": name}
            for kind, dense in (("fast", 0), ("dense", 1)):
                if dense and n3 * 64 * (8 if prec == tm.FP64 else 4) > (160 - 8) * 1024:
                    row[kind] = "not run: a 64-tube tile of this length exceeds the LDS"
                    continue
                ctx = tm.Context(0)
                try:
                    ctx.set_option(tm.OPT_LONG_TUBES, dense)
                    ctx.set_option(tm.OPT_PROFILE, 1)
                    tm.tsvt_dct(X, 1.0, prec=prec, ctx=ctx)
                    torch.cuda.synchronize()
                    ctx.stats(reset=True)
                    for _ in range(reps):
                        tm.tsvt_dct(X, 1.0, prec=prec, ctx=ctx)
                    torch.cuda.synchronize()
                    st = ctx.stats(reset=True)
                    row[kind + "_forward_us"] = round(1e3 * st["ms"]["forward_transform"] / reps, 1)
                    row[kind + "_inverse_us"] = round(1e3 * st["ms"]["inverse_transform"] / reps, 1)
                except tm.TsvdError as e:
                    row[kind] = "not run: %s" % e
                finally:
                    ctx.close()
            if "fast_forward_us" in row:
                nbytes = 2.0 * n1 * n2 * n3 * (8 if prec == tm.FP64 else 4)
                gbs = nbytes / (row["fast_forward_us"] * 1e-6) / 1e9
                row["fast_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"],
                                        "unit": "GB/s", "frac": round(gbs / PEAK["hbm_GBs"], 4)}
            rows.append(row)
            log("long tubes:", row)
    return {"rows": rows, "data": "random N(0,1) tensors",
            "note": "dense = the vector-ALU product; FP64 tubes beyond 304 have only the fast kernel"}


def synth_seed(i):
    import synth

    return synth.SEED_BASE + i


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inputs, budget_s=10.0, max_rounds=40):
    """The FP64 oracle, as it stands, on the host's threads (frontal slices split
    over threads; per-slice arithmetic unchanged): rounds of one t-SVT of each
    input, repeated until about budget_s seconds of host work."""
    import oracle

    oracle.build(force=False)
    T = min(16, oracle.host_threads())
    oracle.set_threads(T)
    rounds = 0
    t0 = time.perf_counter()
    while True:
        for Zh, tau in inputs:
            oracle.tsvt_dct(Zh, float(tau))
        rounds += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or rounds >= max_rounds:
            break
    n = rounds * len(inputs)
    return {"value": round(n / dt, 5), "unit": "t-SVT/s", "cores": T, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": "%d FP64 oracle t-SVTs (%d rounds of Z_0 at tau 10 and Z_99 at tau 0.1) at 256x256x31 on %d "
                      "host threads, %.1f s" % (n, rounds, T, dt)}


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
    if args.serving_stream > 0:
        out = {"serving_stream": serving_stream(tm, torch, tprod, args.serving_stream, args.serving_warmup,
                                                [float(x) for x in args.serving_loads.split(",")],
                                                args.serving_pool, args.serving_saturation)}
        tm.close_all()
        print(json.dumps(out), flush=True)
        return
    case = synth.completion_case(tprod, N1, N2, N3, RANK, SR, L_FULL, synth.SEED_BASE + 2)
    Z0 = tm.fortran(torch.from_numpy(case.B).to("cuda:0"))
    Z99, cap = capture_last_iterate(tm, torch, case)
    inputs = [(Z0, case.taus[0]), (Z99, case.taus[L_FULL - 1])]
    log("captured Z_99 (FP64, %d iterations, status %d)" % (cap["iters"], cap["status"]))
    paths = args.paths.split(",")
    precs = {"fp64": tm.FP64, "fp32": tm.FP32, "mixed": tm.MIXED}
    results = {}
    for name in paths:
        r = timed_tsvt(tm, torch, inputs, precs[name], args.steps, args.warmup)
        results[name] = r
        log("%s: %.4f s for %d steps (%.4f ms/step), jacobi %.4f ms/launch, slice-sweeps %d, status %d" % (
            name, r["seconds"], args.steps, 1e3 * r["seconds"] / args.steps,
            r["stats"]["ms"]["jacobi"] / max(1, r["stats"]["launches"]["jacobi"]), r["stats"]["slice_sweeps"],
            r["status"]))
    head = paths[0]
    r = results[head]
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
        "config": {"workload": WORKLOAD + ", path=%s" % head, "n1": N1, "n2": N2, "n3": N3, "rank": RANK,
                   "observed": SR, "taus": [float(case.taus[0]), float(case.taus[L_FULL - 1])]},
        "roofline": jacobi_roofline(r["stats"], head, False, N3),
    }
    for name, rr in results.items():
        out.setdefault("paths", {})[name] = {
            "t_svt_per_s": round(args.steps / rr["seconds"], 3),
            "ms_per_step": round(1e3 * rr["seconds"] / args.steps, 4),
            "per_input_ms": {"Z_0": rr["per_input_ms"][0], "Z_99": rr["per_input_ms"][1]},
            "jacobi_roofline": jacobi_roofline(rr["stats"], name, False, N3),
            "status": rr["status"], "max_sweeps": rr["max_sweeps"], "jacobi_tile": rr["tile"],
            "phase_ms_per_step": rr["phase_ms_per_step"]}
    if "fp64" in results and head != "fp64":
        out["speedup_vs_fp64"] = round(results["fp64"]["seconds"] / r["seconds"], 3)
    # the same loop with the full Jacobi iteration on every slice (the kept-column
    # mode and its threshold certificate switched off)
    fr = timed_tsvt(tm, torch, inputs, precs[head], args.steps, args.warmup, kept=0, phases=False)
    out["full_iteration"] = {"t_svt_per_s": round(args.steps / fr["seconds"], 3),
                             "ms_per_step": round(1e3 * fr["seconds"] / args.steps, 4),
                             "per_input_ms": {"Z_0": fr["per_input_ms"][0], "Z_99": fr["per_input_ms"][1]},
                             "jacobi_roofline": jacobi_roofline(fr["stats"], head, False, N3), "status": fr["status"]}
    log("%s, full iteration: %.4f ms/step" % (head, out["full_iteration"]["ms_per_step"]))
    if not args.no_extras:
        out["completion_in_situ"] = completion_in_situ(tm, torch, case)
        out["video_shaped"] = video_shaped(tm, torch, tprod, 100)
        log("video-shaped:", out["video_shaped"])
        out["batched"] = batched(tm, torch, tprod)
        log("batched:", out["batched"])
        out["beta_sweep"] = beta_sweep(tm, torch, case)
        out["dct_vs_dft"] = dct_vs_dft(tm, torch)
        out["long_tubes"] = long_tubes(tm, torch)
        out["other_transforms"] = other_transforms(tm, torch, inputs[0][0], inputs[0][1])
        out["serving"] = serving(tm, torch, tprod, args.serving_requests,
                                 [float(x) for x in args.serving_loads.split(",")])
        log("serving:", out["serving"])
    if args.copy_calibration:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = a.clone()
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        host = [(np.asfortranarray(Z.detach().cpu().numpy()), tau) for Z, tau in inputs]
        out["cpu_baseline"] = cpu_baseline(host)
    tm.close_all()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
