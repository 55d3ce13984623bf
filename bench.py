"""Benchmark: Vecchia conditionals per second, FP64 log-likelihood + gradient.

Default workload: n = 1,000,000 uniform points in the unit square, random
order, m = 120 nearest previous neighbours, Matern nu = 0.5,
theta = (sigma2, beta, tau2) = (1.5, 0.03, 1e-4), z ~ N(0, 1) i.i.d.
One step = one full evaluation of the log-likelihood and its gradient
(every conditional: gather, covariance, Cholesky, solves, adjoint, sums).
Inputs are resident in HBM before timing starts.

Two forms are timed on the same inputs:
  plain    one vecchia_loglik_grad call per step with the built-in default
           kernel variant;
  batched  the variant chosen by the autotuner for (m, gradient), a batched
           plan over the field, captured once into a HIP graph; one graph
           launch per step.
`value` is the batched form; the plain figures are reported beside it.

Prints one JSON line.  Extra objects:
  roofline      algorithmic FP64 flops of the conditional kernel per launch
                divided by its measured launch duration, against the FP64 peak;
  cpu_baseline  the oracle timed on a bounded sample of the same workload on
                the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Vecchia conditionals/sec (logL+grad, FP64) n=1M m=120; batched vs plain"
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (and matrix) peak: 256 CU x 2.4 GHz x 128 flop/clk


# HBM traffic of the conditional kernel per launch on the default workload,
# from two rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE,
# KiB per dispatch) with --copy-probe: the probe's 512 MiB device copy reads
# 262161.9 KiB of FETCH_SIZE and 524288 KiB of WRITE_SIZE, which fixes the
# scale factors.  It describes the kernel sources it was measured on only, so
# it is reported when their digest still matches (kernel_sources_digest).
MEASURED_TRAFFIC = {
    "sources_sha256": "49ecc728110aa664f6ba8b9b093e12cf94c4b84d52df36ab14f0af3118f30a59",
    "workload": "n1M_m120_nu0.5", "variant": "tile_w4",
    "fetch_kib_raw": 16933536.75, "fetch_factor": 524288.0 / 262161.6875,
    "write_kib_raw": 27507389.3125, "write_factor": 524288.0 / 524288.0,
}


KERNEL_SOURCES = ("device_common.h", "exp_table.h", "kernel_lds.h", "kernel_tile.h", "launch.h",
                  "kernels_nu05.hip", "kernels_nu15.hip", "kernels_nu25.hip")


def kernel_sources_digest() -> str:
    """sha256 over the sources that make up the conditional kernel and its compile flags, in path order."""
    import hashlib

    h = hashlib.sha256()
    files = [os.path.join(ROOT, "paper_2403_07412_amd", "csrc", f) for f in KERNEL_SOURCES]
    files.append(os.path.join(ROOT, "paper_2403_07412_amd", "build.py"))
    for path in files:
        h.update(os.path.relpath(path, ROOT).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic_bytes(workload: str, variant: str):
    t = MEASURED_TRAFFIC
    if t["workload"] != workload or t["variant"] != variant or t["sources_sha256"] != kernel_sources_digest():
        return None
    return (t["fetch_kib_raw"] * t["fetch_factor"] + t["write_kib_raw"] * t["write_factor"]) * 1024.0


def la_flops_per_conditional(k: np.ndarray, with_grad: bool) -> np.ndarray:
    """Algorithmic dense-LA flops of one conditional with k neighbours (the paper's flop model, Sec. IV-C):
    POTRF k^3/3 + k^2/2 + k/6, two TRSVs 2k^2, the two dot products 4k; the gradient adds two
    back substitutions, 2k^2.  Covariance generation (k(k+1)/2 kernel evaluations) is counted apart."""
    k = k.astype(np.float64)
    f = k ** 3 / 3 + k ** 2 / 2 + k / 6 + 2 * k ** 2 + 4 * k
    if with_grad:
        f = f + 2 * k ** 2
    return f


def workload_counts(n: int, m: int, with_grad: bool):
    k = np.minimum(np.arange(n), m)
    flops = float(la_flops_per_conditional(k, with_grad).sum())
    evals = float((k * (k + 1) / 2 + k).sum()) * (2 if with_grad else 1)
    gather_bytes = float((28 * k + 24).sum())
    return flops, evals, gather_bytes


def cpu_baseline(field, with_grad: bool, target_s: float = 15.0):
    """The oracle on a bounded random sample of the workload's conditionals (same inputs)."""
    import oracle

    threads = max(1, min(os.cpu_count() or 1, 16))
    rng = np.random.default_rng(12345)
    th = field.thetas[0]
    size = 64
    elapsed = 0.0
    while True:
        idx = np.sort(rng.choice(field.n, size, replace=False)).astype(np.int64)
        t0 = time.perf_counter()
        oracle.terms(field.locs, field.z, field.nbr, field.m, field.nu, th, idx=idx, with_grad=with_grad,
                     threads=threads)
        elapsed = time.perf_counter() - t0
        if elapsed >= target_s * 0.5 or size >= field.n:
            break
        size = int(min(field.n, max(size * 2, size * target_s / max(elapsed, 1e-3) * 0.7)))
    return {"value": size / elapsed, "unit": "conditionals/s", "cores": threads, "kind": "oracle",
            "sample": f"{size} conditionals drawn uniformly from the {field.n}-point workload "
                      f"({'value+gradient' if with_grad else 'value'}), {elapsed:.1f} s"}


def preprocess_times(v, f, locs, stream, reps: int = 3):
    """The workload's preprocessing on the GPU (conditioning sets, Morton ordering), best of `reps`
    HIP-event timings, beside the CPU grid search that generated the benchmark's sets (16 threads)."""
    import torch

    import workloads as wl

    def best_ms(fn):
        ts = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return min(ts[1:])

    nbr_out = torch.empty((f.n, f.m), dtype=torch.int32, device=locs.device)
    kws = torch.empty(v.vecchia_knn_workspace_size(f.n), dtype=torch.uint8, device=locs.device)
    knn_ms = best_ms(lambda: v.vecchia_knn(locs, f.m, out=nbr_out, ws=kws, stream=stream))
    perm = torch.empty(f.n, dtype=torch.int64, device=locs.device)
    morton_ms = best_ms(lambda: v.vecchia_morton_order(locs, out=perm, stream=stream))
    same = bool(torch.equal(nbr_out.cpu(), torch.from_numpy(f.nbr)))
    t0 = time.perf_counter()
    wl.nearest_previous_neighbours(f.locs, f.m, min(os.cpu_count() or 1, 16))
    cpu_ms = (time.perf_counter() - t0) * 1e3
    return {"knn_ms": knn_ms, "morton_ms": morton_ms, "knn_cpu_grid_ms": cpu_ms,
            "knn_cpu_threads": min(os.cpu_count() or 1, 16), "knn_equals_cpu_sets": same}


def realdata_times(v, stream, reps: int = 2):
    """The real-data configuration of Sec. V-C on synthetic points: 250,000 observed and 25,000
    prediction points as (longitude, latitude) over a 10 x 10 degree box, power-exponential covariance on
    great-circle distances, m = 60.  Best-of-`reps` HIP-event timings of each step: great-circle
    conditioning sets, log-likelihood + gradient, prediction-point neighbour sets, kriging."""
    import torch

    import workloads as wl

    rng = np.random.default_rng(2403)
    n, nq, m = 250_000, 25_000, 60
    dev = torch.device("cuda:0")
    L = torch.from_numpy(wl.lonlat_locations(rng, n)).to(dev)
    Z = torch.from_numpy(rng.standard_normal(n)).to(dev)
    Q = torch.from_numpy(wl.lonlat_locations(rng, nq)).to(dev)
    cov = (v.POWEXP, v.GREAT_CIRCLE, 0.9)
    th = torch.tensor([1.0, 80.0, 0.05], dtype=torch.float64, device=dev)

    def best_ms(fn):
        ts = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return min(ts[1:])

    nbr = torch.empty((n, m), dtype=torch.int32, device=dev)
    kws = torch.empty(v.vecchia_knn_workspace_size(n), dtype=torch.uint8, device=dev)
    knn_ms = best_ms(lambda: v.vecchia_knn(L, m, out=nbr, ws=kws, stream=stream, metric=v.GREAT_CIRCLE))
    ws = torch.empty(v.vecchia_workspace_size(n, m), dtype=torch.uint8, device=dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(3, dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int64, device=dev)
    ll_ms = best_ms(lambda: v.vecchia_loglik_cov(L, Z, nbr, m, cov, th, with_grad=True, out=out, grad=grad,
                                                 status=st, ws=ws, stream=stream))
    qnbr = torch.empty((nq, m), dtype=torch.int32, device=dev)
    q_ms = best_ms(lambda: v.vecchia_knn_query(L, Q, m, metric=v.GREAT_CIRCLE, out=qnbr, ws=kws, stream=stream))
    mean = torch.empty(nq, dtype=torch.float64, device=dev)
    var = torch.empty(nq, dtype=torch.float64, device=dev)
    pst = torch.empty(1, dtype=torch.int64, device=dev)
    p_ms = best_ms(lambda: v.vecchia_predict(L, Z, Q, qnbr, m, cov, th, mean=mean, var=var, status=pst,
                                             stream=stream))
    ok = int(st.item()) == 0 and int(pst.item()) == 0 and bool(torch.isfinite(mean).all())
    # algorithmic dense-LA flops (the same model as the headline roofline) and haversine keys
    ll_flops, _, _ = workload_counts(n, m, True)
    p_flops = float(la_flops_per_conditional(np.full(nq, min(n, m)), False).sum())
    knn_keys = n * (n - 1) / 2.0
    return {"workload": "n250K_q25K_m60 power-exponential alpha=0.9, great-circle", "knn_ms": knn_ms,
            "knn_keys_per_s": knn_keys / (knn_ms * 1e-3),
            "loglik_grad_ms": ll_ms, "loglik_grad_cond_per_s": n / (ll_ms * 1e-3),
            "loglik_grad_tflops": ll_flops / (ll_ms * 1e-3) / 1e12,
            "loglik_grad_frac": ll_flops / (ll_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "knn_query_ms": q_ms, "predict_ms": p_ms, "predict_per_s": nq / (p_ms * 1e-3),
            "predict_tflops": p_flops / (p_ms * 1e-3) / 1e12,
            "predict_frac": p_flops / (p_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, "status_ok": ok}


def multifield_times(v, stream, reps: int = 3):
    """The 32-field workload (n log-uniform in [1e4, 5e5], m uniform in 10..150, Matern nu = 3/2, one
    theta per field, value + gradient): 32 per-field calls with the built-in default variants against
    one batched plan, with variants autotuned per m, replayed from a captured graph; then 1024 small
    fields the same two ways, where per-call launch costs dominate.  Best of `reps` HIP-event timings."""
    import torch

    import workloads as wl

    w = wl.config_multifield(knn_threads=min(os.cpu_count() or 1, 16))
    dev = torch.device("cuda:0")
    fields = [tuple(torch.from_numpy(a).to(dev) for a in (f.locs, f.z, f.nbr)) + (f.m,) for f in w.fields]
    thetas = torch.from_numpy(np.stack([f.thetas[0] for f in w.fields])).to(dev).reshape(-1, 1, 3).contiguous()
    nsum = sum(f.n for f in w.fields)
    wss = [torch.empty(v.vecchia_workspace_size(f.n, f.m), dtype=torch.uint8, device=dev) for f in w.fields]
    outs = [(torch.empty(1, dtype=torch.float64, device=dev), torch.empty(3, dtype=torch.float64, device=dev),
             torch.empty(1, dtype=torch.int64, device=dev)) for _ in w.fields]

    def plain():
        for q, (L, Z, N, m) in enumerate(fields):
            o, g, st = outs[q]
            v.vecchia_loglik_grad(L, Z, N, m, 1.5, thetas[q, 0], out=o, grad=g, status=st, ws=wss[q], stream=stream)

    def best_ms(fn):
        ts = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return min(ts[1:])

    # plain: the built-in default variant of every m
    saved = {f.m: v.vecchia_get_variant(f.m, True) for f in w.fields}
    for mm in saved:
        v.vecchia_set_variant(mm, True, "auto")
    p_ms = best_ms(plain)
    # batched: variants autotuned per m on each field's own points, then one plan and one graph
    tuned = {}
    for q, (L, Z, N, m) in enumerate(fields):
        if m not in tuned:
            tuned[m], _ = v.vecchia_autotune(L, Z, N, m, 1.5, thetas[q, 0].contiguous(), True,
                                             sample=min(w.fields[q].n, 50000), reps=2)
    plan = v.BatchedPlan(fields, 1, 1.5, True)
    b_out, b_grad, b_st = plan.outputs()
    graph = plan.capture(thetas, b_out, b_grad, b_st)
    b_ms = best_ms(lambda: graph.launch(stream))
    graph.close()
    plan.close()
    for mm, var in saved.items():
        v.vecchia_set_variant(mm, True, var if mm == 120 else "auto")
    changed = sum(1 for q, f in enumerate(w.fields) if tuned[f.m] != v.vecchia_get_variant(f.m, True))
    # many small fields (1024 fields of 2,000 points, m = 30): per-call launch costs against one graph
    rng = np.random.default_rng(2404)
    small = []
    for _ in range(1024):
        locs = wl.uniform_locations(rng, 2000)
        small.append(wl.Field(locs, rng.standard_normal(2000), wl.nearest_previous_neighbours(locs, 30), 30, 1.5,
                              np.array([[1.0, 0.1, 1e-3]])))
    sf = [tuple(torch.from_numpy(a).to(dev) for a in (f.locs, f.z, f.nbr)) + (f.m,) for f in small]
    sth = torch.tensor([1.0, 0.1, 1e-3], dtype=torch.float64, device=dev)
    sws = torch.empty(v.vecchia_workspace_size(2000, 30), dtype=torch.uint8, device=dev)
    so, sg, sst = outs[0]

    def plain_small():
        for (L, Z, N, m) in sf:
            v.vecchia_loglik_grad(L, Z, N, m, 1.5, sth, out=so, grad=sg, status=sst, ws=sws, stream=stream)

    sp_ms = best_ms(plain_small)
    splan = v.BatchedPlan(sf, 1, 1.5, True)
    s_out, s_grad, s_st = splan.outputs()
    sthetas = sth.reshape(1, 1, 3).expand(len(sf), 1, 3).contiguous()
    sgraph = splan.capture(sthetas, s_out, s_grad, s_st)
    sb_ms = best_ms(lambda: sgraph.launch(stream))
    sgraph.close()
    splan.close()
    return {"workload": f"{len(fields)} fields, n log-uniform [1e4, 5e5] (sum {nsum}), m 10..150, nu=1.5, "
                        "value+gradient", "plain_ms": p_ms, "batched_ms": b_ms,
            "plain_cond_per_s": nsum / (p_ms * 1e-3), "batched_cond_per_s": nsum / (b_ms * 1e-3),
            "batched_speedup": p_ms / b_ms, "fields_with_tuned_variant_other_than_default": changed,
            "small_fields": {"workload": "1024 fields of 2,000 uniform points, m=30, nu=1.5, value+gradient",
                             "plain_ms": sp_ms, "batched_ms": sb_ms, "batched_speedup": sp_ms / sb_ms}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--m", type=int, default=120)
    ap.add_argument("--variant", default="auto", help="plain form: kernel variant (auto, unblocked, tile_w1/2/4/8)")
    ap.add_argument("--form", default="both", choices=["both", "plain", "batched"])
    ap.add_argument("--tune-sample", type=int, default=0,
                    help="conditionals the autotuner times per variant (0: the whole field, so that every launch "
                         "of the chosen kernel in a profile of this command has the full size)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-realdata", action="store_true",
                    help="skip the real-data configuration leg (power exponential, great-circle, kriging)")
    ap.add_argument("--no-multifield", action="store_true",
                    help="skip the 32-field leg (per-field calls against one batched launch)")
    ap.add_argument("--no-preprocess", action="store_true",
                    help="skip timing the GPU conditioning-set search and Morton ordering of the workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, copy a 512 MiB device buffer once (a kernel of known traffic that scales "
                         "the FETCH_SIZE / WRITE_SIZE counters of a profiled run)")
    ap.add_argument("--traffic-kib", type=float, nargs=2, default=None, metavar=("FETCH", "WRITE"),
                    help="HBM KiB per launch of the conditional kernel (FETCH_SIZE, WRITE_SIZE), already scaled "
                         "by the copy-probe factor, to report as roofline.traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the method's conditionals are independent and a multi-GPU run "
              "would shard them by cost and all-reduce four doubles; it measures one GPU's share.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2403_07412_amd as v
    import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    v.library()
    t0 = time.time()
    w = wl.config_large(n=args.n, m=args.m, knn_threads=min(os.cpu_count() or 1, 16))
    f = w.fields[0]
    print(f"# workload {w.name}: inputs ready in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    locs = torch.from_numpy(f.locs).to(dev)
    z = torch.from_numpy(f.z).to(dev)
    nbr = torch.from_numpy(f.nbr).to(dev)
    theta = torch.from_numpy(f.thetas[0].copy()).to(dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(3, dtype=torch.float64, device=dev)
    status = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(v.vecchia_workspace_size(f.n, f.m), dtype=torch.uint8, device=dev)

    stream = torch.cuda.current_stream()

    def timed(step, steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            step()
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return wall, [a.elapsed_time(b) for a, b in ev]

    results = {}
    if args.form in ("both", "plain"):
        def plain_step():
            v.vecchia_loglik_variant(locs, z, nbr, f.m, f.nu, theta, args.variant, with_grad=True, out=out,
                                     grad=grad, status=status, ws=ws)
        wall, launch_ms = timed(plain_step, args.steps, args.warmup)
        if int(status.item()) != 0:
            raise RuntimeError(f"plain: status {int(status.item())}")
        results["plain"] = (wall, launch_ms, out.item(), grad.cpu().numpy().copy(),
                            args.variant if args.variant != "auto" else v.vecchia_get_variant(f.m, True))
    if args.form in ("both", "batched"):
        best, us = v.vecchia_autotune(locs, z, nbr, f.m, f.nu, theta, True, sample=args.tune_sample or f.n, reps=2)
        print(f"# autotune m={f.m} grad: best variant {best}; us/point {us}", file=sys.stderr, flush=True)
        plan = v.BatchedPlan([(locs, z, nbr, f.m)], 1, f.nu, True)
        thetas = theta.reshape(1, 1, 3).contiguous()
        b_out, b_grad, b_status = plan.outputs()
        graph = plan.capture(thetas, b_out, b_grad, b_status)
        wall, launch_ms = timed(lambda: graph.launch(stream), args.steps, args.warmup)
        if int(b_status.reshape(-1)[0].item()) != 0:
            raise RuntimeError(f"batched: status {int(b_status.reshape(-1)[0].item())}")
        results["batched"] = (wall, launch_ms, b_out.reshape(-1)[0].item(), b_grad.reshape(3).cpu().numpy().copy(),
                              plan.classes()[0][1])
        graph.close()
        plan.close()
    for form, (wall, launch_ms, ell, g, var) in results.items():
        print(f"# {form}: variant {var}; {args.steps} steps: wall {wall * 1e3 / args.steps:.3f} ms/step, events mean "
              f"{np.mean(launch_ms):.3f} ms (min {min(launch_ms):.3f}); loglik {ell:.12e} grad {g}",
              file=sys.stderr, flush=True)
    main_form = "batched" if "batched" in results else "plain"
    wall, launch_ms, _, _, variant = results[main_form]
    ms = float(np.mean(launch_ms))

    flops, evals, gbytes = workload_counts(f.n, f.m, True)
    achieved = flops / (ms * 1e-3) / 1e12
    value = f.n * args.steps / wall
    names = {val: k for k, val in v.VARIANTS.items()}
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "conditionals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name} value+gradient", "n": f.n, "m": f.m, "nu": f.nu,
                   "theta": [float(x) for x in f.thetas[0]], "form": main_form,
                   "variant": names.get(variant, variant)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "algorithmic_flops_per_launch": flops, "kernel_evals_per_launch": evals,
                     "gather_bytes_per_launch": gbytes, "launch_ms": ms},
    }
    if "plain" in results and main_form != "plain":
        pw, pl, _, _, pv = results["plain"]
        rec["plain"] = {"value": f.n * args.steps / pw, "ms_per_step": pw * 1e3 / args.steps,
                        "launch_ms": float(np.mean(pl)), "variant": names.get(pv, pv)}
    if args.traffic_kib is not None:
        rec["roofline"]["traffic"] = (args.traffic_kib[0] + args.traffic_kib[1]) * 1024.0
    else:
        rec["roofline"]["traffic"] = measured_traffic_bytes(w.name, names.get(variant, variant))
    if args.copy_probe:
        src = torch.empty(512 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_preprocess:
        rec["preprocess"] = preprocess_times(v, f, locs, stream)
    if not args.no_realdata:
        rec["realdata"] = realdata_times(v, stream)
    if not args.no_multifield:
        rec["multifield"] = multifield_times(v, stream)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(f, True)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
