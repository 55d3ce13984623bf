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
           plan over the field (one persistent launch), captured once into a
           HIP graph; one graph launch per step.
`value` is the faster form; both are reported.  Further objects time the
other workloads: the 250K jittered grid (forward), 64 parameter vectors at
200K points (per-call against batched), the paper's m grid at 250K points,
32 uneven fields, the real-data configuration and the preprocessing.

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
# 262167.3 KiB of FETCH_SIZE and 524288 KiB of WRITE_SIZE, which fixes the
# scale factors (the kernel's counts are the mean of three dispatches).  The FP64
# instruction counters of the same kernel (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64,
# SQ_INSTS_VALU_MFMA_MOPS_F64, one run of their own) give the FP64 flops it
# executes per launch: 64 lanes x (ADD + MUL + TRANS + 2 FMA) + 512 x MOPS.
# The record describes the kernel sources it was measured on only, so it is
# reported when their digest still matches (kernel_sources_digest).
MEASURED_TRAFFIC = {
    "sources_sha256": "889c220c3831158fe298add76f30a8e6c52522e07d8e3b70db4fb2defa6e8b6d",
    "workload": "n1M_m120_nu0.5", "variant": "tile_w4",
    "fetch_kib_raw": 9754650.7083, "fetch_factor": 524288.0 / 262167.25,
    "write_kib_raw": 8415836.7500, "write_factor": 524288.0 / 524288.0,
    "f64_add": 1628957056.0, "f64_mul": 3441903358.0, "f64_fma": 8037825600.0, "f64_trans": 433989312.0,
    "f64_mfma_mops": 1792000000.0,
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


def measured_fp64_flops(workload: str, variant: str):
    """FP64 flops the kernel executes per launch, from its instruction counters (None if they are stale)."""
    t = MEASURED_TRAFFIC
    if t["workload"] != workload or t["variant"] != variant or t["sources_sha256"] != kernel_sources_digest():
        return None
    return 64.0 * (t["f64_add"] + t["f64_mul"] + t["f64_trans"] + 2.0 * t["f64_fma"]) + 512.0 * t["f64_mfma_mops"]


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


def host_cpu_info():
    """The host's processor model (lscpu), its logical CPU count, and the CPUs this process may use."""
    import subprocess

    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except Exception:
        allowed = os.cpu_count() or 1
    return {"lscpu_model": model, "nproc": os.cpu_count() or 1, "cpus_allowed": allowed}


# The GPU machine gives one GPU a share of 16 host CPUs, whatever nproc shows; the
# oracle's OpenMP threads stay within that share.
HOST_CPU_SHARE = 16


def oracle_rate(field, with_grad: bool, threads: int, target_s: float, seed: int = 12345):
    """Conditionals per second of the oracle on a random sample of the field's points grown until it takes
    about target_s / 2 .. target_s seconds (the whole field if that is quicker)."""
    import oracle

    rng = np.random.default_rng(seed)
    th = field.thetas[0]
    size = 64
    while True:
        idx = np.sort(rng.choice(field.n, size, replace=False)).astype(np.int64)
        t0 = time.perf_counter()
        oracle.terms(field.locs, field.z, field.nbr, field.m, field.nu, th, idx=idx, with_grad=with_grad,
                     threads=threads)
        elapsed = time.perf_counter() - t0
        if elapsed >= target_s * 0.5 or size >= field.n:
            return size, elapsed
        size = int(min(field.n, max(size * 2, size * target_s / max(elapsed, 1e-3) * 0.7)))


def cpu_baseline(field, with_grad: bool, target_s: float = 15.0):
    """The oracle on a bounded random sample of the workload's conditionals (same inputs), on every CPU of
    the host share, plus single-thread rates of the two forward-only workloads (2,000 points, m = 30, in
    full; the 250,000-point grid, m = 60, on a sample)."""
    import workloads as wl

    info = host_cpu_info()
    threads = max(1, min(info["cpus_allowed"], HOST_CPU_SHARE))
    size, elapsed = oracle_rate(field, with_grad, threads, target_s)
    single = {}
    small = wl.config_small().fields[0]
    s_size, s_el = oracle_rate(small, False, 1, 2.0)
    single["n2k_m30_nu0.5 value"] = {"conditionals_per_s": s_size / s_el, "sample": s_size, "seconds": s_el}
    grid = wl.config_grid(knn_threads=threads).fields[0]
    g_size, g_el = oracle_rate(grid, False, 1, 4.0)
    single["n250k_m60_nu1.5_grid value"] = {"conditionals_per_s": g_size / g_el, "sample": g_size,
                                            "seconds": g_el}
    return {"value": size / elapsed, "unit": "conditionals/s", "cores": threads, "kind": "oracle",
            "sample": f"{size} conditionals drawn uniformly from the {field.n}-point workload "
                      f"({'value+gradient' if with_grad else 'value'}), {elapsed:.1f} s",
            "host": info, "single_thread": single}


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


def event_ms(stream, fn, steps: int = 5, warmup: int = 2):
    """Mean and minimum HIP-event time (ms) of fn() on `stream` over `steps` runs after `warmup`."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.mean(ts)), float(min(ts))


def grid_forward_times(v, stream):
    """The 250,000-point jittered grid, m = 60, Matern nu = 3/2, theta = (1, 0.05, 1e-6): one forward
    (value-only) evaluation per call, the default variant."""
    import torch

    import workloads as wl

    w = wl.config_grid(knn_threads=min(os.cpu_count() or 1, HOST_CPU_SHARE))
    f = w.fields[0]
    dev = torch.device("cuda:0")
    L, Z, N = (torch.from_numpy(a).to(dev) for a in (f.locs, f.z, f.nbr))
    th = torch.from_numpy(f.thetas[0].copy()).to(dev)
    ws = torch.empty(v.vecchia_workspace_size(f.n, f.m), dtype=torch.uint8, device=dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int64, device=dev)
    ms, ms_min = event_ms(stream, lambda: v.vecchia_loglik(L, Z, N, f.m, f.nu, th, out=out, status=st, ws=ws,
                                                             stream=stream), steps=10)
    if int(st.item()) != 0:
        raise RuntimeError(f"grid workload: status {int(st.item())}")
    flops, _, gbytes = workload_counts(f.n, f.m, False)
    names = {val: k for k, val in v.VARIANTS.items()}
    return {"workload": f"{w.name} value", "n": f.n, "m": f.m, "nu": f.nu, "ms": ms, "ms_min": ms_min,
            "cond_per_s": f.n / (ms * 1e-3), "algorithmic_tflops": flops / (ms * 1e-3) / 1e12,
            "frac": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, "gather_gb_per_s": gbytes / (ms * 1e-3) / 1e9,
            "variant": names.get(v.vecchia_get_variant(f.m, False)), "loglik": out.item()}


def multitheta_times(v, stream):
    """200,000 uniform points, m = 60, Matern nu = 5/2, 64 parameter vectors, value + gradient for each:
    64 per-call evaluations against one batched plan over the 64 vectors replayed from a graph."""
    import torch

    import workloads as wl

    w = wl.config_multitheta(knn_threads=min(os.cpu_count() or 1, HOST_CPU_SHARE))
    f = w.fields[0]
    P = f.thetas.shape[0]
    dev = torch.device("cuda:0")
    L, Z, N = (torch.from_numpy(a).to(dev) for a in (f.locs, f.z, f.nbr))
    thetas = torch.from_numpy(f.thetas.reshape(1, P, 3).copy()).to(dev)
    ws = torch.empty(v.vecchia_workspace_size(f.n, f.m), dtype=torch.uint8, device=dev)
    outs = torch.empty((P, 1), dtype=torch.float64, device=dev)
    grads = torch.empty((P, 3), dtype=torch.float64, device=dev)
    sts = torch.empty((P, 1), dtype=torch.int64, device=dev)

    def plain():
        for q in range(P):
            v.vecchia_loglik_grad(L, Z, N, f.m, f.nu, thetas[0, q], out=outs[q], grad=grads[q], status=sts[q],
                                  ws=ws, stream=stream)

    p_ms, p_min = event_ms(stream, plain, steps=3, warmup=1)

    def batched(lockstep):
        prev = v.set_lockstep(lockstep)
        try:
            plan = v.BatchedPlan([(L, Z, N, f.m)], P, f.nu, True)
        finally:
            v.set_lockstep(prev)
        b_out, b_grad, b_st = plan.outputs()
        graph = plan.capture(thetas, b_out, b_grad, b_st)
        b_ms, _ = event_ms(stream, lambda: graph.launch(stream), steps=3, warmup=1)
        torch.cuda.synchronize()
        ok = bool((b_st == 0).all())
        same = bool(torch.equal(b_out.reshape(-1), outs.reshape(-1))) and bool(torch.equal(b_grad.reshape(-1, 3),
                                                                                          grads))
        groups = plan.groups()
        graph.close()
        plan.close()
        return b_ms, ok, same, groups

    b_ms, b_ok, b_same, groups = batched(True)
    s_ms, s_ok, s_same, _ = batched(False)
    ok = bool((sts == 0).all()) and b_ok and s_ok
    flops, _, _ = workload_counts(f.n, f.m, True)
    conds = P * f.n
    return {"workload": f"{w.name} value+gradient", "n": f.n, "m": f.m, "nu": f.nu, "thetas": P,
            "plain_ms": p_ms, "batched_ms": b_ms, "plain_cond_per_s": conds / (p_ms * 1e-3),
            "batched_cond_per_s": conds / (b_ms * 1e-3), "batched_speedup": p_ms / b_ms,
            "batched_frac": P * flops / (b_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "plain_frac": P * flops / (p_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "vectors_per_workgroup": groups,
            "batched_one_vector_per_workgroup_ms": s_ms,
            "status_ok": ok, "batched_equals_plain_bitwise": b_same and s_same}


def m_sweep_times(v, stream, n: int = 250_000, ms=(10, 30, 60, 90, 120, 150), nu: float = 1.5):
    """The paper's m grid (Sec. V-D, Fig. 7) at a fixed n: uniform points in random order, Matern nu = 3/2,
    theta = (1, 0.1, 1e-4), value + gradient per call with the default variant; conditioning sets from the
    GPU search."""
    import torch

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(7001)
    L = torch.from_numpy(rng.uniform(size=(n, 2))).to(dev)
    Z = torch.from_numpy(rng.standard_normal(n)).to(dev)
    th = torch.tensor([1.0, 0.1, 1e-4], dtype=torch.float64, device=dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(3, dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int64, device=dev)
    names = {val: k for k, val in v.VARIANTS.items()}
    rows = []
    for m in ms:
        N = v.vecchia_knn(L, int(m), stream=stream)
        ws = torch.empty(v.vecchia_workspace_size(n, m), dtype=torch.uint8, device=dev)
        t, t_min = event_ms(stream, lambda: v.vecchia_loglik_grad(L, Z, N, m, nu, th, out=out, grad=grad, status=st,
                                                                   ws=ws, stream=stream))
        if int(st.item()) != 0:
            raise RuntimeError(f"m sweep m={m}: status {int(st.item())}")
        flops, _, _ = workload_counts(n, m, True)
        rows.append({"m": int(m), "ms": t, "cond_per_s": n / (t * 1e-3),
                     "algorithmic_tflops": flops / (t * 1e-3) / 1e12,
                     "frac": flops / (t * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                     "variant": names.get(v.vecchia_get_variant(int(m), True))})
        del N, ws
    return {"workload": f"n={n} uniform, Matern nu={nu}, value+gradient, m in {list(ms)}", "rows": rows}


def mle_times(v, stream, n: int = 20_000, m: int = 30, nu: float = 1.5):
    """Maximum-likelihood fit (Sec. V's use of the likelihood) of 20,000 uniform points, Matern 3/2, z ~ N(0, 1)
    i.i.d.: the line search with one trial step per device round trip against four; same estimate, wall
    time and round trips."""
    import torch

    rng = np.random.default_rng(7002)
    dev = torch.device("cuda:0")
    L = torch.from_numpy(rng.uniform(size=(n, 2))).to(dev)
    Z = torch.from_numpy(rng.standard_normal(n)).to(dev)
    N = v.vecchia_knn(L, m, stream=stream)
    out = {}
    for k in (1, 4):
        opt = v.mle_default_options()
        opt.trial_steps = k
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = v.vecchia_mle(L, Z, N, m, nu, (0.5, 0.3, 0.2), options=opt, stream=stream)
        sec = time.perf_counter() - t0
        out[f"trial_steps_{k}"] = {"seconds": sec, "iterations": r["iterations"], "evaluations": r["evaluations"],
                                   "round_trips": r["round_trips"], "theta": [float(x) for x in r["theta"]],
                                   "loglik": r["loglik"]}
    out["workload"] = f"n={n} uniform, m={m}, Matern nu={nu}, z iid N(0,1), start (0.5, 0.3, 0.2)"
    out["same_estimate"] = out["trial_steps_1"]["theta"] == out["trial_steps_4"]["theta"]
    return out


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
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads: the 250K grid forward pass, 64 parameter vectors at 200K "
                         "points, and the m sweep")
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
    # the headline is the faster of the two forms; the other is reported beside it
    main_form = min(results, key=lambda k: results[k][0])
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
    for form, (fw, fl, _, _, fv) in results.items():
        rec[form] = {"value": f.n * args.steps / fw, "ms_per_step": fw * 1e3 / args.steps,
                     "launch_ms": float(np.mean(fl)), "variant": names.get(fv, fv)}
    if len(results) == 2:
        rec["batched_over_plain"] = rec["plain"]["ms_per_step"] / rec["batched"]["ms_per_step"]
    if args.traffic_kib is not None:
        rec["roofline"]["traffic"] = (args.traffic_kib[0] + args.traffic_kib[1]) * 1024.0
    else:
        rec["roofline"]["traffic"] = measured_traffic_bytes(w.name, names.get(variant, variant))
    executed = measured_fp64_flops(w.name, names.get(variant, variant))
    if executed is not None:
        # counter-based FP64 rate beside the algorithmic one (covariance evaluation, repeated rows
        # and padding included), over the same live launch time
        rate = executed / (rec["roofline"]["launch_ms"] * 1e-3) / 1e12
        rec["roofline"]["executed_fp64"] = {"flops_per_launch": executed, "tflops": rate,
                                            "frac": rate / FP64_PEAK_TFLOPS, "source": "rocprofv3 --pmc"}
    if args.copy_probe:
        src = torch.empty(512 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_configs:
        rec["grid_forward"] = grid_forward_times(v, stream)
        rec["multitheta"] = multitheta_times(v, stream)
        rec["m_sweep"] = m_sweep_times(v, stream)
        rec["mle"] = mle_times(v, stream)
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
