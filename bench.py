"""Benchmark of the coverage-flow hot path on one MI355X.

One step = one full gradient pass of the large 2-D workload (T = 65536 samples of
a unicycle trajectory, M = 262144 reference samples from a 16-component Gaussian
mixture with a 10 % uniform floor): the debiased Sinkhorn divergence (eps = 0.002,
500 iterations) through its autograd form (value, gradient with respect to the
samples and to the reference weights: cross and trajectory-self solves plus the
extrapolation pass, with the reference self potential computed once per
reference outside the timed steps because it does not depend on the trajectory),
and the Stein flow on the same samples (mixture score, median bandwidth, T x T
sum).  Legs beside it: the 2-D gradient-field workload (T = 4096, M = 16384), the
3-D autograd workload (T = 16384, M = 65536), the Stein flow alone, the
256-problem ragged batch (eager and graph-replayed against plain calls) and the
FP64 oracle on the host cores.

Prints one JSON line.  `value` is the pair evaluations (one exp each) of the
step divided by the step's wall time on the GPU stream.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "T·M pair-evals/s per gradient pass; batched vs plain speedup at ≤1e-5 rel err"
# Roofline of the lagged sweep (the dominant kernel).  One point pair costs, on the
# vector ALU: d subtractions (x'_i - y'_j), d FMAs (squared distance with the
# shift folded in), 1 subtraction (key term), 1 add (accumulate) and 1 v_exp_f32.
# Per-CU issue rates per clock of those instructions on gfx950 (4 SIMDs per CU):
# v_add_f32 128 lanes, v_fma_f32 64 lanes, v_exp_f32 32 lanes (the live probe,
# ct_probe_alu_rates, measures them on the box and is reported beside the peak;
# the published 157.3 TFLOP/s FP32 counts packed FMAs, which these kernels do not
# use).  The FP32 matrix cores do not help: they issue exclusively of the VALU
# (measured overlap ratio 1.0) and sum products relative to the largest term.
NOMINAL_RATES = {"add": 128.0, "fma": 64.0, "exp": 32.0}
N_CU, CLOCK_HZ = 256, 2.4e9


def pair_mix(d: int, expanded: bool = False) -> dict:
    """Instructions per point pair of the lagged sweep: difference form (d
    subtractions, d FMAs, one subtraction, the exp, the accumulate) or expanded
    form (d FMAs, one add, the exp, the accumulate)."""
    if expanded:
        return {"add": 2.0, "fma": float(d), "exp": 1.0}
    return {"add": d + 2.0, "fma": float(d), "exp": 1.0}


def pair_roof(d: int, rates: dict, n_cu=N_CU, clock=CLOCK_HZ, mix=None) -> float:
    """Pairs per second when every CU issues the pair mix back to back."""
    clk_per_pair = sum(n / rates[k] for k, n in (mix or pair_mix(d)).items())
    return n_cu * clock / clk_per_pair


# The Stein flow's T x T sum (d = 2) issues per pair 2 subtractions, 1 multiply,
# 5 FMAs and 1 v_exp_f32 (from its compiled loop); the multiply is counted at the
# add rate, which gives the higher (stricter) peak.
STEIN_MIX = {"add": 3.0, "fma": 5.0, "exp": 1.0}


def sweep_source_hash() -> str:
    """Hash of what decides the sweeps' memory traffic: their sources and the stored
    schedule table (queries per lane, key splits, blocks, merge mode)."""
    h = hashlib.sha256()
    for f in (("csrc", "sweep_device.h"), ("csrc", "sweep.hip"), ("tuning", "mi355x.txt")):
        with open(os.path.join(ROOT, "paper_2511_11514_amd", *f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pairs_per_pass(T: int, M: int, K: int, debias=True, ref=True, value=True,
                   ref_cached=False) -> float:
    """Point pairs (one exp each) of one gradient pass: K iterations of the cross,
    trajectory-self and (unless cached) reference-self sweeps, then the final pass."""
    per_iter = 2.0 * T * M + (T * T if debias else 0) + (M * M if ref and not ref_cached else 0)
    final = T * M + (T * T if debias else 0) + ((T * M + (M * M if ref else 0)) if value else 0)
    return K * per_iter + final


def omp_threads() -> int:
    """Threads the oracle's OpenMP loops use: OMP_NUM_THREADS, else every CPU this
    process may run on."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    return int(v) if v.strip().isdigit() else len(os.sched_getaffinity(0))


_ONE_CORE = """
import json, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import oracle
import workloads as W
cfg = W.CONFIGS["roofline_2d"]
x, y, w, _g = W.config_inputs(cfg)
x = x[:{rows}]
logb = np.log(w.astype(np.float64) / np.sum(w, dtype=np.float64))
oracle.lse_update(x[:16], y, logb, np.zeros(len(y)), cfg.eps)
t0 = time.perf_counter()
oracle.lse_update(x, y, logb, np.zeros(len(y)), cfg.eps)
print(json.dumps({{"pairs": float(len(x)) * len(y), "s": time.perf_counter() - t0}}))
"""


def cpu_baseline(x, y, w, eps, iters_sample: int, one_core_rows: int = 2048) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the headline workload:
    `iters_sample` Sinkhorn iterations (cross and trajectory-self solves) and the
    final pass over the full inputs on every host thread, and one soft-min update
    of `one_core_rows` trajectory rows against all reference samples on one core
    (a child process with OMP_NUM_THREADS=1)."""
    import subprocess
    import numpy as np
    import oracle
    T, M = len(x), len(y)
    z = np.zeros(16)
    oracle.lse_update(x[:16], y[:16], z, z, eps)   # load the C library
    t0 = time.perf_counter()
    oracle.sinkhorn(x, y, w, eps=eps, iters=iters_sample, want_value=False, want_grad_w=False)
    dt = time.perf_counter() - t0
    pairs = pairs_per_pass(T, M, iters_sample, ref=False, value=False)
    res = {"value": pairs / dt, "unit": "pair-evals/s", "cores": omp_threads(), "kind": "oracle",
           "sample": f"same inputs (T={T}, M={M}), {iters_sample} Sinkhorn iterations of the "
                     f"cross and trajectory-self solves + the final pass (grad_x): "
                     f"{pairs:.3e} pairs in {dt:.1f} s"}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_CORE.format(root=ROOT, rows=one_core_rows)],
                       env=env, stdout=subprocess.PIPE, text=True, check=True)
    one = json.loads(r.stdout.strip().splitlines()[-1])
    res["one_core"] = {"value": one["pairs"] / one["s"], "unit": "pair-evals/s", "cores": 1,
                       "sample": f"one soft-min update of {one_core_rows} trajectory rows "
                                 f"against all {M} reference samples: {one['pairs']:.3e} pairs "
                                 f"in {one['s']:.2f} s"}
    return res


_ONE_CORE_CFG = """
import json, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import oracle
import workloads as W
cfg = W.CONFIGS[{name!r}]
x, y, w, _g = W.config_inputs(cfg, T={T}, M={M})
x = x[:{rows}]
logb = np.log(w.astype(np.float64) / np.sum(w, dtype=np.float64))
oracle.lse_update(x[:16], y, logb, np.zeros(len(y)), cfg.eps)
best = float("inf")
for _ in range(3):
    t0 = time.perf_counter()
    oracle.lse_update(x, y, logb, np.zeros(len(y)), cfg.eps)
    best = min(best, time.perf_counter() - t0)
print(json.dumps({{"pairs": float(len(x)) * len(y), "s": best}}))
"""


def oracle_configs(ct, torch, dev) -> None:
    """The FP64 oracle, as it stands, timed per workload on the host cores beside
    the GPU path on the same workload: one JSON line per workload with the
    oracle's rate on every host thread (a bounded sample: the whole pass where it
    takes seconds, else a few iterations of the same solves plus the final pass,
    scaled by pair counts), its rate on one core (a child process with one thread:
    one soft-min update of up to 2048 rows against all keys, best of three) and
    the GPU's time for one full pass (S, dS/dx and dS/dw; the batch: its
    gradients), best of three after a warm-up."""
    import subprocess
    import numpy as np
    import oracle
    import workloads as W
    threads = omp_threads()
    z = np.zeros(16)
    oracle.lse_update(np.zeros((16, 2)), np.zeros((16, 2)), z, z, 0.01)   # load the C library

    def gpu_best(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    def one_core(name, T=None, M=None, rows=2048):
        env = dict(os.environ, OMP_NUM_THREADS="1")
        code = _ONE_CORE_CFG.format(root=ROOT, name=name, T=T, M=M, rows=rows)
        r = subprocess.run([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE,
                           text=True, check=True)
        one = json.loads(r.stdout.strip().splitlines()[-1])
        return one["pairs"] / one["s"]

    for name, sample_iters in (("planner_2d", None), ("grad_2d", 10), ("autograd_3d", 2),
                               ("roofline_2d", 1)):
        cfg = W.CONFIGS[name]
        x, y, w, _g = W.config_inputs(cfg)
        T, M, K = len(x), len(y), cfg.iters
        it = K if sample_iters is None else sample_iters
        full = pairs_per_pass(T, M, K)
        t0 = time.perf_counter()
        oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=it)
        dt = time.perf_counter() - t0
        sample = pairs_per_pass(T, M, it)
        rate = sample / dt
        xt, yt, wt = (torch.as_tensor(a, device=dev) for a in (x, y, w))
        g = gpu_best(lambda: ct.sinkhorn_grad(xt, yt, wt, eps=cfg.eps, iters=K, value=True,
                                              grad_w=True), reps=1 if name == "roofline_2d" else 3)
        row = {"workload": name, "d": cfg.d, "T": T, "M": M, "K": K, "pairs_per_pass": full,
               "oracle_sample": f"{it} iterations + final pass ({sample:.3e} pairs) in {dt:.2f} s",
               "oracle_pairs_per_s": rate, "oracle_threads": threads,
               "oracle_s_per_pass": full / rate,
               "oracle_one_core_pairs_per_s": one_core(name), "gpu_s_per_pass": g,
               "gpu_over_oracle": (full / rate) / g}
        print(json.dumps(row), flush=True)
    # the ragged batch: 16 of its problems through the oracle (5 iterations each, scaled to
    # the batch's pair count), against the batched GPU path on the whole batch
    cfg = W.CONFIGS["batched_2d"]
    probs = W.batch_inputs(cfg)
    full = sum(pairs_per_pass(len(p[0]), len(p[1]), cfg.iters, ref=False, value=False)
               for p in probs)
    pick = list(range(0, len(probs), 16))
    t0 = time.perf_counter()
    sample = 0.0
    for b in pick:
        xb, yb, wb = probs[b]
        oracle.sinkhorn(xb, yb, wb, eps=cfg.eps, iters=5, want_value=False, want_grad_w=False)
        sample += pairs_per_pass(len(xb), len(yb), 5, ref=False, value=False)
    dt = time.perf_counter() - t0
    rate = sample / dt
    xs = [torch.as_tensor(p[0], device=dev) for p in probs]
    ys = [torch.as_tensor(p[1], device=dev) for p in probs]
    bs = ct.BatchedSinkhorn(xs, ys, None, eps=cfg.eps, iters=cfg.iters)
    g = gpu_best(bs.run)
    print(json.dumps({"workload": "batched_2d", "problems": len(probs), "K": cfg.iters,
                      "pairs_per_batch": full,
                      "oracle_sample": f"{len(pick)} problems x 5 iterations + final pass "
                                       f"({sample:.3e} pairs) in {dt:.2f} s",
                      "oracle_pairs_per_s": rate, "oracle_threads": threads,
                      "oracle_s_per_batch": full / rate, "gpu_s_per_batch": g,
                      "gpu_over_oracle": (full / rate) / g}), flush=True)


def read_profile(L, _lib) -> list:
    """Launch records of ct_profile_*: (kind0, kind1, pairs, ms) per launch."""
    kind = (ctypes.c_int32 * 4)()
    pr, t = ctypes.c_double(), ctypes.c_float()
    out = []
    for i in range(L.ct_profile_count()):
        _lib.check("ct_profile_read", L.ct_profile_read(i, kind, ctypes.byref(pr), ctypes.byref(t)))
        out.append((kind[0], kind[1], pr.value, t.value))
    L.ct_profile_clear()
    return out


def dominant_sweeps(recs) -> tuple:
    """(pairs, ms, launches) of the lagged-shift sweeps without offsets."""
    sel = [r for r in recs if r[0] == 1 and r[1] == 0]
    return sum(r[2] for r in sel), sum(r[3] for r in sel), len(sel)


def sinkhorn_step(ct, x, y, w, eps, K, gmm=None, ref_q=None, one_stream=False, expanded=True):
    """One gradient pass: S, dS/dx and dS/dw through the autograd form, then the
    Stein flow on the same samples when a mixture is given."""
    def step():
        xr = x.detach().requires_grad_(True)
        wr = w.detach().requires_grad_(True)
        S = ct.sinkhorn_divergence(xr, y, wr, eps=eps, iters=K, one_stream=one_stream,
                                   ref_q=ref_q, expanded=expanded)
        S.backward()
        out = [S, xr.grad, wr.grad]
        if gmm is not None:
            out.append(ct.svgd_grad(x, gmm)[0])
        return out
    return step


def rel_err(a, b) -> float:
    import numpy as np
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=2,
                    help="Sinkhorn iterations of the CPU oracle sample (large workload)")
    ap.add_argument("--no-legs", action="store_true",
                    help="only the headline step (no 2-D, 3-D, Stein and batched legs)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--two-stream", action="store_true",
                    help="run the self sweeps of the headline step on the library's auxiliary "
                         "stream (default: one stream, as every launch fills the GPU)")
    ap.add_argument("--events-separately", action="store_true",
                    help="take the per-launch events in one extra step instead of in the timed "
                         "steps")
    ap.add_argument("--autotune", action="store_true",
                    help="re-tune the sweep schedules instead of loading the stored tuning table")
    ap.add_argument("--graph", action="store_true",
                    help="also time the 2-D leg's step captured into a HIP graph (replays)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy a 256 MiB buffer (reference kernel for HBM counters)")
    ap.add_argument("--horizon-sweep", action="store_true",
                    help="instead of the benchmark line: planner time versus horizon (the "
                         "paper's timing benchmark shape), one JSON line per horizon")
    ap.add_argument("--ensemble", action="store_true",
                    help="instead of the benchmark line: a 16-seed planner ensemble in lockstep "
                         "(one batched flow launch per outer iteration) against 16 plain runs")
    ap.add_argument("--grid", action="store_true",
                    help="instead of the benchmark line: flows toward a continuous utility map "
                         "on a grid (Stein flow on its score, Sinkhorn flow on its weighted nodes)")
    ap.add_argument("--grad-2d-only", action="store_true",
                    help="instead of the benchmark line: only the 2-D gradient-field leg "
                         "(T = 4096, M = 16384), for profiling its launches")
    ap.add_argument("--difference", action="store_true",
                    help="headline step with the lagged sweeps' exponent in the difference "
                         "form (CT_DIFFERENCE; default: the expanded form); the roof follows "
                         "its pair mix")
    ap.add_argument("--oracle-configs", action="store_true",
                    help="instead of the benchmark line: the FP64 oracle timed per workload on "
                         "the host cores (all threads and one core) beside the GPU's full pass")
    ap.add_argument("--stein-only", action="store_true",
                    help="instead of the benchmark line: only the Stein leg (T = 65536), for "
                         "profiling its median and sum kernels")
    ap.add_argument("--batched-only", action="store_true",
                    help="instead of the benchmark line: only the batched leg (256 uneven "
                         "problems), for profiling its launches")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2511_11514_amd as ct
    import workloads as W
    from paper_2511_11514_amd import _lib

    dev = torch.device("cuda:0")
    if args.horizon_sweep:
        horizon_sweep(ct, torch, dev)
        return 0
    if args.ensemble:
        ensemble_leg(ct, torch, dev)
        return 0
    if args.grid:
        grid_leg(ct, torch, dev)
        return 0
    if args.oracle_configs:
        ct.tuning_load(os.path.join(ROOT, "paper_2511_11514_amd", "tuning", "mi355x.txt"))
        oracle_configs(ct, torch, dev)
        return 0
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    L = _lib.lib()
    # sweep schedules: the stored table written by the autotuner on an MI355X
    table = os.path.join(ROOT, "paper_2511_11514_amd", "tuning", "mi355x.txt")
    tuned = "stored table " + os.path.relpath(table, ROOT)
    if args.autotune or not os.path.exists(table):
        tuned = None
    else:
        ct.tuning_load(table)
    if args.stein_only:
        print(json.dumps(stein_leg(ct, torch, dev, L, _lib)))
        return 0
    if args.grad_2d_only:
        print(json.dumps(grad_2d_leg(ct, torch, dev, L, _lib, tuned, steps=args.steps,
                                     warmup=args.warmup, graph=args.graph)))
        return 0
    if args.batched_only:
        print(json.dumps(batched_leg(ct, torch, dev, reps=max(1, args.steps))))
        return 0

    # headline: one gradient pass of the large 2-D workload (unicycle trajectory
    # samples T = 65536, M = 262144 reference samples of a 16-component mixture with
    # a 10 % uniform floor, eps = 0.002, K = 500): S, dS/dx, dS/dw through autograd
    # with the reference self potential computed once per reference (it does not
    # depend on the trajectory), plus the Stein flow on the same samples
    cfg = W.CONFIGS["roofline_2d"]
    T, M, d, eps, K = cfg.T, cfg.M, cfg.d, cfg.eps, cfg.iters
    x_np, y_np, w_np, g_np = W.config_inputs(cfg)
    x = torch.as_tensor(x_np, device=dev)
    y = torch.as_tensor(y_np, device=dev)
    w = torch.as_tensor(w_np, device=dev)
    gmm = ct.GMM.from_numpy(g_np, dev)
    if tuned is None:
        ct.autotune_sinkhorn(T, M, d, eps)
        tuned = "autotuned in this run"
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ref_q = ct.reference_self_potential(y, w, eps=eps, iters=K)
    e1.record()
    torch.cuda.synchronize()
    ref_ms = e0.elapsed_time(e1)
    print(f"# reference self potential: {ref_ms:.0f} ms", file=sys.stderr, flush=True)
    step = sinkhorn_step(ct, x, y, w, eps, K, gmm=gmm, ref_q=ref_q,
                         one_stream=not args.two_stream, expanded=not args.difference)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"# warm-up step {i + 1}/{args.warmup}", file=sys.stderr, flush=True)
    live_events = not args.events_separately
    L.ct_profile_clear()
    if live_events:
        L.ct_profile_enable(1)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        out = step()
    e1.record()
    torch.cuda.synchronize()
    L.ct_profile_enable(0)
    ms = e0.elapsed_time(e1) / args.steps
    print(f"# timed {args.steps} steps: {ms:.1f} ms each", file=sys.stderr, flush=True)
    assert all(torch.isfinite(t).all().item() for t in out)
    if not live_events:
        L.ct_profile_enable(1)
        step()
        torch.cuda.synchronize()
        L.ct_profile_enable(0)
    recs = read_profile(L, _lib)
    dom_pairs, dom_ms, n_dom = dominant_sweeps(recs)
    sk_pairs = pairs_per_pass(T, M, K, ref_cached=True)
    svgd_pairs = T * T
    total_pairs = sk_pairs + svgd_pairs
    ach = dom_pairs / (dom_ms * 1e-3) / 1e12
    mix = pair_mix(d, not args.difference)
    peak = pair_roof(d, NOMINAL_RATES, mix=mix) / 1e12
    probe = ct.probe_alu_rates(str(dev))
    probe_peak = pair_roof(d, probe, clock=probe["clock_hz"], mix=mix) / 1e12
    traffic = None
    tf = os.path.join(ROOT, "profiles", "sweep_traffic_roofline_2d.json")
    if os.path.exists(tf):
        with open(tf) as fh:
            rec = json.load(fh)
        if rec.get("source_hash") == sweep_source_hash():
            traffic = rec.get("bytes_per_launch")

    res = {
        "metric": METRIC,
        "value": total_pairs / (ms * 1e-3),
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"roofline_2d: d=2 T={T} unicycle-trajectory samples, M={M} reference "
                        f"samples (16-component GMM + 10% uniform floor), Sinkhorn eps={eps} "
                        f"K={K} debiased, S + dS/dx + dS/dw via autograd with the reference "
                        f"self potential cached per reference, plus Stein flow (median "
                        f"bandwidth)",
            "pairs_per_step": total_pairs,
            "sinkhorn_pairs": sk_pairs,
            "svgd_pairs": svgd_pairs,
            "tm_pair_evals_per_s": K * T * M / (ms * 1e-3),
            "streams": 2 if args.two_stream else 1,
            "schedules": tuned,
            "reference_self_potential_ms": ref_ms,
            "reference_self_pairs": float(K) * M * M,
        },
        "roofline": {
            "bound": "alu",
            "kernel": f"k_sweep (lagged shift, no offsets, d={d}"
                      f"{', difference form' if args.difference else ', expanded exponent'})",
            "achieved": ach,
            "peak": peak,
            "unit": "Tpair/s",
            "frac": ach / peak,
            "traffic": traffic,
            "launches": n_dom,
            "avg_launch_us": dom_ms / max(n_dom, 1) * 1e3,
            "events": "in the timed steps" if live_events else "one extra step",
            "pair_mix": mix,
            "nominal_lanes_per_clk_per_cu": NOMINAL_RATES,
            "probe": {k: round(v, 4) for k, v in probe.items()},
            "probe_peak": probe_peak,
            "frac_of_probe_peak": ach / probe_peak,
        },
    }
    res["parity"] = parity_roofline_2d(out, x_np)
    res["system"] = system_info(torch, dev)
    del out, step, ref_q
    if not args.no_legs:
        res["grad_2d"] = grad_2d_leg(ct, torch, dev, L, _lib, tuned, graph=args.graph)
        print("# 2-D leg done", file=sys.stderr, flush=True)
        res["autograd_3d"] = autograd_3d_leg(ct, torch, dev)
        print("# 3-D leg done", file=sys.stderr, flush=True)
        res["stein"] = stein_leg(ct, torch, dev, L, _lib)
        if not args.no_batched:
            res["batched"] = batched_leg(ct, torch, dev)
            print("# batched leg done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(x_np, y_np, w_np, eps, args.cpu_iters)
    print(json.dumps(res))
    return 0


def parity_roofline_2d(out, x_np) -> dict:
    """The headline step's gradient against the stored FP64 oracle pass over the
    same inputs (tests/golden/roofline_2d_full.npz, written by the fixture script
    from the oracle alone; it holds the cross and trajectory-self solves, so the
    gradient with respect to the samples, not the value or weight gradient)."""
    import numpy as np
    f = os.path.join(ROOT, "tests", "golden", "roofline_2d_full.npz")
    if not os.path.exists(f):
        return {"tolerance": 1e-5, "reference": None}
    F = np.load(f, allow_pickle=False)
    return {"tolerance": 1e-5, "reference": "FP64 oracle, tests/golden/roofline_2d_full.npz",
            "grad_x": rel_err(out[1].cpu().numpy(), F["grad_x"])}


def grad_2d_leg(ct, torch, dev, L, _lib, tuned, steps: int = 20, warmup: int = 3,
                graph: bool = False) -> dict:
    """The 2-D gradient-field workload (T = 4096 random-walk samples, M = 16384
    samples of a 5-component mixture, eps = 0.005, K = 200): S, dS/dx, dS/dw through
    autograd (cross, self and reference-self solves) plus the Stein flow, on two
    streams; its lagged sweeps' launch times from events in one more step; errors
    against the stored FP64 oracle pass."""
    import workloads as W
    cfg = W.CONFIGS["grad_2d"]
    T, M, d, eps, K = cfg.T, cfg.M, cfg.d, cfg.eps, cfg.iters
    x_np, y_np, w_np, g_np = W.config_inputs(cfg)
    x, y, w = (torch.as_tensor(a, device=dev) for a in (x_np, y_np, w_np))
    gmm = ct.GMM.from_numpy(g_np, dev)
    step = sinkhorn_step(ct, x, y, w, eps, K, gmm=gmm)
    one = sinkhorn_step(ct, x, y, w, eps, K, gmm=gmm, one_stream=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        out = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    graph_ms = None
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            gout = step()
        gr.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            gr.replay()
        e1.record()
        torch.cuda.synchronize()
        graph_ms = e0.elapsed_time(e1) / steps
        assert torch.equal(gout[1], out[1])
    L.ct_profile_clear()
    L.ct_profile_enable(1)
    one()
    torch.cuda.synchronize()
    L.ct_profile_enable(0)
    dp, dms, nd = dominant_sweeps(read_profile(L, _lib))
    pairs = pairs_per_pass(T, M, K) + T * T
    ach = dp / (dms * 1e-3) / 1e12
    peak = pair_roof(d, NOMINAL_RATES, mix=pair_mix(d, True)) / 1e12
    traffic = None
    tf = os.path.join(ROOT, "profiles", "sweep_traffic_grad_2d.json")
    if os.path.exists(tf):
        with open(tf) as fh:
            rec = json.load(fh)
        if rec.get("source_hash") == sweep_source_hash():
            traffic = rec.get("bytes_per_launch")
    return {"workload": f"grad_2d: d=2 T={T} M={M}, Sinkhorn eps={eps} K={K} debiased, S + "
                        f"dS/dx + dS/dw via autograd (two streams), plus Stein flow",
            "ms_per_step": ms, "pairs_per_step": pairs, "pair_evals_per_s": pairs / (ms * 1e-3),
            "graph_ms_per_step": graph_ms, "schedules": tuned,
            "sweep_launches": {"achieved": ach, "peak": peak, "unit": "Tpair/s",
                               "frac": ach / peak, "launches": nd,
                               "avg_launch_us": dms / max(nd, 1) * 1e3, "traffic": traffic,
                               "events": "one extra step, launches serialised on one stream"},
            "parity": parity_vs_stored_oracle(out, ct, torch, dev)}


def planner_2d_row(ct, torch, dev, reps: int = 3) -> None:
    """The 2-D planner workload (double integrator, T = 256, M = 512, eps = 0.01,
    K = 100, ten outer iterations, step 0.5): ct_plan wall time per outer
    iteration with the library's default execution (the exchange solve at this
    size) and with one launch per sweep, best of `reps` runs after a warm-up call."""
    import numpy as np
    import workloads as W
    cfg = W.CONFIGS["planner_2d"]
    e = cfg.extra
    _x, y, w, _g = W.config_inputs(cfg)
    u0 = np.random.default_rng(cfg.seed + 1).normal(size=(cfg.T, 2)) * e["u_std"]
    s0 = np.array(e["s0"])
    Q, R = e["Q"] * np.eye(2), e["R"] * np.eye(2)
    kw = dict(y=torch.as_tensor(y, device=dev), w=torch.as_tensor(w, device=dev), eps=cfg.eps,
              iters=cfg.iters)
    row = {"workload": "planner_2d", "T": cfg.T, "M": cfg.M, "K": cfg.iters, "outer": e["outer"]}
    for key, fused in (("default", None), ("unfused", False)):
        ct.plan(e["dynamics"], s0, u0, e["dt"], Q, R, "sinkhorn", 1, 0.5, fused=fused, **kw)
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            _u, _s, hist = ct.plan(e["dynamics"], s0, u0, e["dt"], Q, R, "sinkhorn", e["outer"],
                                   0.5, fused=fused, **kw)
            best = min(best, time.perf_counter() - t0)
        row[f"ms_per_outer_{key}"] = 1e3 * best / e["outer"]
        row[f"objective_{key}"] = [float(hist[0]), float(hist[-1])]
    row["unfused_over_default"] = row["ms_per_outer_unfused"] / row["ms_per_outer_default"]
    print(json.dumps(row), flush=True)


def horizon_sweep(ct, torch, dev) -> None:
    """Planner wall time against the horizon T: the Stein flow with differential
    drive and the Sinkhorn flow with the 3-D point mass (stand-in for the paper's
    aircraft), each for its sweep's outer iterations on the GPU (flow on the GPU,
    LQR on the host, ct_plan), beside one outer iteration of the FP64 oracle planner
    on the host cores (bounded: Stein up to T = 5000)."""
    import numpy as np
    import oracle
    import workloads as W
    cpu_limit = {"svgd_drive": 5000, "sinkhorn_aircraft": 2500}
    threads = omp_threads()
    planner_2d_row(ct, torch, dev)
    for name, c in W.HORIZON_SWEEPS.items():
        warm = True
        for T in c["horizons"]:
            s0, u0, y, w, g = W.horizon_inputs(name, T)
            d = c["d"]
            Q, R = c["Q"] * np.eye(d), c["R"] * np.eye(u0.shape[1])
            if c["flow"] == "svgd":
                kw = dict(gmm=ct.GMM.from_numpy(g, dev))
                okw = dict(gmm=g)
            else:
                kw = dict(y=torch.as_tensor(y, device=dev), w=torch.as_tensor(w, device=dev),
                          eps=c["eps"], iters=c["iters"])
                okw = dict(y=y, w=w, eps=c["eps"], iters=c["iters"])
            ct.plan(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"], 1, c["step"], **kw)  # warm-up
            # best of three up to 1000 samples (a run there is a few ms and noisy)
            reps = 3 if T <= 1000 else 1
            gpu = float("inf")
            for _ in range(reps):
                t0 = time.perf_counter()
                _u, _s, hist = ct.plan(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"],
                                       c["outer"], c["step"], **kw)
                gpu = min(gpu, time.perf_counter() - t0)
            row = {"sweep": name, "flow": c["flow"], "dynamics": c["dynamics"], "d": d, "T": T,
                   "M": None if y is None else len(y), "outer": c["outer"], "gpu_s": gpu,
                   "gpu_s_per_outer": gpu / c["outer"], "first_objective": float(hist[0]),
                   "last_objective": float(hist[-1])}
            if c["flow"] == "sinkhorn":
                # the same planner with one launch per sweep
                ct.plan(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"], 1, c["step"],
                        fused=False, **kw)
                gpu2 = float("inf")
                for _ in range(reps):
                    t0 = time.perf_counter()
                    _u2, _s2, hist2 = ct.plan(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"],
                                              c["outer"], c["step"], fused=False, **kw)
                    gpu2 = min(gpu2, time.perf_counter() - t0)
                row.update({"gpu_s_per_outer_unfused": gpu2 / c["outer"],
                            "unfused_over_default": gpu2 / gpu,
                            "last_objective_unfused": float(hist2[-1])})
            if T <= cpu_limit[name]:
                if warm or T <= 1000:
                    # untimed call first: the oracle's first call loads its C library, and
                    # the first calls at a new size start its thread pool and page in memory
                    oracle.plan_step(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"],
                                     step=c["step"], **okw)
                    warm = False
                # best of three below 1000 samples (single runs there are a few ms and noisy)
                cpu = float("inf")
                for _ in range(3 if T <= 1000 else 1):
                    t0 = time.perf_counter()
                    oracle.plan_step(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"],
                                     step=c["step"], **okw)
                    cpu = min(cpu, time.perf_counter() - t0)
                row.update({"cpu_oracle_s_per_outer": cpu, "cpu_threads": threads,
                            "oracle_over_gpu": cpu / (gpu / c["outer"])})
            print(json.dumps(row), flush=True)


def ensemble_leg(ct, torch, dev, S: int = 16, T: int = 1000) -> None:
    """Seed ensemble of the Sinkhorn planner (3-D point-mass workload of the horizon
    sweep, T = M = 1000, 10 outer iterations): ct_plan_ensemble against S
    sequential ct_plan runs from the same seeds."""
    import numpy as np
    import workloads as W
    c = W.HORIZON_SWEEPS["sinkhorn_aircraft"]
    s0, _u0, y, w, _g = W.horizon_inputs("sinkhorn_aircraft", T)
    rng = np.random.default_rng(321)
    U0 = rng.normal(size=(S, T, c["d"])) * c["u_std"] * rng.uniform(0.5, 3.0, size=(S, 1, 1))
    Q, R = c["Q"] * np.eye(c["d"]), c["R"] * np.eye(c["d"])
    yt, wt = torch.as_tensor(y, device=dev), torch.as_tensor(w, device=dev)
    kw = dict(y=yt, w=wt, eps=c["eps"], iters=c["iters"])
    ct.plan_ensemble(c["dynamics"], s0, U0[:2], c["dt"], Q, R, 1, c["step"], **kw)  # warm-up
    ct.plan(c["dynamics"], s0, U0[0], c["dt"], Q, R, "sinkhorn", 1, c["step"], **kw)
    t0 = time.perf_counter()
    _U, _s, values, best = ct.plan_ensemble(c["dynamics"], s0, U0, c["dt"], Q, R, c["outer"],
                                            c["step"], **kw)
    t_ens = time.perf_counter() - t0
    t0 = time.perf_counter()
    for b in range(S):
        ct.plan(c["dynamics"], s0, U0[b], c["dt"], Q, R, "sinkhorn", c["outer"], c["step"], **kw)
    t_seq = time.perf_counter() - t0
    print(json.dumps({"ensemble": "sinkhorn_aircraft", "seeds": S, "T": T, "M": T,
                      "outer": c["outer"], "ensemble_s": t_ens, "sequential_s": t_seq,
                      "speedup": t_seq / t_ens, "best": best, "best_value": float(values[best]),
                      "worst_value": float(values.max()),
                      "median_value": float(np.median(values))}), flush=True)


def grid_leg(ct, torch, dev, reps: int = 20) -> None:
    """Flows toward a continuous utility map (a grid of node values over the unit
    box): the Stein flow on the map's score at the Stein sweep's largest horizon
    (T = 10000, 256 x 256 nodes), and the Sinkhorn flow on the map's weighted nodes
    at the benchmark workload's T, eps and iterations (128 x 128 nodes), each timed
    over `reps` evaluations, with the FP64 oracle beside them on a bounded sample."""
    import numpy as np
    import oracle
    import workloads as W
    threads = omp_threads()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    # Stein flow: score of the interpolated map, then the T x T sum
    T = 10000
    u, lo, hi = W.utility_map(np.random.default_rng(8100), (256, 256))
    grid = ct.UtilityGrid(torch.as_tensor(u, device=dev), list(lo), list(hi), 0.0)
    x = W.random_walk(np.random.default_rng(8101), T, 2)
    xt = torch.as_tensor(x, device=dev)
    t_score = timed(lambda: ct.grid_score(xt, grid))
    t_flow = timed(lambda: ct.svgd_grad_score(xt, ct.grid_score(xt, grid)))
    og = oracle.grid.Grid(u.astype(np.float64), lo.astype(np.float64), hi.astype(np.float64), 0.0)
    Tc = 5000
    xc = x[:Tc].astype(np.float64)
    oracle.svgd_phi(xc[:500], oracle.grid.score(og, xc[:500]), 0.01)        # load the library
    t0 = time.perf_counter()
    oracle.svgd_phi(xc, oracle.grid.score(og, xc), oracle.median_bandwidth(xc))
    t_cpu = time.perf_counter() - t0
    print(json.dumps({"grid_leg": "stein", "T": T, "grid": [256, 256], "score_ms": 1e3 * t_score,
                      "flow_ms": 1e3 * t_flow, "pairs_per_s": T * T / t_flow,
                      "cpu_oracle_ms": 1e3 * t_cpu, "cpu_sample": f"T={Tc}",
                      "cpu_threads": threads}), flush=True)

    # Sinkhorn flow: the map's weighted nodes as the reference
    cfg = W.CONFIGS["grad_2d"]
    u2, lo2, hi2 = W.utility_map(np.random.default_rng(8102), (128, 128))
    grid2 = ct.UtilityGrid(torch.as_tensor(u2, device=dev), list(lo2), list(hi2), 0.0)
    t_samples = timed(lambda: ct.grid_samples(grid2))
    y, w = ct.grid_samples(grid2)
    xs, _y, _w, _g = W.config_inputs(cfg)
    xst = torch.as_tensor(xs, device=dev)
    t_sk = timed(lambda: ct.sinkhorn_grad(xst, y, w, eps=cfg.eps, iters=cfg.iters, grad_w=True,
                                          value=True))
    ry, rw = oracle.grid.samples(oracle.grid.Grid(u2.astype(np.float64), lo2.astype(np.float64),
                                                  hi2.astype(np.float64), 0.0))
    it_cpu = 10
    t0 = time.perf_counter()
    oracle.sinkhorn(xs, ry.astype(np.float32).astype(np.float64), rw, eps=cfg.eps, iters=it_cpu)
    t_cpu2 = (time.perf_counter() - t0) * cfg.iters / it_cpu
    print(json.dumps({"grid_leg": "sinkhorn", "T": cfg.T, "M": int(y.shape[0]),
                      "grid": [128, 128], "eps": cfg.eps, "iters": cfg.iters,
                      "samples_ms": 1e3 * t_samples, "flow_ms": 1e3 * t_sk,
                      "cpu_oracle_ms": 1e3 * t_cpu2,
                      "cpu_sample": f"{it_cpu} iterations scaled to {cfg.iters}",
                      "cpu_threads": threads}), flush=True)


def parity_vs_stored_oracle(out, ct, torch, dev) -> dict:
    """Norm-wise relative errors of the timed step's last outputs against the FP64
    oracle's pass over the same inputs, stored in tests/golden (written by the
    fixture script from the oracle only).  The stored Stein flow was taken on the
    workload's samples drawn beside a 16-point reference, so it is checked with one
    more call on those inputs."""
    import workloads as W
    import numpy as np
    res = {"tolerance": 1e-5, "reference": "FP64 oracle, tests/golden/grad_2d_full*.npz"}

    def rel(a, b):
        a = np.asarray(a, np.float64).ravel()
        b = np.asarray(b, np.float64).ravel()
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    gold = os.path.join(ROOT, "tests", "golden")
    F = np.load(os.path.join(gold, "grad_2d_full.npz"))
    res["value"] = abs(float(out[0].item()) - float(F["value"])) / abs(float(F["value"]))
    res["grad_x"] = rel(out[1].cpu().numpy(), F["grad_x"])
    res["grad_w"] = rel(out[2].cpu().numpy(), F["grad_w"])
    if len(out) > 3:
        G = np.load(os.path.join(gold, "grad_2d_full_svgd.npz"))
        x, _y, _w, g = W.config_inputs(W.CONFIGS[str(G["workload"])], T=int(G["T"]), M=16)
        phi, _h = ct.svgd_grad(torch.as_tensor(x, device=dev), ct.GMM.from_numpy(g, dev))
        res["stein_phi"] = rel(phi.cpu().numpy(), G["phi"])
    return res


def system_info(torch, dev) -> dict:
    cpu = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"gpu": torch.cuda.get_device_name(dev), "host_cpu": cpu,
            "host_threads": os.cpu_count()}


def autograd_3d_leg(ct, torch, dev, reps: int = 2) -> dict:
    """The autograd form at its 3-D workload (T = 16384 random-walk samples, M = 65536
    samples of an anisotropic 8-component mixture, eps = 0.01, K = 300): S with
    dS/dx and dS/dw through torch.autograd, whole-pass time and pair throughput
    against the 3-D issue roof."""
    import workloads as W
    cfg = W.CONFIGS["autograd_3d"]
    x, y, w, _g = W.config_inputs(cfg)
    T, M, K = len(x), len(y), cfg.iters
    xt, yt, wt = (torch.as_tensor(a, device=dev) for a in (x, y, w))

    def step():
        xr = xt.detach().requires_grad_(True)
        wr = wt.detach().requires_grad_(True)
        S = ct.sinkhorn_divergence(xr, yt, wr, eps=cfg.eps, iters=K)
        S.backward()
        return xr.grad

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g = step()
    e1.record()
    torch.cuda.synchronize()
    assert torch.isfinite(g).all().item()
    ms = e0.elapsed_time(e1) / reps
    pairs = pairs_per_pass(T, M, K)
    # the expanded pair mix of the lagged sweeps (the stricter roof for the whole pass)
    peak = pair_roof(3, NOMINAL_RATES, mix=pair_mix(3, True)) / 1e12
    rate = pairs / (ms * 1e-3) / 1e12
    return {"workload": f"autograd_3d: d=3 T={T} M={M} eps={cfg.eps} K={K}, S + dS/dx + dS/dw "
                        "through autograd", "ms_per_pass": ms, "pairs_per_pass": pairs,
            "pair_evals_per_s": rate * 1e12, "peak": peak, "unit": "Tpair/s",
            "frac_of_peak": rate / peak}


def stein_leg(ct, torch, dev, L, _lib) -> dict:
    """The Stein flow at the large workload's size (T = 65536, 16-component mixture
    with a 10 % floor, median bandwidth): whole-flow time, the time with the
    bandwidth given (no median), and the T x T sum kernel against its issue roof
    (events stamped with the kernel's start and end)."""
    import workloads as W
    cfg = W.CONFIGS["roofline_2d"]
    x, _y, _w, g = W.config_inputs(cfg, M=16)
    T = len(x)
    xt = torch.as_tensor(x, device=dev)
    gm = ct.GMM.from_numpy(g, dev)

    def timed(h, reps=3):
        out = ct.svgd_grad(xt, gm, h)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = ct.svgd_grad(xt, gm, h)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    flow_ms, (_phi, hu) = timed(None)
    h = float(hu.item())
    fixed_ms, _ = timed(h)
    L.ct_profile_clear()
    L.ct_profile_enable(1)
    ct.svgd_grad(xt, gm, h)
    torch.cuda.synchronize()
    L.ct_profile_enable(0)
    kind = (ctypes.c_int32 * 4)()
    pr, t = ctypes.c_double(), ctypes.c_float()
    sum_ms = None
    for i in range(L.ct_profile_count()):
        _lib.check("ct_profile_read", L.ct_profile_read(i, kind, ctypes.byref(pr), ctypes.byref(t)))
        if kind[0] == 2:
            sum_ms = t.value
    L.ct_profile_clear()
    peak = pair_roof(2, NOMINAL_RATES, mix=STEIN_MIX) / 1e12
    ach = T * T / (sum_ms * 1e-3) / 1e12 if sum_ms else None
    return {"workload": f"roofline_2d Stein flow: T={T}, 16-component mixture + 10% floor",
            "flow_ms": flow_ms, "flow_fixed_h_ms": fixed_ms, "median_ms": flow_ms - fixed_ms,
            "sum_kernel": {"us": None if sum_ms is None else sum_ms * 1e3, "achieved": ach,
                           "peak": peak, "unit": "Tpair/s",
                           "frac": None if ach is None else ach / peak, "pair_mix": STEIN_MIX}}


def batched_leg(ct, torch, dev, reps: int = 3) -> dict:
    """The 256-problem ragged batch (T_b in [500, 8000], M_b in [1024, 32768], eps =
    0.01, K = 150, debiased gradient): the batched path (lockstep launches over job
    tables, two sweep launches per iteration) run eagerly and as a captured HIP
    graph replayed, against 256 plain calls; accuracy against the plain calls and
    against the stored FP64 oracle passes of 16 of the problems."""
    import numpy as np
    import workloads as W
    cfg = W.CONFIGS["batched_2d"]
    probs = W.batch_inputs(cfg)
    eps, K = cfg.eps, cfg.iters
    xs = [torch.as_tensor(p[0], device=dev) for p in probs]
    ys = [torch.as_tensor(p[1], device=dev) for p in probs]
    bs = ct.BatchedSinkhorn(xs, ys, None, eps=eps, iters=K)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_b = timed(bs.run)
    eager = bs.grad_x.clone()
    gr = bs.capture()
    t_g = timed(gr.replay)
    graph_equal = bool(torch.equal(bs.grad_x, eager))
    plain = [None] * len(probs)

    def run_plain():
        for b in range(len(probs)):
            plain[b] = ct.sinkhorn_grad(xs[b], ys[b], None, eps=eps, iters=K).grad_x

    t_p = timed(run_plain)
    gx = bs.split(bs.grad_x, bs.T_off)
    err = max(float((gx[b] - plain[b]).norm() / plain[b].norm()) for b in range(len(probs)))
    oracle_err = None
    f = os.path.join(ROOT, "tests", "golden", "batched_2d_sample16.npz")
    if os.path.exists(f):
        F = np.load(f, allow_pickle=False)
        off = np.concatenate([[0], np.cumsum(F["T"])])
        oracle_err = max(rel_err(gx[int(b)].cpu().numpy(), F["grad_x"][off[i]:off[i + 1]])
                         for i, b in enumerate(F["problems"]))
    pairs = sum(K * (2.0 * len(p[0]) * len(p[1]) + len(p[0]) ** 2) + len(p[0]) * len(p[1]) +
                len(p[0]) ** 2 for p in probs)
    return {"workload": f"batched_2d: {len(probs)} problems, T in {cfg.extra['T_range']}, "
                        f"M in {cfg.extra['M_range']}, eps={eps}, K={K}, debiased grad_x",
            "pairs": pairs, "batched_ms": t_b, "graph_replay_ms": t_g, "plain_ms": t_p,
            "speedup": t_p / t_b, "graph_speedup": t_p / t_g,
            "batched_pair_evals_per_s": pairs / (t_b * 1e-3),
            "plain_pair_evals_per_s": pairs / (t_p * 1e-3),
            "graph_replay_equals_eager": graph_equal,
            "max_rel_diff_batched_vs_plain": err,
            "max_rel_err_vs_oracle_16_problems": oracle_err}


if __name__ == "__main__":
    sys.exit(main())
