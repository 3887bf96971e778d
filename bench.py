"""Benchmark: outer COPA (AO-ADMM) iterations per second on one MI355X.

One step = one outer iteration of Algorithm 1 over the whole cohort (Procrustes, the three
MTTKRPs, the three ADMM factor updates and the FIT), launched by copa_fit from libcopa.so.
Inputs are synthetic EHR-shaped tensors already resident in HBM when the timed region starts.

    python bench.py [--steps K] [--warmup W] [--workload c2]

Prints one JSON line. Per-kernel times come from HIP events recorded by the library on the
stream its kernels run on (copa_set_timing); `roofline` describes the kernel with the largest
share of the iteration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "outer AO-ADMM iters/sec + MTTKRP HBM GB/s at fixed fit vs FP64 oracle"
CSRC = os.path.join(ROOT, "paper_1803_04572_amd", "csrc")
# rocprofv3 kernel-name stem of each timed kernel
ROCPROF_NAME = {"pass1": "k_pass1", "procrustes": "k_procrustes", "gram_FH": "k_rows_gram_fit",
                "mode_H": "k_mode_H", "w_admm": "k_w_admm", "gram_WM": "k_rows_gram",
                "pass2": "k_pass2c", "v_admm": "k_v_admm"}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/hbm_traffic_<workload>.txt: FETCH_SIZE x2 + WRITE_SIZE x1, scales from a plain copy),
    or None when the summary is missing or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    m = re.search(r"^# source_hash=(\w+)", text, re.M)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"^kernel=%s\S* .*bytes_per_launch=(\d+)" % re.escape(ROCPROF_NAME[kernel]),
                  text, re.M)
    return int(m.group(1)) if m else None


def algorithmic_bytes(coh, R, l, compact):
    """Bytes each kernel of one outer iteration must move at least (inputs read once, outputs
    written once), for FP32 factors. Pass 1 streams the CSR nonzeros (4 B each in the lossless
    compact form: 16-bit feature id + bfloat16 value; else 8 B) with 4-B row offsets; pass 2 streams
    the feature-sorted (key, value) pairs (8 B) and one subject id per row; smoothed passes read the
    l basis coefficients of each row. rows = projected rows (K*l smoothed, S plain)."""
    K, J, S, nnz = coh.K, coh.J, coh.S, coh.nnz
    rows = K * l if l > 0 else S
    basis = S * l * 4 if l > 0 else 0
    x1 = nnz * (4 if compact else 8) + (S + 1) * 4 + (K + 1) * 4 + basis
    x2 = nnz * 8 + S * 4 + basis
    return {
        "pass1": x1 + J * R * 4 + rows * R * 4,
        "procrustes": rows * R * 4 * 2 + K * R * 4 + R * R * 4,
        "gram_FH": rows * R * 4 * 2 + K * R * 4,
        "mode_H": R * R * 8 * 3,
        "w_admm": rows * R * 4 * 3 + K * R * 4 * 5,
        "gram_WM": K * R * 4 + rows * R * 4,
        "pass2": x2 + rows * R * 4 + J * R * 4,
        "v_admm": J * R * 4 * 5,
    }


def cpu_baseline(cfg_name, R, l, K_full, n_subjects=10000, iters=10):
    """The FP64 oracle, as it is, on a bounded sample of the same workload: `iters` outer
    iterations on a cohort of `n_subjects` drawn with the same recipe, scaled by subject count."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import copa_oracle as co
    from paper_1803_04572_amd import synth
    coh, cfg = synth.make_config(cfg_name, K=n_subjects)
    import contextlib
    ctx = threadpool_limits(limits=1) if threadpool_limits else contextlib.nullcontext()
    with ctx:
        prob = co.build_problem(coh, l)
        H0, W0, V0 = synth.init_factors(coh.K, coh.J, R, 0)
        opt = co.Options(R=R, outer_iters=iters, inner_iters=cfg["inner"])
        t0 = time.perf_counter()
        co.copa_fit(prob, H0, W0, V0, opt)
        dt = time.perf_counter() - t0
    per_iter_full = dt / iters * (K_full / n_subjects)
    return {"value": 1.0 / per_iter_full, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} outer iterations on a {n_subjects}-subject cohort of the same "
                      f"recipe ({dt:.1f} s), scaled by K={K_full}/{n_subjects}; FP64 NumPy, "
                      f"one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not supported "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1803_04572_amd import copa, synth
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    copa.lib()  # fails loudly when libcopa.so is missing

    def progress(msg):
        print(f"bench.py: {msg}", file=sys.stderr, flush=True)

    progress(f"generating {args.workload}")
    coh, cfg = synth.make_config(args.workload)
    R, l = cfg["R"], cfg["l"]
    progress(f"K={coh.K} S={coh.S} nnz={coh.nnz}; creating the plan")
    plan = copa.Plan.from_cohort(coh, R=R, l=l, inner_iters=cfg["inner"])
    progress("plan ready")
    H0, W0, V0 = synth.init_factors(coh.K, coh.J, R, 0)
    state = plan.new_state(H0, W0, V0)
    torch.cuda.synchronize()

    plan.fit(state, args.warmup, qtilde=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep, _ = plan.fit(state, args.steps, qtilde=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps / dt

    # same number of steps again with HIP events around every kernel launch
    plan.set_timing(True)
    t1 = time.perf_counter()
    rep_t, _ = plan.fit(state, args.steps, qtilde=False)
    torch.cuda.synchronize()
    dt_t = time.perf_counter() - t1
    timing = plan.read_timing()
    plan.set_timing(False)

    compact = plan.query("compact")
    abytes = algorithmic_bytes(coh, R, l, compact)
    per_kernel = {k: {"avg_us": 1e3 * ms / n, "launches": n} for k, (ms, n) in timing.items()
                  if n > 0}
    for k, v in per_kernel.items():
        if k in abytes:
            v["alg_bytes"] = abytes[k]
            v["GBps"] = abytes[k] / (v["avg_us"] * 1e-6) / 1e9
    dom = max((k for k in per_kernel if k in abytes), key=lambda k: per_kernel[k]["avg_us"])
    ach = per_kernel[dom]["GBps"]
    traffic = measured_traffic(dom, args.workload)
    if args.copy_probe:
        n = 64 << 20
        a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.workload, R, l, coh.K)

    mttkrp = {k: {"GBps": round(per_kernel[k]["GBps"], 1),
                  "frac_hbm": round(per_kernel[k]["GBps"] / HBM_PEAK_GBS, 4)}
              for k in ("pass1", "pass2") if k in per_kernel}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['name']}", "K": coh.K, "J": coh.J,
                   "R": R, "l": l, "S": coh.S, "nnz": coh.nnz, "inner_iters": cfg["inner"],
                   "constraints": "H free, W nonneg, V l1 (lambda 0.1), cubic spline smoothing",
                   "nonzeros": "compact 4-byte (lossless)" if compact else "fp32 8-byte"},
        "fit": rep["fit"],
        "fit_after_timed_steps": rep_t["fit"],
        "mttkrp_hbm": mttkrp,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "alg_bytes_per_launch": abytes[dom],
                     "avg_launch_us": round(per_kernel[dom]["avg_us"], 2)},
        "kernels": {k: {kk: (round(vv, 2) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in per_kernel.items()},
        "ms_per_step_with_kernel_events": 1e3 * dt_t / args.steps,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
