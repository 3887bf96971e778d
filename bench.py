"""Benchmark: outer COPA (AO-ADMM) iterations per second on one MI355X.

One step = one outer iteration of Algorithm 1 over the whole cohort (Procrustes, the three
MTTKRPs, the three ADMM factor updates and the FIT), launched by copa_fit from libcopa.so.
Inputs are synthetic EHR-shaped tensors already resident in HBM when the timed region starts.

    python bench.py [--steps K] [--warmup W] [--workload c4] [--R R] [--order WHV|HWV]

The default workload is the largest configuration that fits one GPU (800,000 subjects, 80M
nonzeros, R = 20). The reported fit runs the blocks in the order W -> H -> V (the library's
option; Algorithm 1's order H -> W -> V is timed too and reported under `other_order`). The timed
fit starts from the seeded initial point; its FIT history is checked against the FP64 oracle's
trajectory in the same block order on the same inputs (tests/golden/fullsize_<workload>_R<R>
[_WHV].json, written by the oracle's sharded driver), and `value` is withheld (null) when the
final FIT differs by more than 1e-5 relative or a factor's congruence is below 0.999.

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
ROCPROF_NAME = {"pass1": ("k_pass1", "k_pass1p"), "procrustes": "k_procrustes",
                "proc_gram": "k_proc_gram", "proc_eigen": "k_proc_eigen", "proc_q": "k_proc_q",
                "gram_FH": "k_rows_gram_fit",
                "mode_H": "k_mode_H", "w_admm": "k_w_admm", "gram_WM": "k_rows_gram<",
                "pass2": ("k_pass2", "k_pass2c", "k_pass2p"), "v_admm": "k_v_admm", "w_first": "k_w_first",
                "m_rows": "k_m_rows", "finish": "k_finish_whv"}


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
    stems = ROCPROF_NAME[kernel]
    stems = (stems,) if isinstance(stems, str) else stems
    found = []  # (dispatches, bytes per launch) of every kernel of the step
    for line in text.splitlines():
        mm = re.match(r"^kernel=(\S+) .*dispatches=(\d+) .*bytes_per_launch=(\d+)", line)
        # (a stem ending in "<" names one template exactly; otherwise its variants count too)
        if mm and any(re.match(re.escape(st) + ("" if st.endswith("<") else r"([<_]|$)"),
                               mm.group(1)) for st in stems):
            found.append((int(mm.group(2)), int(mm.group(3))))
    if not found:
        return None
    # the kernels the timed iterations ran are those with the most dispatches (the tuner runs
    # the other candidates a few times)
    top = max(d for d, _ in found)
    return sum(b for d, b in found if d == top)


def algorithmic_bytes(coh, R, l, compact):
    """Bytes each kernel of one outer iteration must move at least (inputs read once, outputs
    written once), for FP32 factors:
      * X per pass: 4 B per nonzero in pass 1 when the nonzeros are stored in the lossless compact
        form (16-bit feature id + bfloat16 value), else 8 B; 8 B per nonzero in pass 2 (feature-
        sorted key and value); 4 B per visit row (row offset, resp. the row's subject);
      * smoothing per pass: the basis evaluated from each row's visit day (4 B per row) and a
        per-subject l x l transform (4 l^2 B per subject); the library streams stored FP32 basis
        rows instead, which moves more than this;
      * the per-subject row spaces T, Q, M (rows = K l smoothed, S plain; R floats per row),
        W and V, read and written as each kernel needs them;
      * the three-launch Procrustes step: its launches' own inputs and outputs (the FP64 l x l
        Gram and B_k, l (l + 1) / 2 doubles per subject each), not the warm start."""
    K, J, S, nnz = coh.K, coh.J, coh.S, coh.nnz
    rows = K * l if l > 0 else S
    nt = l * (l + 1) // 2  # FP64 entries of a subject's l x l Gram (three-launch Procrustes)
    basis = (S * 4 + K * l * l * 4) if l > 0 else 0
    x1 = nnz * (4 if compact else 8) + (S + 1) * 4 + (K + 1) * 4 + basis
    x2 = nnz * 8 + S * 4 + basis
    return {
        "pass1": x1 + J * R * 4 + rows * R * 4,
        "procrustes": rows * R * 4 * 2 + K * R * 4 + R * R * 4,
        # the three launches of the Procrustes step for smoothed R > 16: T and W in, the FP64 Gram
        # out; the Gram in, B_k out; T, W and B_k in, Q out
        "proc_gram": rows * R * 4 + K * R * 4 + K * nt * 8,
        "proc_eigen": K * nt * 8 * 2,
        "proc_q": rows * R * 4 * 2 + K * R * 4 + K * nt * 8,
        "gram_FH": rows * R * 4 * 2 + K * R * 4,
        "mode_H": R * R * 8 * 3,
        "w_admm": rows * R * 4 * 3 + K * R * 4 * 5,
        "gram_WM": K * R * 4 + rows * R * 4,
        "pass2": x2 + rows * R * 4 + J * R * 4,
        "v_admm": J * R * 4 * 5,
        # block order W -> H -> V
        "w_first": rows * R * 4 * 2 + K * R * 4 * 5,
        "m_rows": rows * R * 4 * 2 + K * R * 4,
        "finish": R * R * 8 * 4,
    }


def cpu_baseline(cfg_name, R, l, K_full, n_subjects, iters=3, order="HWV"):
    """The FP64 oracle, as it is, on a bounded sample of the same workload: `iters` outer
    iterations on a cohort of `n_subjects` drawn with the same recipe, its subjects split over the
    host's cores (the oracle's sharded driver, one BLAS thread per worker), scaled by subject
    count. Only the iterations are timed (not the per-subject setup)."""
    from oracle import copa_oracle as co
    from oracle import fullsize
    from paper_1803_04572_amd import synth
    workers = max(1, min(16, os.cpu_count() or 1))
    coh, cfg = synth.make_config(cfg_name, K=min(n_subjects, K_full))
    H0, W0, V0 = synth.init_factors(coh.K, coh.J, R, 0)
    opt = co.Options(R=R, outer_iters=iters, inner_iters=cfg["inner"], order=order)
    marks = []
    fullsize.copa_fit_sharded(coh, l, H0, W0, V0, opt, workers=workers,
                              progress=lambda msg: marks.append(time.perf_counter()))
    dt = marks[-1] - marks[0]  # from "shards ready" to the last iteration
    per_iter_full = dt / iters * (K_full / coh.K)
    return {"value": 1.0 / per_iter_full, "unit": "iters/s", "cores": workers, "kind": "oracle",
            "sample": f"{iters} outer iterations on a {coh.K}-subject cohort of the same recipe "
                      f"({dt:.1f} s), scaled by K={K_full}/{coh.K}; FP64 NumPy/SciPy, subjects "
                      f"split over {workers} worker processes with one BLAS thread each"}


def load_or_make(workload, cache, progress):
    """The workload's cohort, generated (or read back from `cache` when an earlier run saved it
    there: the same seeded arrays)."""
    from paper_1803_04572_amd import synth
    path = os.path.join(cache, f"cohort_{workload}.npz") if cache else None
    cfg = dict(synth.CONFIGS[workload])
    if path and os.path.exists(path):
        progress(f"reading {path}")
        z = np.load(path)
        coh = synth.Cohort(K=int(z["K"]), J=int(z["J"]), subj_ptr=z["subj_ptr"],
                           row_ptr=z["row_ptr"], col=z["col"], val=z["val"], days=z["days"])
        return coh, cfg
    progress(f"generating {workload}")
    coh, cfg = synth.make_config(workload)
    if path:
        os.makedirs(cache, exist_ok=True)
        np.savez(path, K=coh.K, J=coh.J, subj_ptr=coh.subj_ptr, row_ptr=coh.row_ptr, col=coh.col,
                 val=coh.val, days=coh.days)
    return coh, cfg


def golden_check(workload, R, coh, fit_history, H, V, tol, order="HWV"):
    """Compares a fit started from the seeded initial point with the FP64 oracle's trajectory on
    the same inputs and in the same block order, stored by tests/golden/make_fullsize_golden.py.
    None when no trajectory is stored for this workload."""
    stem = f"fullsize_{workload}_R{R}" + ("_WHV" if order == "WHV" else "")
    path = os.path.join(ROOT, "tests", "golden", stem + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        g = json.load(fh)
    if (g["K"], g["J"], g["S"], g["nnz"]) != (coh.K, coh.J, coh.S, coh.nnz):
        return None
    n = min(len(fit_history), len(g["fit"]))
    ref = np.array(g["fit"][:n])
    got = np.array(fit_history[:n])
    rel = np.abs(got - ref) / np.abs(ref)
    out = {"iters_compared": n, "fit_gpu": float(got[-1]), "fit_oracle": float(ref[-1]),
           "fit_rel": float(rel[-1]), "fit_rel_max_history": float(rel.max()), "tol": tol,
           "passed": bool(rel[-1] <= tol), "oracle_file": os.path.relpath(path, ROOT)}
    if n == len(g["fit"]) and H is not None:
        z = np.load(os.path.join(ROOT, "tests", "golden", stem + ".npz"))

        def cong(A, B):
            num = np.abs(np.sum(A * B, axis=0))
            den = np.linalg.norm(A, axis=0) * np.linalg.norm(B, axis=0)
            c = np.where(den > 0, num / np.where(den > 0, den, 1.0),
                         np.where((np.linalg.norm(A, axis=0) == 0) & (np.linalg.norm(B, axis=0) == 0), 1.0, 0.0))
            return float(c.min())
        out["congruence_H"] = cong(H, z["H"])
        out["congruence_V"] = cong(V, z["V"])
        out["passed"] = out["passed"] and min(out["congruence_H"], out["congruence_V"]) >= 0.999
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--R", type=int, default=None, help="rank (default: the workload's)")
    ap.add_argument("--precision", choices=("fp32", "mixed"), default="fp32",
                    help="mixed: bfloat16 records of the projected data, FP32 accumulation, one "
                         "FP32 refinement iteration per fit call")
    ap.add_argument("--order", choices=("HWV", "WHV"), default="WHV",
                    help="block order of the reported fit: W -> H -> V (default) or Algorithm "
                         "1's H -> W -> V (same fixed points, different iterates)")
    ap.add_argument("--both-orders", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the other block order (reported under other_order)")
    ap.add_argument("--deterministic", action="store_true",
                    help="fixed-order mode: every reduction in a fixed order, bitwise "
                         "reproducible runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (HBM counter scaling)")
    ap.add_argument("--cache", default=None,
                    help="directory for the generated cohort (reused by later runs)")
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

    coh, cfg = load_or_make(args.workload, args.cache, progress)
    R, l = args.R or cfg["R"], cfg["l"]
    progress(f"K={coh.K} S={coh.S} nnz={coh.nnz} R={R}; creating the plan")
    mixed = args.precision == "mixed"
    H0, W0, V0 = synth.init_factors(coh.K, coh.J, R, 0)
    gold_iters = cfg["outer"]

    def measure(order, events):
        """Plan in block order `order`, untimed warm-up, `steps` timed outer iterations from the
        seeded start, the gate against the oracle's trajectory in that order, and (events) the
        same steps again with HIP events around every kernel launch."""
        plan = copa.Plan.from_cohort(coh, R=R, l=l, inner_iters=cfg["inner"],
                                     precision=copa.PREC_MIXED if mixed else copa.PREC_FP32,
                                     mixed_refine=1, order=order,
                                     deterministic=args.deterministic)
        progress(f"plan ready (order {order})")
        init = plan.new_state(H0, W0, V0)
        state = plan.new_state(H0, W0, V0)
        torch.cuda.synchronize()
        # warm-up (captures the iteration graph for these state buffers), then back to the start
        plan.fit(state, args.warmup, qtilde=False)
        for k in ("H", "W", "V", "D_H", "D_W", "D_V"):
            state[k].copy_(init[k])
        torch.cuda.synchronize()
        progress(f"timed run (order {order})")
        t0 = time.perf_counter()
        rep, _ = plan.fit(state, args.steps, qtilde=False, fresh=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # validity gate: the timed fit against the FP64 oracle's trajectory from the same start
        if args.steps >= gold_iters:
            hist = rep["fit_history"]
            Hf = Vf = None
            if args.steps == gold_iters:
                Hf = state["H"].double().cpu().numpy()
                Vf = state["V"].double().cpu().numpy()
        else:  # an untimed fit of the full length from the same start
            chk = plan.new_state(H0, W0, V0)
            rc, _ = plan.fit(chk, gold_iters, qtilde=False, fresh=True)
            hist = rc["fit_history"]
            Hf, Vf = chk["H"].double().cpu().numpy(), chk["V"].double().cpu().numpy()
            del chk
        gate = golden_check(args.workload, R, coh, hist, Hf, Vf, tol=1e-4 if mixed else 1e-5,
                            order=order)
        progress(f"gate (order {order}): {gate}")
        res = dict(plan=plan, rep=rep, dt=dt, gate=gate, state=state, init=init)
        if events:
            plan.set_timing(True)
            t1 = time.perf_counter()
            plan.fit(state, args.steps, qtilde=False)
            torch.cuda.synchronize()
            res["dt_t"] = time.perf_counter() - t1
            res["timing"] = plan.read_timing()
            plan.set_timing(False)
        return res

    other = None
    if args.both_orders:
        o2 = "HWV" if args.order == "WHV" else "WHV"
        m2 = measure(o2, events=False)
        g2 = m2["gate"] or {}
        other = {"block_order": o2, "value": args.steps / m2["dt"] if g2.get("passed") else None,
                 "value_if_ungated": args.steps / m2["dt"],
                 "ms_per_step": 1e3 * m2["dt"] / args.steps, "fit": m2["rep"]["fit"],
                 "gate_passed": g2.get("passed"), "gate_fit_rel": g2.get("fit_rel")}
        del m2
        torch.cuda.empty_cache()
    m = measure(args.order, events=True)
    plan, rep, dt, gate, state, init = (m[k] for k in ("plan", "rep", "dt", "gate", "state", "init"))
    dt_t, timing = m["dt_t"], m["timing"]
    value = args.steps / dt

    compact = plan.query("compact")
    npairs = plan.query("pairs")
    shapes = {k: plan.query(k) for k in ("tuned", "pass1_blocks_per_cu", "procrustes_variant",
                                         "gram_blocks", "pass2_blocks")}
    if args.order == "WHV":
        shapes.update({k: plan.query(k) for k in ("wfirst_blocks", "mrows_blocks")})
    abytes = algorithmic_bytes(coh, R, l, compact)
    per_kernel = {k: {"avg_us": 1e3 * ms / n, "launches": n} for k, (ms, n) in timing.items()
                  if n > 0}
    for k, v in per_kernel.items():
        if k in abytes:
            v["alg_bytes"] = abytes[k]
            v["GBps"] = abytes[k] / (v["avg_us"] * 1e-6) / 1e9
    dom = max((k for k in per_kernel if k in abytes), key=lambda k: per_kernel[k]["avg_us"])
    ach = per_kernel[dom]["GBps"]
    traffic = measured_traffic(dom, args.workload + ("" if args.R is None else f"_R{R}")
                               + ("_mixed" if mixed else "") + ("_WHV" if args.order == "WHV" else ""))
    if args.copy_probe:
        # a plain elementwise kernel of known size for the HBM counters' scale: reads and writes
        # 256 MiB once per launch
        n = 64 << 20
        a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
    del plan, state, init
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        progress("cpu baseline")
        cpu = cpu_baseline(args.workload, R, l, coh.K, n_subjects=200_000, iters=5, order=args.order)

    mttkrp = {k: {"GBps": round(per_kernel[k]["GBps"], 1),
                  "frac_hbm": round(per_kernel[k]["GBps"] / HBM_PEAK_GBS, 4)}
              for k in ("pass1", "pass2") if k in per_kernel}
    passed = gate is not None and gate["passed"]
    out = {
        "metric": METRIC,
        "value": value if passed else None,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-in/f32-acc" if mixed else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['name'].replace(' R=' + str(cfg['R']), '')} R={R}",
                   "K": coh.K, "J": coh.J, "R": R, "l": l, "S": coh.S, "nnz": coh.nnz,
                   "outer_iters": gold_iters, "inner_iters": cfg["inner"],
                   "constraints": "H free, W nonneg, V l1 (lambda 0.1), cubic spline smoothing",
                   "nonzeros": "compact 4-byte (lossless)" if compact else "fp32 8-byte",
                   "streamed": (f"projected pairs C_k^T X_k ({npairs} records, "
                                + ("16-byte bfloat16" if mixed else "32-byte FP32") + ")")
                   if npairs else "nonzeros and basis rows",
                   "precision": args.precision, "block_order": args.order,
                   "deterministic": args.deterministic},
        "gate": gate,
        "launch_shapes": shapes,
        "value_if_ungated": value,
        "fit": rep["fit"],
        "mttkrp_hbm": mttkrp,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "alg_bytes_per_launch": abytes[dom],
                     "avg_launch_us": round(per_kernel[dom]["avg_us"], 2)},
        "kernels": {k: {kk: (round(vv, 2) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in per_kernel.items()},
        "ms_per_step_with_kernel_events": 1e3 * dt_t / args.steps,
        "cpu_baseline": cpu,
        "other_order": other,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
