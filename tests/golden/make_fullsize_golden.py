"""Writes the FP64 oracle's trajectory on a full-size synthetic workload (a stored expected value
for the GPU path at that size). Calls only the oracle and the seeded input generators.

    python tests/golden/make_fullsize_golden.py c4 [--R 20] [--iters 20] [--workers 8] [--K K]
                                                   [--order WHV]

Output: tests/golden/fullsize_<cfg>_R<R>[_K<K>][_WHV].json (FIT, objective, sparsity, rho, rank counts
per outer iteration) and .npz (final H, V in FP64). The run starts from the seeded initial point
(seed 0) with the workload's constraints: H free, W nonnegative, l1 (lambda 0.1) on V, 5 ADMM steps.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import copa_oracle as co  # noqa: E402
from oracle import fullsize  # noqa: E402
from paper_1803_04572_amd import synth  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cfg")
    ap.add_argument("--R", type=int, default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--K", type=int, default=None)
    ap.add_argument("--order", default="HWV", choices=["HWV", "WHV"])
    args = ap.parse_args()
    t0 = time.time()

    def progress(msg):
        print(f"[{time.time() - t0:8.1f}s] {msg}", flush=True)

    coh, cfg = synth.make_config(args.cfg, K=args.K)
    R = args.R or cfg["R"]
    iters = args.iters or cfg["outer"]
    l = cfg["l"]
    progress(f"{args.cfg}: K={coh.K} J={coh.J} S={coh.S} nnz={coh.nnz} R={R} l={l}")
    H0, W0, V0 = synth.init_factors(coh.K, coh.J, R, 0)
    opt = co.Options(R=R, outer_iters=iters, inner_iters=cfg["inner"], order=args.order)
    out = fullsize.copa_fit_sharded(coh, l, H0, W0, V0, opt, workers=args.workers,
                                    progress=progress)
    tag = (f"fullsize_{args.cfg}_R{R}" + (f"_K{coh.K}" if args.K else "")
           + ("_WHV" if args.order == "WHV" else ""))
    meta = dict(cfg=args.cfg, K=coh.K, J=coh.J, S=coh.S, nnz=coh.nnz, R=R, l=l, iters=iters,
                inner=cfg["inner"], order=opt.order, seed_init=0,
                prox=[opt.prox_H, opt.prox_W, opt.prox_V],
                lam=[opt.lam_H, opt.lam_W, opt.lam_V], rank_rtol=opt.rank_rtol,
                normX2=out["normX2"], fit=out["fit"], objective=out["objective"],
                sparsity=out["sparsity"], rho=out["rho"], rank_deficient=out["rank_deficient"],
                ambiguous_band=out["ambiguous_band"], wall_s=time.time() - t0,
                workers=args.workers, generator="tests/golden/make_fullsize_golden.py")
    with open(os.path.join(HERE, tag + ".json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    np.savez_compressed(os.path.join(HERE, tag + ".npz"), H=out["H"], V=out["V"])
    progress(f"wrote {tag}.json/.npz")


if __name__ == "__main__":
    main()
