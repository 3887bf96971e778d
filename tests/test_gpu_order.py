"""The block order W -> H -> V (copa_options.order = COPA_ORDER_WHV) on the GPU against the FP64
oracle run in the same order: FIT and objective histories, factors, sparsity, Procrustes ranks,
the last MTTKRPs, and the twenty-iteration trajectories of the full-size workloads cut to their
first 3,000 subjects (written by tests/golden/make_fullsize_golden.py --order WHV, which calls
only the oracle). Also: fixed-order mode is bitwise reproducible and resumable in this order."""
import json
import os

import numpy as np
import pytest

from oracle import copa_oracle as co
from paper_1803_04572_amd import synth
from gpu_common import (CONGRUENCE_MIN, FIT_RTOL, check_fit, congruence, run_gpu, run_oracle)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("cfg_name,K,R,l,iters", [
    ("c2", 500, 10, 7, 8),     # smoothed, the pair path
    ("c5", 300, 5, 0, 8),      # no smoothing: Procrustes on the visit rows
    ("c4", 400, 20, 7, 6),     # smoothed, R > 16
    ("c3", 200, 40, 7, 5),     # smoothed, R = 40 (one subject per wavefront)
    ("c1", 150, 8, 5, 6),      # smoothed, dense visit rows (row passes)
])
def test_whv_matches_oracle(cfg_name, K, R, l, iters):
    coh, _ = synth.make_config(cfg_name, K=K)
    g = run_gpu(coh, R, l, iters, order="WHV")
    o, prob = run_oracle(coh, R, l, iters, order="WHV")
    check_fit(f"whv {cfg_name} K={K} R={R} l={l}", coh, g, o, prob, R)
    # the last MTTKRPs of the W -> H -> V order: F_W with the previous H, F_H with the new W
    import torch
    F_H, F_W, _ = g["plan"].mttkrp_last()
    torch.cuda.synchronize()
    for name, got in (("H", F_H), ("W", F_W)):
        ref = o.F[name]
        err = np.abs(got.double().cpu().numpy() - ref).max() / max(np.abs(ref).max(), 1e-30)
        print(f"  F_{name} rel max err {err:.2e}", flush=True)
        assert err <= 1e-3


def test_orders_differ_on_the_gpu_as_in_the_oracle():
    """The GPU's two orders give the oracle's two different trajectories, each matching its own."""
    coh, _ = synth.make_config("c2", K=400)
    R, l, iters = 10, 7, 6
    gh = run_gpu(coh, R, l, iters, order="HWV")
    gw = run_gpu(coh, R, l, iters, order="WHV")
    oh, _ = run_oracle(coh, R, l, iters, order="HWV")
    ow, _ = run_oracle(coh, R, l, iters, order="WHV")
    fh, fw = np.array(gh["rep"]["fit_history"]), np.array(gw["rep"]["fit_history"])
    gap = np.abs(np.array(oh.fit) - np.array(ow.fit)) / np.abs(oh.fit)
    print(f"orders: oracle gap max {gap.max():.2e}; gpu HWV err "
          f"{(np.abs(fh - oh.fit) / np.abs(oh.fit)).max():.2e}, WHV err "
          f"{(np.abs(fw - ow.fit) / np.abs(ow.fit)).max():.2e}", flush=True)
    assert gap.max() > 100 * FIT_RTOL
    assert (np.abs(fh - oh.fit) / np.abs(oh.fit)).max() <= FIT_RTOL
    assert (np.abs(fw - ow.fit) / np.abs(ow.fit)).max() <= FIT_RTOL


@pytest.mark.parametrize("cfg_name,R,K", [("c3", 15, 3000), ("c3", 40, 3000), ("c4", 20, 3000)])
def test_whv_twenty_iteration_trajectory(cfg_name, R, K):
    tag = f"fullsize_{cfg_name}_R{R}_K{K}_WHV"
    with open(os.path.join(GOLDEN, tag + ".json")) as fh:
        ref = json.load(fh)
    z = np.load(os.path.join(GOLDEN, tag + ".npz"))
    coh, cfg = synth.make_config(cfg_name, K=K)
    assert ref["order"] == "WHV"
    assert (ref["K"], ref["J"], ref["S"], ref["nnz"], ref["l"]) == (coh.K, coh.J, coh.S, coh.nnz,
                                                                   cfg["l"])
    g = run_gpu(coh, R, cfg["l"], ref["iters"], order="WHV")
    rep = g["rep"]
    fit = np.abs(np.array(rep["fit_history"]) - np.array(ref["fit"])) / np.abs(ref["fit"])
    obj = np.abs(np.array(rep["objective_history"]) - np.array(ref["objective"])) / \
        np.abs(ref["objective"])
    cong = dict(H=congruence(g["H"], z["H"]), V=congruence(g["V"], z["V"]))
    dz = abs(rep["sparsity_V"] - ref["sparsity"][-1]) * coh.J * R
    print(f"trajectory {tag}: fit_gpu={rep['fit']:.9f} fit_oracle={ref['fit'][-1]:.9f} "
          f"fit_rel={fit[-1]:.2e} hist_max={fit.max():.2e} obj_max={obj.max():.2e} "
          f"rank_def={rep['rank_deficient']}/{ref['rank_deficient'][-1]} "
          f"band={ref['ambiguous_band'][-1]} sparsity_entries_diff={dz:.0f} "
          + " ".join(f"cong_{k}={v:.9f}" for k, v in cong.items()), flush=True)
    assert fit[-1] <= FIT_RTOL and fit.max() <= FIT_RTOL
    assert obj.max() <= FIT_RTOL
    assert min(cong.values()) >= CONGRUENCE_MIN
    assert abs(rep["rank_deficient"] - ref["rank_deficient"][-1]) <= ref["ambiguous_band"][-1]
    assert dz <= 3


def _fit(plan, init, iters):
    import torch
    st = plan.new_state(*init)
    rep, Qt = plan.fit(st, iters)
    torch.cuda.synchronize()
    return rep, {k: v.cpu().numpy() for k, v in st.items() if k != "iter"}, Qt.cpu().numpy()


@pytest.mark.parametrize("l", [7, 0])
def test_whv_fixed_order_reproducible_and_resumable(l):
    """Fixed-order mode in the W -> H -> V order: two plans give bitwise equal fits, and 4 + 4
    iterations in two calls equal 8 in one call."""
    import torch
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c2", K=600)
    R = 10
    init = synth.init_factors(coh.K, coh.J, R, 0)
    a = copa.Plan.from_cohort(coh, R=R, l=l, deterministic=True, order="WHV")
    b = copa.Plan.from_cohort(coh, R=R, l=l, deterministic=True, order="WHV")
    ra, sa, qa = _fit(a, init, 8)
    rb, sb, qb = _fit(b, init, 8)
    assert ra["fit_history"] == rb["fit_history"]
    assert all(np.array_equal(sa[k], sb[k]) for k in sa) and np.array_equal(qa, qb)
    st = a.new_state(*init)
    r1, _ = a.fit(st, 4)
    r2, Qt = a.fit(st, 4)
    torch.cuda.synchronize()
    sc = {k: v.cpu().numpy() for k, v in st.items() if k != "iter"}
    assert r1["fit_history"] + r2["fit_history"] == ra["fit_history"]
    assert all(np.array_equal(sa[k], sc[k]) for k in sa) and np.array_equal(qa, Qt.cpu().numpy())


def test_whv_constraint_variants():
    """Other proximal operators in the W -> H -> V order (nonnegative H and l1 on W)."""
    coh, _ = synth.make_config("c2", K=300)
    R, l, iters = 8, 7, 6
    prox = (co.PROX_NONNEG, co.PROX_NONNEG_L1, co.PROX_L1)
    lam = (0.0, 0.05, 0.1)
    H0, W0, V0 = synth.init_factors(coh.K, coh.J, R, 0)
    init = (np.abs(H0), W0, V0)
    g = run_gpu(coh, R, l, iters, prox=prox, lam=lam, init=init, order="WHV")
    o, prob = run_oracle(coh, R, l, iters, prox=prox, lam=lam, init=init, order="WHV")
    check_fit("whv constraints", coh, g, o, prob, R)


@pytest.mark.parametrize("cfg_name,R", [("c4", 20), ("c3", 40)])
def test_whv_every_procrustes_variant_on_trajectory(cfg_name, R, tmp_path, monkeypatch):
    """Each Procrustes kernel for smoothed R > 16, forced through the tuning cache file, in the
    W -> H -> V order, follows the oracle's 20-iteration trajectory in this order."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("COPA_TUNE_CACHE", str(cache))
    with open(os.path.join(GOLDEN, f"fullsize_{cfg_name}_R{R}_K3000_WHV.json")) as fh:
        ref = json.load(fh)
    coh, cfg = synth.make_config(cfg_name, K=3000)
    first = run_gpu(coh, R, cfg["l"], 1, adjoint=False, order="WHV")
    key, shapes = cache.read_text().strip().splitlines()[0].split(":")
    a, _, c, d = shapes.split()
    for v in (0, 1, 2):
        cache.write_text(f"{key}: {a} {v} {c} {d}\n")
        g = run_gpu(coh, R, cfg["l"], ref["iters"], adjoint=False, order="WHV")
        assert g["plan"].query("tuned") == 2 and g["plan"].query("procrustes_variant") == v
        fit = np.abs(np.array(g["rep"]["fit_history"]) - np.array(ref["fit"])) / np.abs(ref["fit"])
        print(f"whv procrustes variant {v} {cfg_name} R={R}: fit_rel={fit[-1]:.2e} "
              f"hist_max={fit.max():.2e} rank_def={g['rep']['rank_deficient']}/"
              f"{ref['rank_deficient'][-1]}", flush=True)
        assert fit.max() <= FIT_RTOL
        assert abs(g["rep"]["rank_deficient"] - ref["rank_deficient"][-1]) <= \
            ref["ambiguous_band"][-1]
    del first
