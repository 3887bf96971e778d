"""The W -> H -> V block order at full size: 20 outer iterations of the 50,000-subject workload
(R = 10) and of the 250,000-subject workload (R = 15 and 40), through the launch path bench.py
times, against the oracle's trajectories in that order (written by
tests/golden/make_fullsize_golden.py --order WHV, which calls only the oracle)."""
import json
import os

import numpy as np
import pytest

from paper_1803_04572_amd import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
_COHORTS = {}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cohort(name):
    if name not in _COHORTS:
        _COHORTS.clear()  # one full-size cohort in host memory at a time
        _COHORTS[name] = synth.make_config(name)
    return _COHORTS[name]


@pytest.mark.parametrize("cfg_name,R", [("c2", 10), ("c3", 15), ("c3", 40)])
def test_full_size_whv_trajectory_matches_oracle(cfg_name, R):
    """FIT and objective histories within 1e-5 of the FP64 oracle's W -> H -> V trajectory, H and
    V congruent to its final factors, and the same sparsity of V within three entries."""
    import torch
    from paper_1803_04572_amd import copa
    from gpu_common import congruence
    coh, cfg = _cohort(cfg_name)
    tag = f"fullsize_{cfg_name}_R{R}_WHV"
    with open(os.path.join(GOLDEN, tag + ".json")) as fh:
        ref = json.load(fh)
    z = np.load(os.path.join(GOLDEN, tag + ".npz"))
    assert ref["order"] == "WHV"
    assert (ref["K"], ref["S"], ref["nnz"]) == (coh.K, coh.S, coh.nnz)
    print(f"case {tag}: K={coh.K} R={R}", flush=True)
    plan = copa.Plan.from_cohort(coh, R=R, l=cfg["l"], inner_iters=cfg["inner"], order="WHV")
    st = plan.new_state(*synth.init_factors(coh.K, coh.J, R, 0))
    rep, _ = plan.fit(st, ref["iters"], qtilde=False)
    torch.cuda.synchronize()
    fit = np.abs(np.array(rep["fit_history"]) - np.array(ref["fit"])) / np.abs(ref["fit"])
    obj = np.abs(np.array(rep["objective_history"]) - np.array(ref["objective"])) / \
        np.abs(ref["objective"])
    cH = congruence(st["H"].double().cpu().numpy(), z["H"])
    cV = congruence(st["V"].double().cpu().numpy(), z["V"])
    dz = abs(rep["sparsity_V"] - ref["sparsity"][-1]) * coh.J * R
    print(f"full-size {tag}: fit_rel={fit[-1]:.2e} hist_max={fit.max():.2e} "
          f"obj_max={obj.max():.2e} cong_H={cH:.9f} cong_V={cV:.9f} sparsity_entries_diff={dz:.0f}",
          flush=True)
    assert fit.max() <= 1e-5 and obj.max() <= 1e-5
    assert min(cH, cV) >= 0.999
    assert dz <= 3
    del plan, st
