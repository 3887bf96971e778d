"""Twenty outer iterations of the GPU path against the FP64 oracle's stored trajectory on the same
seeded inputs: the workloads with 250,000 subjects (R = 15 and R = 40) and 800,000 subjects (R =
20), cut to their first 3,000 subjects. The oracle's trajectories were written by
tests/golden/make_fullsize_golden.py (which calls only the oracle) with --K 3000."""
import json
import os

import numpy as np
import pytest

from paper_1803_04572_amd import synth
from gpu_common import CONGRUENCE_MIN, FIT_RTOL, congruence, run_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("cfg_name,R,K", [("c3", 15, 3000), ("c3", 40, 3000), ("c4", 20, 3000)])
def test_twenty_iteration_trajectory(cfg_name, R, K):
    tag = f"fullsize_{cfg_name}_R{R}_K{K}"
    with open(os.path.join(GOLDEN, tag + ".json")) as fh:
        ref = json.load(fh)
    z = np.load(os.path.join(GOLDEN, tag + ".npz"))
    coh, cfg = synth.make_config(cfg_name, K=K)
    assert (ref["K"], ref["J"], ref["S"], ref["nnz"], ref["l"]) == (coh.K, coh.J, coh.S, coh.nnz,
                                                                   cfg["l"])
    iters = ref["iters"]
    g = run_gpu(coh, R, cfg["l"], iters)
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
