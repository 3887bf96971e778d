"""The launch-shape autotuner: the first fit on a plan times the candidate shapes on its own data
(or reads them from the COPA_TUNE_CACHE file) and the fit stays on the oracle's trajectory."""
import json
import os

import numpy as np
import pytest

from paper_1803_04572_amd import synth
from gpu_common import run_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SHAPES = ("pass1_blocks_per_cu", "procrustes_variant", "gram_blocks", "pass2_blocks")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_tuned_shapes_cached_and_on_trajectory(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("COPA_TUNE_CACHE", str(cache))
    with open(os.path.join(GOLDEN, "fullsize_c4_R20_K3000.json")) as fh:
        ref = json.load(fh)
    coh, cfg = synth.make_config("c4", K=3000)
    a = run_gpu(coh, 20, cfg["l"], ref["iters"], adjoint=False)
    assert a["plan"].query("tuned") == 1
    shapes = {k: a["plan"].query(k) for k in SHAPES}
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and ":" in lines[0]
    b = run_gpu(coh, 20, cfg["l"], ref["iters"], adjoint=False)
    assert b["plan"].query("tuned") == 2
    assert {k: b["plan"].query(k) for k in SHAPES} == shapes
    for g in (a, b):
        fit = abs(g["rep"]["fit"] - ref["fit"][-1]) / ref["fit"][-1]
        assert fit <= 1e-5
    print("tuned shapes", shapes, flush=True)


def test_untuned_plan_keeps_default_shapes():
    from paper_1803_04572_amd import copa
    coh, cfg = synth.make_config("c4", K=500)
    g = run_gpu(coh, 20, cfg["l"], 2, adjoint=False, autotune=False)
    p = g["plan"]
    assert p.query("tuned") == 0
    assert p.query("pass1_blocks_per_cu") == 4 and p.query("procrustes_variant") == 2
    d = run_gpu(coh, 20, cfg["l"], 2, adjoint=False, deterministic=True)
    assert d["plan"].query("tuned") == 0  # fixed summation order: fixed shapes


@pytest.mark.parametrize("cfg_name,R", [("c4", 20), ("c3", 40)])
def test_every_procrustes_variant_on_trajectory(cfg_name, R, tmp_path, monkeypatch):
    """Each of the three Procrustes kernels for smoothed R > 16, forced through the cache file,
    follows the oracle's 20-iteration trajectory."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("COPA_TUNE_CACHE", str(cache))
    with open(os.path.join(GOLDEN, f"fullsize_{cfg_name}_R{R}_K3000.json")) as fh:
        ref = json.load(fh)
    coh, cfg = synth.make_config(cfg_name, K=3000)
    first = run_gpu(coh, R, cfg["l"], 1, adjoint=False)
    key, shapes = cache.read_text().strip().splitlines()[0].split(":")
    a, _, c, d = shapes.split()
    for v in (0, 1, 2):
        cache.write_text(f"{key}: {a} {v} {c} {d}\n")
        g = run_gpu(coh, R, cfg["l"], ref["iters"], adjoint=False)
        assert g["plan"].query("tuned") == 2 and g["plan"].query("procrustes_variant") == v
        fit = np.abs(np.array(g["rep"]["fit_history"]) - np.array(ref["fit"])) / np.abs(ref["fit"])
        print(f"procrustes variant {v} {cfg_name} R={R}: fit_rel={fit[-1]:.2e} "
              f"hist_max={fit.max():.2e} rank_def={g['rep']['rank_deficient']}/"
              f"{ref['rank_deficient'][-1]}", flush=True)
        assert fit.max() <= 1e-5
        assert abs(g["rep"]["rank_deficient"] - ref["rank_deficient"][-1]) <= \
            ref["ambiguous_band"][-1]
    del first
