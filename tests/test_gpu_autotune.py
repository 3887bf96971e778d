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
    assert p.query("pass1_blocks_per_cu") == 4 and p.query("procrustes_variant") == 0
    d = run_gpu(coh, 20, cfg["l"], 2, adjoint=False, deterministic=True)
    assert d["plan"].query("tuned") == 0  # fixed summation order: fixed shapes
