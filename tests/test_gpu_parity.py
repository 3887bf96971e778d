"""GPU path (libcopa.so through the C ABI) against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

from oracle import copa_oracle as co
from paper_1803_04572_amd import synth
from gpu_common import (CONGRUENCE_MIN, FIT_RTOL, congruence, procrustes_condition, run_gpu,
                        run_oracle, split_rows, stacked_U)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _report(tag, **kv):
    print(tag, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                        for k, v in kv.items()), flush=True)


def test_smoothing_basis_matches_oracle():
    coh, cfg = synth.make_config("c1")
    from paper_1803_04572_amd import copa
    plan = copa.Plan.from_cohort(coh, R=5, l=7)
    C, rk = plan.basis()
    C, rk = C.double().cpu().numpy(), rk.cpu().numpy()
    worst = 0.0
    for k in range(coh.K):
        r0, r1 = coh.subj_ptr[k], coh.subj_ptr[k + 1]
        Co = co.smoothing_basis(coh.days[r0:r1], 7)
        assert rk[k] == Co.shape[1], f"subject {k}: rank {rk[k]} vs {Co.shape[1]}"
        Cg = C[r0:r1, :rk[k]]
        worst = max(worst, np.abs(Cg @ Cg.T - Co @ Co.T).max())
        assert np.abs(C[r0:r1, rk[k]:]).max(initial=0.0) == 0.0
    _report("basis", worst_projector_diff=worst)
    assert worst < 1e-5


@pytest.mark.parametrize("cfg_name,K,R,l", [("c1", None, 5, 7), ("c2", 400, 10, 7),
                                            ("c5", 300, 5, 0), ("c5", 200, 10, 0),
                                            ("c3", 300, 40, 7)])
def test_one_iteration_step_parity(cfg_name, K, R, l):
    """After one outer iteration: Q_k (via Qtilde), each MTTKRP and each updated factor."""
    coh, cfg = synth.make_config(cfg_name, K=K)
    g = run_gpu(coh, R, l, 1)
    o, prob = run_oracle(coh, R, l, 1)
    FH, FW, FV = (t.double().cpu().numpy() for t in g["plan"].mttkrp_last())
    # Q_k: a relative FP32 perturbation of A_k moves the polar factor by up to ~ eps * kappa_k
    H0, W0, V0 = synth.init_factors(coh.K, coh.J, R, 0)
    kappa = procrustes_condition(coh, R, l, H0, W0, V0)
    Qg = split_rows(coh, g["Qt"])
    qerr = max((np.abs(a - b).max(initial=0.0) / (1e-5 + 1e-6 * kap)
                for a, b, kap in zip(Qg, o.Qtilde, kappa)), default=0.0)
    errs = dict(
        Qt_scaled=qerr * 2e-4,
        FH=np.abs(FH - o.F["H"]).max() / np.abs(o.F["H"]).max(),
        FW=np.abs(FW - o.F["W"]).max() / np.abs(o.F["W"]).max(),
        FV=np.abs(FV - o.F["V"]).max() / np.abs(o.F["V"]).max(),
        H=np.abs(g["H"] - o.H).max() / np.abs(o.H).max(),
        W=np.abs(g["W"] - o.W).max() / np.abs(o.W).max(),
        V=np.abs(g["V"] - o.V).max() / np.abs(o.V).max(),
        fit=abs(g["rep"]["fit"] - o.fit[-1]) / abs(o.fit[-1]))
    _report(f"step {cfg_name}", **errs)
    for k, v in errs.items():
        assert v < 2e-4, (k, v)


@pytest.mark.parametrize("cfg_name,K,R,l,iters", [("c1", None, 5, 7, 10), ("c2", 1000, 10, 7, 20),
                                                  ("c5", 300, 5, 0, 10), ("c5", 300, 10, 0, 10),
                                                  ("c3", 600, 15, 7, 5), ("c4", 400, 20, 7, 5)])
def test_fit_parity(cfg_name, K, R, l, iters):
    coh, cfg = synth.make_config(cfg_name, K=K)
    g = run_gpu(coh, R, l, iters)
    o, prob = run_oracle(coh, R, l, iters)
    fit_rel = abs(g["rep"]["fit"] - o.fit[-1]) / abs(o.fit[-1])
    hist = np.abs(np.array(g["rep"]["fit_history"]) - np.array(o.fit)) / np.abs(o.fit)
    cong = dict(H=congruence(g["H"], o.H), V=congruence(g["V"], o.V), W=congruence(g["W"], o.W),
                U=congruence(stacked_U(split_rows(coh, g["Qt"]), g["H"]),
                             stacked_U(o.Qtilde, o.H)))
    _report(f"fit {cfg_name}", fit_gpu=g["rep"]["fit"], fit_oracle=o.fit[-1], fit_rel=fit_rel,
            hist_rel_max=float(hist.max()), spars_gpu=g["rep"]["sparsity_V"],
            spars_oracle=o.sparsity[-1], rank_def=g["rep"]["rank_deficient"],
            **{f"cong_{k}": v for k, v in cong.items()})
    assert fit_rel <= FIT_RTOL
    assert min(cong.values()) >= CONGRUENCE_MIN


@pytest.mark.parametrize("J,chunked", [(8000, True), (9800, False)])
@pytest.mark.parametrize("l", [7, 0])
def test_wide_feature_space_parity(J, chunked, l):
    """Thousands of features at R = 10: the V tile no longer fits one workgroup's LDS, so both
    passes run three column tiles of 4, 4 and 2 columns; at J = 9800 the pass-2 F_V tile plus one
    chunk of u rows does not fit either and pass 2 takes its unchunked form. All fit the oracle."""
    from paper_1803_04572_amd import copa
    K, R, iters = 150, 10, 5
    ik = np.random.default_rng(11).integers(3, 40, size=K)
    coh = synth.ehr_cohort(K, J, ik, 7, 1.1, 11)
    plan = copa.Plan.from_cohort(coh, R=R, l=l)
    assert (plan.query("chunks") > 0) == chunked
    g = run_gpu(coh, R, l, iters)
    o, prob = run_oracle(coh, R, l, iters)
    fit_rel = abs(g["rep"]["fit"] - o.fit[-1]) / abs(o.fit[-1])
    cong = dict(H=congruence(g["H"], o.H), V=congruence(g["V"], o.V), W=congruence(g["W"], o.W),
                U=congruence(stacked_U(split_rows(coh, g["Qt"]), g["H"]),
                             stacked_U(o.Qtilde, o.H)))
    _report(f"wide J={J} l={l}", fit_gpu=g["rep"]["fit"], fit_oracle=o.fit[-1], fit_rel=fit_rel,
            **{f"cong_{k}": v for k, v in cong.items()})
    assert fit_rel <= FIT_RTOL
    assert min(cong.values()) >= CONGRUENCE_MIN


@pytest.mark.parametrize("scale,compact", [(1.0, 1), (1.1, 0)])
def test_value_storage_forms(scale, compact):
    """Integer counts are stored in the lossless 4-byte form (feature id + bfloat16 value); other
    values keep FP32 nonzeros. Both forms fit the oracle."""
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c2", K=300)
    coh.val = (coh.val * np.float32(scale)).astype(np.float32)
    plan = copa.Plan.from_cohort(coh, R=10, l=7)
    assert plan.query("compact") == compact
    assert plan.query("chunks") > 0
    g = run_gpu(coh, 10, 7, 10)
    o, prob = run_oracle(coh, 10, 7, 10)
    fit_rel = abs(g["rep"]["fit"] - o.fit[-1]) / abs(o.fit[-1])
    cong = min(congruence(g["H"], o.H), congruence(g["V"], o.V), congruence(g["W"], o.W))
    _report(f"storage scale={scale}", fit_rel=fit_rel, cong=cong)
    assert fit_rel <= FIT_RTOL and cong >= CONGRUENCE_MIN


def test_graph_replay_matches_kernel_by_kernel_launches():
    """Outer iterations replayed from the captured hipGraph give the same fit as launching the
    kernels one by one; the graph is replayed several times (same and changed state buffers) with
    eager work and synchronisations between the replays, and every replay is checked."""
    import torch
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c2", K=500)
    R, l = 10, 7
    plan = copa.Plan.from_cohort(coh, R=R, l=l)
    init = synth.init_factors(coh.K, coh.J, R, 0)
    plan.set_graph(False)
    st = plan.new_state(*init)
    ref, _ = plan.fit(st, 6)
    torch.cuda.synchronize()
    ref_V = st["V"].double().cpu().numpy()
    plan.set_graph(True)
    st2 = None
    for rep in range(3):
        if rep == 1:  # the same buffers again, reset to the initial point
            fresh = plan.new_state(*init)
            for k in ("H", "W", "V", "D_H", "D_W", "D_V"):
                st2[k].copy_(fresh[k])
            st2["iter"] = 0
        else:  # new buffers (a new capture)
            st2 = plan.new_state(*init)
        got, _ = plan.fit(st2, 6)
        torch.cuda.synchronize()
        x = torch.randn(1 << 20, device="cuda").sum().item()  # eager work between replays
        assert np.isfinite(x)
        rel = abs(got["fit"] - ref["fit"]) / abs(ref["fit"])
        dV = np.abs(st2["V"].double().cpu().numpy() - ref_V).max() / np.abs(ref_V).max()
        _report(f"graph replay {rep}", fit_rel=rel, dV=dV)
        assert rel <= 1e-6 and dV <= 1e-4
        assert np.allclose(got["fit_history"], ref["fit_history"], rtol=1e-6)


def test_invalid_csr_is_rejected_on_device():
    import torch
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c1", K=10)
    bad = coh.col.copy()
    bad[3] = coh.J + 5
    with pytest.raises(copa.CopaError) as e:
        copa.Plan(torch.as_tensor(coh.subj_ptr).cuda(), torch.as_tensor(coh.row_ptr).cuda(),
                  torch.as_tensor(bad).cuda(), torch.as_tensor(coh.val).cuda(),
                  torch.as_tensor(coh.days).cuda(), coh.J, 7, 5)
    assert e.value.status == copa.EINVAL and "outside" in str(e.value)
