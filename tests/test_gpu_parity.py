"""GPU path (libcopa.so through the C ABI) against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

from oracle import copa_oracle as co
from paper_1803_04572_amd import synth
from gpu_common import (CONGRUENCE_MIN, FIT_RTOL, ambiguous_band, check_fit, congruence,
                        procrustes_condition, run_gpu, run_oracle, split_rows, stacked_U)

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
    # Q_k: a relative perturbation eps of A_k moves its polar factor by up to about eps * kappa_k
    # (kappa_k = sigma_1 / sigma_r over the kept singular values); the bound is asserted where
    # kappa_k <= 1e4 and capped at 1e-3. Subjects past that, or with a singular value near the
    # truncation threshold (the ambiguous band), are checked for structure instead: Qtilde_k^T
    # Qtilde_k is a projector of the oracle's rank.
    H0, W0, V0 = synth.init_factors(coh.K, coh.J, R, 0)
    kappa = procrustes_condition(coh, R, l, H0, W0, V0)
    Qg = split_rows(coh, g["Qt"])
    band = [bool(sv.size and sv[0] > 0 and np.any((sv / sv[0] >= 1e-7) & (sv / sv[0] <= 1e-5)))
            for sv in o.sigmas]
    worst_scaled, worst_abs, n_struct = 0.0, 0.0, 0
    for a, b, kap, amb, r in zip(Qg, o.Qtilde, kappa, band, o.ranks):
        d = np.abs(a - b).max(initial=0.0)
        worst_abs = max(worst_abs, d)
        if kap <= 1e4 and not amb:
            worst_scaled = max(worst_scaled, d / min(1e-5 + 1e-6 * kap, 1e-3))
        else:
            n_struct += 1
            P = a.T @ a
            assert np.abs(P @ P - P).max() < 1e-4 and abs(np.trace(P) - r) < 1e-3
        if a.size:  # ranks agree wherever the truncation is not ambiguous
            if not amb:
                assert abs(np.trace(a.T @ a) - r) < 1e-3
    errs = dict(
        Qt_scaled=worst_scaled * 2e-4,
        FH=np.abs(FH - o.F["H"]).max() / np.abs(o.F["H"]).max(),
        FW=np.abs(FW - o.F["W"]).max() / np.abs(o.F["W"]).max(),
        FV=np.abs(FV - o.F["V"]).max() / np.abs(o.F["V"]).max(),
        H=np.abs(g["H"] - o.H).max() / np.abs(o.H).max(),
        W=np.abs(g["W"] - o.W).max() / np.abs(o.W).max(),
        V=np.abs(g["V"] - o.V).max() / np.abs(o.V).max(),
        fit=abs(g["rep"]["fit"] - o.fit[-1]) / abs(o.fit[-1]))
    print(f"step {cfg_name}: max |dQ| {worst_abs:.2e}, structure-checked subjects {n_struct}, "
          f"ambiguous band {sum(band)}", flush=True)
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
    check_fit(f"fit {cfg_name} K={coh.K} R={R} l={l}", coh, g, o, prob, R)


# Constraint variants of Section "Examples of useful constraints": l0 (hard threshold, mu passed
# as the weight), non-negativity on every factor ("Non-neg COPA"), nonnegative l1, and l1 on W.
PX = co
@pytest.mark.parametrize("name,prox,lam", [
    ("l0_V", (PX.PROX_NONE, PX.PROX_NONNEG, PX.PROX_L0), (0.0, 0.0, 0.01)),
    ("nonneg_all", (PX.PROX_NONNEG, PX.PROX_NONNEG, PX.PROX_NONNEG), (0.0, 0.0, 0.0)),
    ("nonneg_l1_V", (PX.PROX_NONE, PX.PROX_NONNEG, PX.PROX_NONNEG_L1), (0.0, 0.0, 2.0)),
    ("l1_W_l1_V", (PX.PROX_NONE, PX.PROX_L1, PX.PROX_L1), (0.0, 0.5, 2.0)),
])
@pytest.mark.parametrize("cfg_name,K,R,l", [("c2", 400, 10, 7), ("c5", 300, 10, 0)])
def test_constraint_variants_parity(name, prox, lam, cfg_name, K, R, l):
    coh, cfg = synth.make_config(cfg_name, K=K)
    init = synth.init_factors(coh.K, coh.J, R, 0)
    if prox[0] == PX.PROX_NONNEG:
        # from H = I the non-negative H block collapses to zero on this data (then G_W = 0 and
        # the W system is singular, in the oracle as well): start from a seeded non-negative H
        H1 = np.random.default_rng(3).random((R, R)).astype(np.float32).astype(np.float64)
        init = (H1, init[1], init[2])
    g = run_gpu(coh, R, l, 10, prox=prox, lam=lam, init=init)
    o, prob = run_oracle(coh, R, l, 10, prox=prox, lam=lam, init=init)
    check_fit(f"constraints {name} {cfg_name}", coh, g, o, prob, R, spars_entries=3)
    if prox[2] in (PX.PROX_L0, PX.PROX_NONNEG_L1):
        assert o.sparsity[-1] > 0.05  # the variant really zeroes entries of V
    if prox[2] in (PX.PROX_NONNEG, PX.PROX_NONNEG_L1):
        assert (g["V"] >= 0).all()
    if prox[0] == PX.PROX_NONNEG:
        assert (g["H"] >= 0).all()


@pytest.mark.parametrize("R,l", [(10, 4), (10, 8), (20, 8), (5, 3)])
def test_basis_sizes_parity(R, l):
    """Spline bases of 3, 4 and 8 functions per subject (the general-l Procrustes kernels)."""
    coh, cfg = synth.make_config("c2", K=300)
    g = run_gpu(coh, R, l, 8)
    o, prob = run_oracle(coh, R, l, 8)
    check_fit(f"basis l={l} R={R}", coh, g, o, prob, R)


@pytest.mark.parametrize("order", ["HWV", "WHV"])
@pytest.mark.parametrize("l", [7, 0])
def test_subjects_without_visits(l, order):
    """Subjects with no visit rows (I_k = 0) among the others: they contribute nothing to any
    MTTKRP and their W rows follow the ADMM steps with F_W = 0, as in the oracle (either block
    order)."""
    base, _ = synth.make_config("c2", K=200)
    ik = np.diff(base.subj_ptr)
    ik2 = np.insert(ik, [0, 5, 5, 77, 200], 0)  # empty subjects first, in a run, inside, last
    subj_ptr = np.concatenate([[0], np.cumsum(ik2)]).astype(np.int64)
    coh = synth.Cohort(K=ik2.size, J=base.J, subj_ptr=subj_ptr, row_ptr=base.row_ptr,
                       col=base.col, val=base.val, days=base.days)
    R = 10
    g = run_gpu(coh, R, l, 8, order=order)
    o, prob = run_oracle(coh, R, l, 8, order=order)
    check_fit(f"empty subjects l={l} order={order}", coh, g, o, prob, R)
    np.testing.assert_allclose(g["W"][ik2 == 0], o.W[ik2 == 0], rtol=1e-4, atol=1e-6)


def test_numeric_failure_is_reported():
    """A weight large enough to zero V leaves the next iteration's Gram of the H block at zero
    (rho = 0, a singular ADMM system): the fit stops with COPA_ENUMERIC at that iteration. The
    oracle's Cholesky of the same system fails the same way."""
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c5", K=100)
    R = 5
    prox, lam = (co.PROX_NONE, co.PROX_NONNEG, co.PROX_L1), (0.0, 0.0, 1e12)
    with pytest.raises(np.linalg.LinAlgError):
        run_oracle(coh, R, 0, 3, prox=prox, lam=lam)
    plan = copa.Plan.from_cohort(coh, R=R, l=0, prox=prox, lam=lam)
    st = plan.new_state(*synth.init_factors(coh.K, coh.J, R, 0))
    with pytest.raises(copa.CopaError) as e:
        plan.fit(st, 3)
    assert e.value.status == copa.ENUMERIC
    assert e.value.report["fail_iter"] == 1
    assert float(np.abs(st["V"].cpu().numpy()).max()) == 0.0


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


@pytest.mark.parametrize("R,l,order", [(1, 7, "HWV"), (3, 0, "HWV"), (12, 7, "HWV"),
                                       (16, 7, "HWV"), (16, 0, "HWV"), (24, 7, "HWV"),
                                       (32, 7, "HWV"), (32, 0, "HWV"), (3, 7, "WHV"),
                                       (16, 7, "WHV"), (32, 7, "WHV"), (6, 0, "WHV")])
def test_rank_coverage(R, l, order):
    """Ranks the library builds beyond the workloads' (R = 1 .. 32, one subject per lane up to a
    wavefront per subject), smoothed and plain, in both block orders, against the oracle."""
    coh, _ = synth.make_config("c2", K=300)
    g = run_gpu(coh, R, l, 6, order=order)
    o, prob = run_oracle(coh, R, l, 6, order=order)
    check_fit(f"rank R={R} l={l} order={order}", coh, g, o, prob, R)
