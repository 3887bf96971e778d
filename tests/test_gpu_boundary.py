"""The C ABI's workspace, caller basis, fixed-order mode and resume, through the library on the GPU.

Each test compares the library with itself under a change that must not change the numbers
(where the workspace lives, how the basis is handed over, where a fit is split), or with the FP64
oracle where the basis changes."""
import numpy as np
import pytest

from oracle import copa_oracle as co
from paper_1803_04572_amd import synth
from gpu_common import CONGRUENCE_MIN, FIT_RTOL, congruence, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _fit(plan, init, iters, fresh=True):
    import torch
    st = plan.new_state(*init)
    rep, Qt = plan.fit(st, iters, fresh=fresh)
    torch.cuda.synchronize()
    return rep, {k: v.cpu().numpy() for k, v in st.items() if k != "iter"}, Qt.cpu().numpy()


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


@pytest.mark.parametrize("order", ["HWV", "WHV"])
def test_caller_workspace_equals_library_workspace(order):
    """A plan laid out in a caller-provided workspace gives bitwise the same fit (fixed-order
    mode) as one whose workspace the library allocated."""
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c2", K=700)
    init = synth.init_factors(coh.K, coh.J, 10, 0)
    a = copa.Plan.from_cohort(coh, R=10, l=7, deterministic=True, order=order)
    b = copa.Plan.from_cohort(coh, R=10, l=7, deterministic=True, workspace="caller", order=order)
    assert b._ws.numel() == copa.Plan.workspace_bytes(coh.K, coh.J, coh.S, coh.nnz, 7, 10,
                                                      deterministic=True, order=order)
    ra, sa, qa = _fit(a, init, 6)
    rb, sb, qb = _fit(b, init, 6)
    assert ra["fit_history"] == rb["fit_history"]
    assert _same(sa, sb) and np.array_equal(qa, qb)


def test_workspace_too_small_or_misaligned_is_rejected():
    import torch
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c1", K=20)
    dev = lambda a, t: torch.as_tensor(a).to("cuda", t)  # noqa: E731
    args = (dev(coh.subj_ptr, torch.int64), dev(coh.row_ptr, torch.int64),
            dev(coh.col, torch.int32), dev(coh.val, torch.float32), dev(coh.days, torch.float64))
    need = copa.Plan.workspace_bytes(coh.K, coh.J, coh.S, coh.nnz, 7, 5)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    L = copa.lib()
    import ctypes
    t = copa.CopaTensor(K=coh.K, J=coh.J, S=coh.S, nnz=coh.nnz,
                        subj_ptr=args[0].data_ptr(), row_ptr=args[1].data_ptr(),
                        col=args[2].data_ptr(), val=args[3].data_ptr(), days=args[4].data_ptr(),
                        l=7)
    o = copa.CopaOptions(R=5, inner_iters=5, prox_H=0, prox_W=1, prox_V=2, lambda_V=0.1)
    h = ctypes.c_void_p()
    st = L.copa_plan_create(ctypes.byref(t), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                            need - 256, None, ctypes.byref(h))
    assert st == copa.EINVAL and "needs" in copa.last_error()
    st = L.copa_plan_create(ctypes.byref(t), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr() + 64),
                            need, None, ctypes.byref(h))
    assert st == copa.EINVAL and "misaligned" in copa.last_error()
    st = L.copa_plan_create(ctypes.byref(t), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                            need, None, ctypes.byref(h))
    assert st == copa.OK
    L.copa_plan_destroy(h)


@pytest.mark.parametrize("scale", [False, True])
def test_caller_basis_equals_days_basis(scale):
    """The spline basis handed over as rows M_k (evaluated on the host) gives the fit of the plan
    that evaluates it from the visit days; a basis with rescaled columns spans the same space and
    gives the same fit too (only span(M_k) enters). Both match the oracle."""
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c2", K=400)
    R, l, iters = 10, 7, 8
    M = np.zeros((coh.S, l))
    for k in range(coh.K):
        r0, r1 = coh.subj_ptr[k], coh.subj_ptr[k + 1]
        d = coh.days[r0:r1]
        M[r0:r1] = (co.spline_basis(d, l) if d.max() > d.min()
                    else np.eye(1, l).repeat(r1 - r0, 0))
    if scale:
        M = M * np.arange(1.0, l + 1.0)[None, :]
    init = synth.init_factors(coh.K, coh.J, R, 0)
    a = copa.Plan.from_cohort(coh, R=R, l=l)
    b = copa.Plan.from_cohort(coh, R=R, l=l, basis=M)
    ra, sa, qa = _fit(a, init, iters)
    rb, sb, qb = _fit(b, init, iters)
    o, _ = run_oracle(coh, R, l, iters)
    rel_ab = abs(ra["fit"] - rb["fit"]) / abs(ra["fit"])
    rel_o = abs(rb["fit"] - o.fit[-1]) / abs(o.fit[-1])
    cong = min(congruence(sa["V"], sb["V"]), congruence(sa["H"], sb["H"]),
               congruence(sa["W"], sb["W"]))
    print(f"caller basis scale={scale}: fit days={ra['fit']:.9f} basis={rb['fit']:.9f} "
          f"oracle={o.fit[-1]:.9f} rel_ab={rel_ab:.2e} rel_oracle={rel_o:.2e} cong={cong:.7f}",
          flush=True)
    assert rel_ab <= 1e-6 and rel_o <= FIT_RTOL and cong >= CONGRUENCE_MIN
    np.testing.assert_allclose(qa, qb, atol=2e-4)


def test_fixed_order_mode_is_bitwise_reproducible():
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c2", K=900)
    init = synth.init_factors(coh.K, coh.J, 10, 0)
    plan = copa.Plan.from_cohort(coh, R=10, l=7, deterministic=True)
    r1, s1, q1 = _fit(plan, init, 8)
    r2, s2, q2 = _fit(plan, init, 8)
    other = copa.Plan.from_cohort(coh, R=10, l=7, deterministic=True)
    r3, s3, q3 = _fit(other, init, 8)
    assert r1["fit_history"] == r2["fit_history"] == r3["fit_history"]
    assert _same(s1, s2) and _same(s1, s3)
    assert np.array_equal(q1, q2) and np.array_equal(q1, q3)
    # and it is the same fit as the default mode up to summation order
    free = copa.Plan.from_cohort(coh, R=10, l=7)
    r4, s4, _ = _fit(free, init, 8)
    assert abs(r4["fit"] - r1["fit"]) <= 1e-6 * abs(r1["fit"])


@pytest.mark.parametrize("l", [7, 0])
def test_resume_continues_exactly(l):
    """10 outer iterations in one call equal 5 + 5 in two calls on the same state, bit for bit
    (fixed-order mode): the second call continues the Procrustes warm start."""
    import torch
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c2", K=600)
    R = 10
    init = synth.init_factors(coh.K, coh.J, R, 0)
    plan = copa.Plan.from_cohort(coh, R=R, l=l, deterministic=True)
    ra, sa, qa = _fit(plan, init, 10)
    st = plan.new_state(*init)
    r1, _ = plan.fit(st, 5)
    assert st["iter"] == 5
    r2, Qt = plan.fit(st, 5)
    torch.cuda.synchronize()
    assert st["iter"] == 10
    sb = {k: v.cpu().numpy() for k, v in st.items() if k != "iter"}
    assert r1["fit_history"] + r2["fit_history"] == ra["fit_history"]
    assert _same(sa, sb) and np.array_equal(qa, Qt.cpu().numpy())


def test_adjoint_needs_its_workspace():
    import torch
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c5", K=50)
    plan = copa.Plan.from_cohort(coh, R=5, l=0)
    st = plan.new_state(*synth.init_factors(coh.K, coh.J, 5, 0))
    rep, Qt = plan.fit(st, 2)
    with pytest.raises(copa.CopaError) as e:
        plan.loss_grad(st["H"], st["V"], st["W"], Qt)
    assert e.value.status == copa.EINVAL and "adjoint" in str(e.value)
    torch.cuda.synchronize()


@pytest.mark.parametrize("order", ["HWV", "WHV"])
def test_stop_checks_do_not_change_the_trajectory(order):
    """Fits that pause every few iterations for the stationarity check follow the plain fit's
    trajectory bit for bit (fixed-order mode)."""
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c5", K=200)
    R = 10
    init = synth.init_factors(coh.K, coh.J, R, 0)
    plain = copa.Plan.from_cohort(coh, R=R, l=0, deterministic=True, order=order)
    ra, sa, _ = _fit(plain, init, 12)
    stop = copa.Plan.from_cohort(coh, R=R, l=0, deterministic=True, stop_tol=1e-30,
                                 check_every=4, order=order)
    rb, sb, _ = _fit(stop, init, 12)
    assert rb["iters_done"] == 12
    assert rb["fit_history"] == ra["fit_history"]
    assert _same(sa, sb)
