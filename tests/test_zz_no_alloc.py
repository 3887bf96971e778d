"""copa_loss_grad_static (the adjoint without device allocation: a static 64 MiB work array per
GPU) against copa_loss_grad on the same plan and inputs, on two calls in a row (the second with a
smaller cohort), on a plan created without the adjoint's workspace, and past its size limit."""
import numpy as np
import pytest

from paper_1803_04572_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(a, b):
    a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("det", [True, False])
def test_static_adjoint_matches_loss_grad(det):
    import torch
    from paper_1803_04572_amd import copa
    R = 10
    for K, l in ((2000, 0), (400, 7)):  # the second call is smaller
        coh, _ = synth.make_config("c5" if l == 0 else "c2", K=K)
        plan = copa.Plan.from_cohort(coh, R=R, l=l, adjoint=True, deterministic=det)
        st = plan.new_state(*synth.init_factors(coh.K, coh.J, R, 0))
        _, Qt = plan.fit(st, 2)
        H, V, W = st["H"], st["V"], st["W"]
        ref = plan.loss_grad(H, V, W, Qt, want_dS=True)
        got = plan.loss_grad_static(H, V, W, Qt, want_dS=True)
        torch.cuda.synchronize()
        rl = abs(got[0] - ref[0]) / abs(ref[0])
        errs = [_rel(g, r) for g, r in zip(got[1:], ref[1:])]
        print(f"static adjoint K={K} l={l} det={det}: loss rel {rl:.2e} grad rel {errs}",
              flush=True)
        # the bar of the adjoint's parity tests (1e-4 of the largest entry); without the fixed
        # order, F_V's float atomics alone move dV = V Psi' - F_V by ~1e-5 between two runs
        assert rl <= 1e-6 and max(errs) <= 1e-4
        if det:
            assert got[0] == ref[0] and all(torch.equal(g, r) for g, r in zip(got[1:], ref[1:]))
        # a plan without the adjoint's workspace gives the same through the static array
        bare = copa.Plan.from_cohort(coh, R=R, l=l, deterministic=det)
        got2 = bare.loss_grad_static(H, V, W, Qt, want_dS=False)
        torch.cuda.synchronize()
        assert abs(got2[0] - ref[0]) <= 1e-6 * abs(ref[0])
        assert max(_rel(g, r) for g, r in zip(got2[1:4], ref[1:4])) <= 1e-4


def test_static_adjoint_refuses_sizes_past_its_array():
    import torch
    from paper_1803_04572_amd import copa
    coh, _ = synth.make_config("c5", K=9000)  # 2 S R > 16 Mi floats at R = 10
    assert 2 * coh.S * 10 > (16 << 20)
    plan = copa.Plan.from_cohort(coh, R=10, l=0)
    st = plan.new_state(*synth.init_factors(coh.K, coh.J, 10, 0))
    _, Qt = plan.fit(st, 1)
    with pytest.raises(copa.CopaError) as e:
        plan.loss_grad_static(st["H"], st["V"], st["W"], Qt)
    assert e.value.status == copa.EINVAL and "static scratch" in str(e.value)
    torch.cuda.synchronize()
