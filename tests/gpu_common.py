"""Helpers shared by the GPU parity tests: run the library and the oracle on the same inputs."""
import numpy as np

import oracle
from oracle import copa_oracle as co
from paper_1803_04572_amd import synth

FIT_RTOL = 1e-5        # relative FIT difference allowed in FP32
CONGRUENCE_MIN = 0.999


def congruence(A, B):
    """Per-column |a.b| / (|a||b|), minimum over columns (both zero -> 1, one zero -> 0)."""
    A, B = np.asarray(A, float), np.asarray(B, float)
    out = []
    for a, b in zip(A.T, B.T):
        na, nb = np.linalg.norm(a), np.linalg.norm(b)
        if na == 0 and nb == 0:
            out.append(1.0)
        elif na == 0 or nb == 0:
            out.append(0.0)
        else:
            out.append(abs(a @ b) / (na * nb))
    return min(out) if out else 1.0


def stacked_U(Qts, H):
    return np.concatenate([Q @ H for Q in Qts], axis=0) if Qts else np.zeros((0, H.shape[0]))


def run_gpu(coh, R, l, iters, seed=0, inner=5, prox=(co.PROX_NONE, co.PROX_NONNEG, co.PROX_L1),
            lam=(0.0, 0.0, 0.1), init=None, **plan_kw):
    import torch
    from paper_1803_04572_amd import copa
    plan_kw.setdefault("adjoint", True)
    plan = copa.Plan.from_cohort(coh, R=R, l=l, inner_iters=inner, prox=prox, lam=lam, **plan_kw)
    H0, W0, V0 = init if init is not None else synth.init_factors(coh.K, coh.J, R, seed)
    st = plan.new_state(H0, W0, V0)
    rep, Qt = plan.fit(st, iters)
    torch.cuda.synchronize()
    out = {k: v.double().cpu().numpy() for k, v in st.items() if k != "iter"}
    out["Qt"] = Qt.double().cpu().numpy()
    out["rep"] = rep
    out["plan"] = plan
    return out


def run_oracle(coh, R, l, iters, seed=0, inner=5, prox=(co.PROX_NONE, co.PROX_NONNEG, co.PROX_L1),
               lam=(0.0, 0.0, 0.1), init=None):
    prob = co.build_problem(coh, l)
    H0, W0, V0 = init if init is not None else synth.init_factors(coh.K, coh.J, R, seed)
    opt = co.Options(R=R, outer_iters=iters, inner_iters=inner, prox_H=prox[0], prox_W=prox[1],
                     prox_V=prox[2], lam_H=lam[0], lam_W=lam[1], lam_V=lam[2])
    return co.copa_fit(prob, H0, W0, V0, opt), prob


def split_rows(coh, X):
    return [X[coh.subj_ptr[k]:coh.subj_ptr[k + 1]] for k in range(coh.K)]


def procrustes_condition(coh, R, l, H, W, V, rtol=1e-6):
    """Per subject: sigma_1 / sigma_r of A_k = X'_k V S_k H^T over the kept singular values (the
    sensitivity of the polar factor to a relative perturbation of A_k)."""
    prob = co.build_problem(coh, l)
    out = []
    for k, Xh in enumerate(prob.Xh):
        A = Xh @ V @ np.diag(W[k]) @ H.T
        s = np.linalg.svd(np.asarray(A), compute_uv=False) if A.size else np.zeros(0)
        if s.size == 0 or s[0] == 0:
            out.append(1.0)
            continue
        kept = s[s > rtol * s[0]]
        out.append(kept[0] / kept[-1])
    return np.array(out)
