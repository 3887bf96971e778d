"""FP64 CPU oracle for COPA (constrained PARAFAC2 fitted by AO-ADMM).

TEST INFRASTRUCTURE ONLY. This module is the plain, slow reference that the GPU library is checked
against. Only the test-suite, the package smoke check and the benchmark's CPU-baseline leg may
import it; the library never calls it and shares no code with it.

Everything is FP64 NumPy/SciPy, one subject at a time, in the order the paper states the steps.
Citations name the paper's sections, equations and Algorithm 1 ("COPA").

Readings of points the paper leaves open (each is also a keyword argument where it is a number):
  * Procrustes (Section "General Framework", eq. solv_Q, Algorithm 1 truncated-SVD step): Q_k is
    the polar factor of A_k = X_k V S_k H^T, truncated to singular values > rtol * sigma_1
    (rtol = 1e-6); the zero matrix when sigma_1 == 0. For I_k < R this gives orthonormal rows.
  * Block order H -> W -> V (Algorithm 1 names Z1=H, Z2=W, Z3=V) by default; each mode's Gram G
    and MTTKRP F use the auxiliary (constrained) value of the modes updated before it. The option
    order="WHV" runs the blocks W -> H -> V instead: W's Gram and MTTKRP then take the H of the
    previous outer iteration and H's take the new W. Both orders are block-coordinate sweeps over
    the same blocks, so they share their fixed points; the iterates differ.
  * rho = trace(G) / R (Algorithm 1; the text's alternative is not used).
  * Auxiliary and dual variables persist across outer iterations; D starts at 0 and is not
    rescaled when rho changes.
  * prox argument is Z - D; l1 is the signed soft threshold sign(x) max(|x| - lam/rho, 0);
    l0 keeps x when x^2 > mu (mu passed directly); nonneg_l1 is max(0, x - lam/rho).
  * Smoothing (Section "Smoothness on U_k"): cubic B-spline basis on [t_1, t_n] in days with
    l - 4 equally spaced interior knots, clamped ends, half-open base intervals with the last one
    closed, 0/0 = 0; C_k = left singular vectors of M_k with sigma > 1e-10 sigma_1. When
    t_1 == t_n the basis is the constant function (C_k = ones / sqrt(I_k)).
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.linalg
import scipy.sparse as sp

PROX_NONE, PROX_NONNEG, PROX_L1, PROX_L0, PROX_NONNEG_L1 = 0, 1, 2, 3, 4

# ---------------------------------------------------------------------------------------------
# Spline basis (Section "Smoothness on U_k": Cox-de Boor style recursion on knots beta)
# ---------------------------------------------------------------------------------------------


def spline_knots(t1, tn, l, degree):
    """Clamped knot vector with l basis functions of the given degree on [t1, tn]."""
    n_inner = l - degree - 1
    inner = [t1 + (tn - t1) * j / (n_inner + 1) for j in range(1, n_inner + 1)]
    return np.array([t1] * (degree + 1) + inner + [tn] * (degree + 1), dtype=np.float64)


def _ratio(num, den):
    return 0.0 if den == 0.0 else num / den


def bspline_value(i, d, t, beta):
    """Basis function i of degree d at t by the recursion of the smoothness section:
    m_{i,d}(t) = (t-b_i)/(b_{i+d}-b_i) m_{i,d-1}(t) + (b_{i+d+1}-t)/(b_{i+d+1}-b_{i+1}) m_{i+1,d-1}(t),
    m_{i,0}(t) = 1 on [b_i, b_{i+1}) (the last nonempty interval also holds its right end)."""
    if d == 0:
        lo, hi = beta[i], beta[i + 1]
        if lo <= t < hi:
            return 1.0
        last = np.flatnonzero(beta[1:] > beta[:-1])
        if last.size and i == last[-1] and t == hi:
            return 1.0
        return 0.0
    a = _ratio(t - beta[i], beta[i + d] - beta[i]) * bspline_value(i, d - 1, t, beta)
    b = _ratio(beta[i + d + 1] - t, beta[i + d + 1] - beta[i + 1]) * \
        bspline_value(i + 1, d - 1, t, beta)
    return a + b


def spline_table(t, beta, d):
    """All basis functions of degree d on knots beta at the points t (n x (len(beta)-1-d)): the
    same recursion as bspline_value, run level by level over arrays instead of one point and one
    function at a time."""
    t = np.asarray(t, dtype=np.float64)[:, None]
    lo, hi = beta[:-1][None, :], beta[1:][None, :]
    m = ((lo <= t) & (t < hi)).astype(np.float64)          # degree 0, half-open pieces
    last = np.flatnonzero(beta[1:] > beta[:-1])
    if last.size:                                          # the last nonempty piece is closed
        j = last[-1]
        m[:, j] = np.where(t[:, 0] == beta[j + 1], 1.0, m[:, j])
    for dd in range(1, d + 1):
        n = len(beta) - 1 - dd
        i = np.arange(n)
        den_a = beta[i + dd] - beta[i]
        den_b = beta[i + dd + 1] - beta[i + 1]
        with np.errstate(divide="ignore", invalid="ignore"):
            a = np.where(den_a > 0, (t - beta[i][None, :]) / np.where(den_a > 0, den_a, 1.0), 0.0)
            b = np.where(den_b > 0, (beta[i + dd + 1][None, :] - t) / np.where(den_b > 0, den_b, 1.0),
                         0.0)
        m = a * m[:, :n] + b * m[:, 1:n + 1]
    return m


def spline_basis(days, l):
    """M_k (I_k x l): the l basis functions evaluated at the subject's visit days."""
    days = np.asarray(days, dtype=np.float64)
    t1, tn = float(days.min()), float(days.max())
    d = min(3, l - 1)
    beta = spline_knots(t1, tn, l, d)
    return spline_table(days, beta, d)


def smoothing_basis(days, l, tol=1e-10):
    """C_k: orthonormal basis of span(M_k) from the thin SVD M_k = C O P^T, keeping singular values
    above tol * sigma_1 (smoothness section: projected data X'_k = C_k^T X_k)."""
    days = np.asarray(days, dtype=np.float64)
    if days.size == 0:
        return np.zeros((0, 0))
    if days.max() == days.min():
        return np.ones((days.size, 1)) / np.sqrt(days.size)
    M = spline_basis(days, l)
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    r = int(np.sum(s > tol * s[0])) if s.size and s[0] > 0 else 0
    return U[:, :r]


# ---------------------------------------------------------------------------------------------
# Procrustes step (eq. solv_Q; Algorithm 1: truncated SVD, Q_k = B_k C_k^T)
# ---------------------------------------------------------------------------------------------


def procrustes(A, rtol=1e-6):
    """Truncated polar factor of A: argmax tr(Q^T A) over ||Q||_2 <= 1 of minimum norm.
    Returns (Q, rank, singular values)."""
    A = np.asarray(A, dtype=np.float64)
    if A.size == 0:
        return np.zeros_like(A), 0, np.zeros(0)
    B, s, Ct = np.linalg.svd(A, full_matrices=False)
    if s[0] <= 0.0:
        return np.zeros_like(A), 0, s
    r = int(np.sum(s > rtol * s[0]))
    return B[:, :r] @ Ct[:r, :], r, s


# ---------------------------------------------------------------------------------------------
# Proximity operators (Section "Examples of useful constraints")
# ---------------------------------------------------------------------------------------------


def prox(x, kind, lam, rho):
    x = np.asarray(x, dtype=np.float64)
    if kind == PROX_NONE:
        return x.copy()
    if kind == PROX_NONNEG:
        return np.maximum(x, 0.0)
    if kind == PROX_L1:
        return np.sign(x) * np.maximum(np.abs(x) - lam / rho, 0.0)
    if kind == PROX_L0:
        return np.where(x * x > lam, x, 0.0)
    if kind == PROX_NONNEG_L1:
        return np.maximum(x - lam / rho, 0.0)
    raise ValueError(f"unknown prox kind {kind}")


# ---------------------------------------------------------------------------------------------
# ADMM update of one factor (update rules after eq. Solve_W; Algorithm 1 inner loop)
# ---------------------------------------------------------------------------------------------


def admm_update(G, F, Zbar, D, kind, lam, n_inner):
    """n_inner ADMM steps for min 1/2||Y_(n)^T - KR Z^T||^2 + c(Zbar), Z = Zbar, rows of Z.
    G: R x R Gram, F: rows x R MTTKRP. Returns (Zbar, D, rho)."""
    R = G.shape[0]
    rho = np.trace(G) / R
    L = np.linalg.cholesky(G + rho * np.eye(R))
    Zbar = np.array(Zbar, dtype=np.float64)
    D = np.array(D, dtype=np.float64)
    for _ in range(n_inner):
        rhs = F + rho * (Zbar + D)
        Zt = scipy.linalg.solve_triangular(L, rhs.T, lower=True)
        Zt = scipy.linalg.solve_triangular(L.T, Zt, lower=False)
        Z = Zt.T
        Zbar = prox(Z - D, kind, lam, rho)
        D = D + Zbar - Z
    return Zbar, D, rho


# ---------------------------------------------------------------------------------------------
# Data access
# ---------------------------------------------------------------------------------------------


def subject_matrices(coh):
    """X_k as FP64 scipy CSR (I_k x J), one per subject."""
    out = []
    for k in range(coh.K):
        r0, r1 = int(coh.subj_ptr[k]), int(coh.subj_ptr[k + 1])
        n0, n1 = int(coh.row_ptr[r0]), int(coh.row_ptr[r1])
        indptr = (coh.row_ptr[r0:r1 + 1] - n0).astype(np.int64)
        out.append(sp.csr_matrix((coh.val[n0:n1].astype(np.float64),
                                  coh.col[n0:n1].astype(np.int64), indptr),
                                 shape=(r1 - r0, coh.J)))
    return out


@dataclasses.dataclass
class Problem:
    """Per-subject data of one fit: X_k, the projection C_k (None when unsmoothed) and X'_k."""
    X: list
    C: list
    Xh: list
    J: int
    normX2: float


def build_problem(coh, l):
    Xs = subject_matrices(coh)
    Cs, Xh = [], []
    for k, Xk in enumerate(Xs):
        if l > 0:
            r0, r1 = int(coh.subj_ptr[k]), int(coh.subj_ptr[k + 1])
            C = smoothing_basis(coh.days[r0:r1], l)
            Cs.append(C)
            Xh.append(np.asarray((Xk.T @ C).T))       # X'_k = C_k^T X_k (dense r_k x J)
        else:
            Cs.append(None)
            Xh.append(Xk)
    normX2 = float(sum(Xk.multiply(Xk).sum() for Xk in Xs))
    return Problem(X=Xs, C=Cs, Xh=Xh, J=coh.J, normX2=normX2)


def _dense(M):
    return M.toarray() if sp.issparse(M) else np.asarray(M)


# ---------------------------------------------------------------------------------------------
# MTTKRP of the intermediate tensor Y (slices Y_k = Q_k^T X'_k), by the slice-wise definition
#   Y_(1)(W (.) V) = sum_k Y_k V diag(W_k)          (R x R)
#   Y_(3)(V (.) H) : row k = diag(H^T Y_k V)        (K x R)
#   Y_(2)(W (.) H) = sum_k Y_k^T H diag(W_k)        (J x R)
# ---------------------------------------------------------------------------------------------


def slices_Y(prob, Qs):
    return [Q.T @ _dense(Xh) for Q, Xh in zip(Qs, prob.Xh)]


def mttkrp_H(Ys, V, W):
    return sum(Y @ V @ np.diag(W[k]) for k, Y in enumerate(Ys))


def mttkrp_W(Ys, H, V):
    return np.array([np.diag(H.T @ Y @ V) for Y in Ys])


def mttkrp_V(Ys, H, W):
    return sum(Y.T @ H @ np.diag(W[k]) for k, Y in enumerate(Ys))


def fit_value(prob, Qs, H, W, V):
    """FIT = 1 - sum_k ||X_k - U_k S_k V^T||^2 / sum_k ||X_k||^2 by dense reconstruction, with
    U_k = C_k Q_k H (Section "Evaluation Metrics"; smoothness section for U_k)."""
    num = 0.0
    for k, Xk in enumerate(prob.X):
        Qt = Qs[k] if prob.C[k] is None else prob.C[k] @ Qs[k]
        E = _dense(Xk) - Qt @ H @ np.diag(W[k]) @ V.T
        num += float(np.sum(E * E))
    return 1.0 - num / prob.normX2, num


@dataclasses.dataclass
class Options:
    R: int
    outer_iters: int = 10
    inner_iters: int = 5
    prox_H: int = PROX_NONE
    prox_W: int = PROX_NONNEG
    prox_V: int = PROX_L1
    lam_H: float = 0.0
    lam_W: float = 0.0
    lam_V: float = 0.1
    rank_rtol: float = 1e-6
    order: str = "HWV"     # block order of one outer iteration: "HWV" or "WHV"


@dataclasses.dataclass
class FitResult:
    H: np.ndarray
    W: np.ndarray
    V: np.ndarray
    D_H: np.ndarray
    D_W: np.ndarray
    D_V: np.ndarray
    Q: list            # Q_k per subject (r_k x R when smoothed, else I_k x R)
    Qtilde: list       # C_k Q_k (I_k x R): U_k = Qtilde_k H
    fit: list
    objective: list
    sparsity: list
    rho: list          # (rho_H, rho_W, rho_V) per outer iteration
    F: dict            # last iteration's MTTKRPs {"H", "W", "V"}
    ranks: list        # Procrustes ranks of the last iteration
    sigmas: list       # singular values of each A_k in the last iteration


def copa_fit(prob, H0, W0, V0, opt: Options, D0=None):
    """Algorithm 1 (COPA) for a fixed number of outer iterations."""
    H, W, V = (np.array(a, dtype=np.float64) for a in (H0, W0, V0))
    if D0 is None:
        D_H, D_W, D_V = np.zeros_like(H), np.zeros_like(W), np.zeros_like(V)
    else:
        D_H, D_W, D_V = (np.array(a, dtype=np.float64) for a in D0)
    if opt.order not in ("HWV", "WHV"):
        raise ValueError(f"order must be 'HWV' or 'WHV', not {opt.order!r}")
    fits, objs, spars, rhos = [], [], [], []
    Qs, ranks, sigmas, F = [], [], [], {}

    def block_H():
        nonlocal H, D_H
        G = (W.T @ W) * (V.T @ V)
        F["H"] = mttkrp_H(Ys, V, W)
        H, D_H, r = admm_update(G, F["H"], H, D_H, opt.prox_H, opt.lam_H, opt.inner_iters)
        return r

    def block_W():
        nonlocal W, D_W
        G = (H.T @ H) * (V.T @ V)
        F["W"] = mttkrp_W(Ys, H, V)
        W, D_W, r = admm_update(G, F["W"], W, D_W, opt.prox_W, opt.lam_W, opt.inner_iters)
        return r

    for _ in range(opt.outer_iters):
        # Procrustes: Q_k from the truncated SVD of X'_k V S_k H^T, then Y_k = Q_k^T X'_k
        Qs, ranks, sigmas = [], [], []
        for k, Xh in enumerate(prob.Xh):
            A = Xh @ V @ np.diag(W[k]) @ H.T
            Q, r, sv = procrustes(A, opt.rank_rtol)
            Qs.append(Q)
            ranks.append(r)
            sigmas.append(sv)
        Ys = slices_Y(prob, Qs)
        # mode 1 of Algorithm 1: H; mode 2: W (the diagonals of S_k); in either order
        if opt.order == "HWV":
            rH = block_H()
            rW = block_W()
        else:
            rW = block_W()
            rH = block_H()
        # mode 3 of Algorithm 1: V
        G = (H.T @ H) * (W.T @ W)
        F["V"] = mttkrp_V(Ys, H, W)
        V, D_V, rV = admm_update(G, F["V"], V, D_V, opt.prox_V, opt.lam_V, opt.inner_iters)
        f, resid = fit_value(prob, Qs, H, W, V)
        fits.append(f)
        objs.append(0.5 * resid + penalty(V, opt.prox_V, opt.lam_V)
                    + penalty(W, opt.prox_W, opt.lam_W) + penalty(H, opt.prox_H, opt.lam_H))
        spars.append(float(np.mean(V == 0.0)))
        rhos.append((rH, rW, rV))
    Qt = [Q if prob.C[k] is None else prob.C[k] @ Q for k, Q in enumerate(Qs)]
    return FitResult(H=H, W=W, V=V, D_H=D_H, D_W=D_W, D_V=D_V, Q=Qs, Qtilde=Qt, fit=fits,
                     objective=objs, sparsity=spars, rho=rhos, F=F, ranks=ranks, sigmas=sigmas)


def penalty(Z, kind, lam):
    if kind in (PROX_L1, PROX_NONNEG_L1):
        return lam * float(np.abs(Z).sum())
    return 0.0


# ---------------------------------------------------------------------------------------------
# Reconstruction loss and its gradient (eq. Classic_PARAFAC2_obj_func with U_k = Qtilde_k H)
# ---------------------------------------------------------------------------------------------


def loss_grad(Xs, Qts, H, V, W):
    """L = 1/2 sum_k ||X_k - Qt_k H S_k V^T||^2 with S_k = diag(W_k) and Qt_k held fixed.
    Returns (L, dL/dH, dL/dV, dL/dW, [dL/dS_k full R x R])."""
    H, V, W = (np.asarray(a, dtype=np.float64) for a in (H, V, W))
    L = 0.0
    dH = np.zeros_like(H)
    dV = np.zeros_like(V)
    dW = np.zeros_like(W)
    dS = []
    for k, Xk in enumerate(Xs):
        S = np.diag(W[k])
        E = _dense(Xk) - Qts[k] @ H @ S @ V.T
        L += 0.5 * float(np.sum(E * E))
        dH -= Qts[k].T @ E @ V @ S
        dV -= E.T @ Qts[k] @ H @ S
        dSk = -H.T @ Qts[k].T @ E @ V
        dS.append(dSk)
        dW[k] = np.diag(dSk)
    return L, dH, dV, dW, dS


def stationarity(Xs, Qts, H, V, W, opt):
    """Stationarity residual of each factor block of the penalised reconstruction loss with Q held
    fixed: r_n = ||Z_n - prox_n(Z_n - grad_n L / rho_n)||_F / ||Z_n||_F, where prox_n is that
    block's proximity operator with its weight (Section "Examples of useful constraints") and
    rho_n = trace(G_n) / R with G_H = W^TW * V^TV, G_W = H^TH * V^TV, G_V = H^TH * W^TW (the step
    of Algorithm 1). r_n = 0 exactly when Z_n is a fixed point of the proximal-gradient map, i.e.
    when Z_n satisfies the first-order conditions of its block. Returns (r_H, r_W, r_V)."""
    H, V, W = (np.asarray(a, dtype=np.float64) for a in (H, V, W))
    _, dH, dV, dW, _ = loss_grad(Xs, Qts, H, V, W)
    HtH, VtV, WtW = H.T @ H, V.T @ V, W.T @ W
    R = H.shape[0]
    out = []
    for Z, G, dZ, kind, lam in ((H, WtW * VtV, dH, opt.prox_H, opt.lam_H),
                                (W, HtH * VtV, dW, opt.prox_W, opt.lam_W),
                                (V, HtH * WtW, dV, opt.prox_V, opt.lam_V)):
        rho = np.trace(G) / R
        step = prox(Z - dZ / rho, kind, lam, rho)
        nz = np.linalg.norm(Z)
        out.append(float(np.linalg.norm(Z - step) / nz) if nz > 0 else 0.0)
    return tuple(out)
