"""Seeded synthetic inputs: EHR-shaped irregular sparse tensors, visit days and initial factors.

This module only draws random data. It holds none of the fitting method's arithmetic, so both the
GPU path and the FP64 CPU oracle can take their inputs from it without sharing any computation.

Layout of a cohort ("CSR by subject"): subject k owns visit rows [subj_ptr[k], subj_ptr[k+1]);
visit row i owns nonzeros [row_ptr[i], row_ptr[i+1]) of (col, val); columns are strictly
increasing within a row. ``days[i]`` is the day of visit i (first visit of each subject is day 0).

The recipes mirror the workloads of the paper's experiments (two EHR cohorts: about 250k patients x
1.4k features with up to 857 visits and 11M nonzeros, and about 843k patients x 284 features with
up to 1500 visits and 84M nonzeros; "Data Set Description", table of dataset statistics). No record
of those datasets is used: every value here is drawn from the distributions named below.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Cohort", "PlantedModel", "ehr_cohort", "planted_cohort", "visit_days", "init_factors",
    "CONFIGS", "make_config", "subset_subjects",
]


@dataclasses.dataclass
class Cohort:
    K: int
    J: int
    subj_ptr: np.ndarray   # int64 [K+1]
    row_ptr: np.ndarray    # int64 [S+1]
    col: np.ndarray        # int32 [nnz]
    val: np.ndarray        # float32 [nnz]
    days: np.ndarray       # float64 [S]

    @property
    def S(self) -> int:
        return int(self.subj_ptr[-1])

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def visits(self) -> np.ndarray:
        return np.diff(self.subj_ptr)


@dataclasses.dataclass
class PlantedModel:
    H: np.ndarray
    V: np.ndarray
    W: np.ndarray
    Q: list


def _lognormal_visits(rng, K, median, sigma, lo, hi):
    z = rng.standard_normal(K)
    ik = np.rint(np.exp(np.log(median) + sigma * z))
    return np.clip(ik, lo, hi).astype(np.int64)


def _zipf_features(rng, counts, J, s):
    """Feature ids for rows with ``counts[i]`` nonzeros each: Zipf(s) popularity over ranks, a
    uniformly random rank->feature map, no repeated feature inside a row, sorted within rows."""
    counts = np.minimum(counts.astype(np.int64), J)
    total = int(counts.sum())
    p = np.arange(1, J + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(p / p.sum())
    cdf[-1] = 1.0
    perm = rng.permutation(J).astype(np.int32)
    row_of = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
    ranks = np.searchsorted(cdf, rng.random(total), side="right").astype(np.int64)
    ranks = np.minimum(ranks, J - 1)
    for _ in range(1000):
        key = row_of * J + ranks
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup_sorted = np.zeros(total, dtype=bool)
        dup_sorted[1:] = ks[1:] == ks[:-1]
        if not dup_sorted.any():
            break
        dup = order[dup_sorted]
        ranks[dup] = np.minimum(
            np.searchsorted(cdf, rng.random(dup.size), side="right"), J - 1)
    else:  # pragma: no cover - probability ~0 for the recipes below
        raise RuntimeError("could not draw distinct features")
    feats = perm[ranks]
    order = np.lexsort((feats, row_of))
    return feats[order].astype(np.int32), counts


def visit_days(rng, subj_ptr):
    """Day of each visit: first visit of a subject is day 0, then gaps of 1+floor(LogNormal(ln 30,
    1.5)) days capped at 3650 (gaps from a day to several years between consecutive visits)."""
    S = int(subj_ptr[-1])
    gaps = 1.0 + np.floor(np.exp(np.log(30.0) + 1.5 * rng.standard_normal(S)))
    gaps = np.minimum(gaps, 3650.0)
    starts = subj_ptr[:-1]
    nonempty = starts < subj_ptr[1:]
    gaps[starts[nonempty]] = 0.0
    c = np.cumsum(gaps)
    base = np.repeat(c[starts[nonempty]], np.diff(subj_ptr)[nonempty])
    return (c - base).astype(np.float64)


def ehr_cohort(K, J, visits, nnz_per_row, zipf_s, seed):
    """EHR-like count tensor. ``visits``: int array [K] of I_k; ``nnz_per_row``: int or callable
    (rng, S) -> int array; values are Poisson(1)+1 counts."""
    rng = np.random.default_rng(seed)
    ik = np.asarray(visits, dtype=np.int64)
    subj_ptr = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(ik, out=subj_ptr[1:])
    S = int(subj_ptr[-1])
    if callable(nnz_per_row):
        counts = np.asarray(nnz_per_row(rng, S), dtype=np.int64)
    else:
        counts = np.full(S, int(nnz_per_row), dtype=np.int64)
    col, counts = _zipf_features(rng, counts, J, zipf_s)
    row_ptr = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    val = (rng.poisson(1.0, size=col.size) + 1).astype(np.float32)
    days = visit_days(rng, subj_ptr)
    return Cohort(K=K, J=J, subj_ptr=subj_ptr, row_ptr=row_ptr, col=col, val=val, days=days)


def _haar_orthonormal(rng, n, r):
    g = rng.standard_normal((n, r))
    q, rr = np.linalg.qr(g)
    return q * np.sign(np.diag(rr))[None, :]


def planted_cohort(K, J, R, ik_lo, ik_hi, seed, scale=2.0, v_zero_frac=0.7, noiseless=False):
    """PARAFAC2-shaped planted counts: X_k = Poisson(scale * max(Q_k H diag(W_k) V^T, 0)) (or the
    clipped mean itself when ``noiseless``), with Q_k Haar-orthonormal, H ~ N(0,1), V nonnegative
    with ``v_zero_frac`` zeros and Exp(1) nonzeros, W ~ U[0,1]."""
    rng = np.random.default_rng(seed)
    ik = rng.integers(ik_lo, ik_hi + 1, size=K).astype(np.int64)
    H = rng.standard_normal((R, R))
    V = rng.exponential(1.0, size=(J, R)) * (rng.random((J, R)) >= v_zero_frac)
    W = rng.random((K, R))
    subj_ptr = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(ik, out=subj_ptr[1:])
    rows_col, rows_val, row_len, Qs = [], [], [], []
    for k in range(K):
        Q = _haar_orthonormal(rng, int(ik[k]), R)
        Qs.append(Q)
        mean = np.maximum(Q @ H @ np.diag(W[k]) @ V.T, 0.0) * scale
        Xk = mean if noiseless else rng.poisson(mean).astype(np.float64)
        for i in range(Xk.shape[0]):
            nz = np.flatnonzero(Xk[i])
            rows_col.append(nz.astype(np.int32))
            rows_val.append(Xk[i, nz].astype(np.float32))
            row_len.append(nz.size)
    row_ptr = np.zeros(len(row_len) + 1, dtype=np.int64)
    np.cumsum(np.asarray(row_len, dtype=np.int64), out=row_ptr[1:])
    col = np.concatenate(rows_col) if rows_col else np.zeros(0, np.int32)
    val = np.concatenate(rows_val) if rows_val else np.zeros(0, np.float32)
    days = visit_days(rng, subj_ptr)
    coh = Cohort(K=K, J=J, subj_ptr=subj_ptr, row_ptr=row_ptr, col=col, val=val, days=days)
    return coh, PlantedModel(H=H, V=V, W=W, Q=Qs)


def init_factors(K, J, R, seed):
    """Seeded initial point shared by every implementation: H0 = I_R, W0 = 1, V0 ~ U[0,1).
    Values are rounded to float32 first so that FP32 and FP64 consumers start from the same point."""
    rng = np.random.default_rng(seed)
    H0 = np.eye(R)
    W0 = np.ones((K, R))
    V0 = rng.random((J, R)).astype(np.float32).astype(np.float64)
    return H0, W0, V0


def subset_subjects(coh: Cohort, idx) -> Cohort:
    """Cohort made of the listed subjects (in that order)."""
    idx = np.asarray(idx, dtype=np.int64)
    ik = coh.subj_ptr[idx + 1] - coh.subj_ptr[idx]
    subj_ptr = np.zeros(idx.size + 1, dtype=np.int64)
    np.cumsum(ik, out=subj_ptr[1:])
    rows = np.concatenate([np.arange(coh.subj_ptr[k], coh.subj_ptr[k + 1]) for k in idx]) \
        if idx.size else np.zeros(0, np.int64)
    rl = coh.row_ptr[rows + 1] - coh.row_ptr[rows]
    row_ptr = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(rl, out=row_ptr[1:])
    nz = np.concatenate([np.arange(coh.row_ptr[r], coh.row_ptr[r + 1]) for r in rows]) \
        if rows.size else np.zeros(0, np.int64)
    return Cohort(K=int(idx.size), J=coh.J, subj_ptr=subj_ptr, row_ptr=row_ptr,
                  col=coh.col[nz].copy(), val=coh.val[nz].copy(), days=coh.days[rows].copy())


# Workload recipes. Options common to the fit: l1 (lambda=0.1) on V, nonnegativity on W,
# unconstrained H, 5 inner ADMM steps; ``l`` = spline basis functions per subject (0 = none).
CONFIGS = {
    "c1": dict(name="planted K=200 J=100 R=5 I_k~U[5,40]", K=200, J=100, R=5, l=7, outer=10,
               inner=5, seed=1001),
    "c2": dict(name="EHR K=50000 J=1000 R=10 I_k~LN(20,1)<=500 7nnz/row", K=50_000, J=1000, R=10,
               l=7, outer=20, inner=5, seed=1002, ik=("ln", 20, 1.0, 1, 500), nnz=7, zipf=1.1),
    "c3": dict(name="EHR K=250000 J=1400 I_k~LN(25,1.2)<=850 1nnz/row", K=250_000, J=1400, R=15,
               l=7, outer=20, inner=5, seed=1003, ik=("ln", 25, 1.2, 3, 850), nnz=1, zipf=1.1),
    "c4": dict(name="EHR K=800000 J=300 R=20 I_k~LN(40,1.3)<=1500 1+Poi(0.105)nnz/row",
               K=800_000, J=300, R=20, l=7, outer=20, inner=5, seed=1004,
               ik=("ln", 40, 1.3, 1, 1500), nnz="1+poi0.105", zipf=1.0),
    "c5": dict(name="EHR K=20000 J=500 R=10 I_k~U[3,200] 6nnz/row", K=20_000, J=500, R=10, l=0,
               outer=0, inner=5, seed=1005, ik=("u", 3, 200), nnz=6, zipf=1.1),
}


def make_config(name, K=None):
    """Cohort for one of the recipes above; ``K`` (optional) keeps only the first K subjects'
    worth of draws by generating a cohort of that size with the same recipe and seed."""
    cfg = dict(CONFIGS[name])
    K = cfg["K"] if K is None else int(K)
    if name == "c1":
        coh, planted = planted_cohort(K, cfg["J"], cfg["R"], 5, 40, cfg["seed"])
        return coh, cfg
    rng = np.random.default_rng(cfg["seed"] + 7919)
    law = cfg["ik"]
    if law[0] == "ln":
        ik = _lognormal_visits(rng, K, law[1], law[2], law[3], law[4])
    else:
        ik = rng.integers(law[1], law[2] + 1, size=K).astype(np.int64)
    nnz = cfg["nnz"]
    if nnz == "1+poi0.105":
        nnz = lambda r, S: 1 + r.poisson(0.105, size=S)  # noqa: E731
    coh = ehr_cohort(K, cfg["J"], ik, nnz, cfg["zipf"], cfg["seed"])
    return coh, cfg
