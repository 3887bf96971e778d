"""Small helpers shared by tests (no method arithmetic)."""
import numpy as np

from paper_1803_04572_amd import synth


def dense_cohort(Xks, J, days=None):
    """Cohort from a list of dense I_k x J matrices (exact zeros dropped)."""
    rows_c, rows_v, lens, ik = [], [], [], []
    for X in Xks:
        ik.append(X.shape[0])
        for row in X:
            nz = np.flatnonzero(row)
            rows_c.append(nz.astype(np.int32))
            rows_v.append(row[nz].astype(np.float32))
            lens.append(nz.size)
    subj_ptr = np.concatenate([[0], np.cumsum(ik)]).astype(np.int64)
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    if days is None:
        days = np.concatenate([np.arange(n) * 30.0 for n in ik])
    return synth.Cohort(K=len(Xks), J=J, subj_ptr=subj_ptr, row_ptr=row_ptr,
                        col=np.concatenate(rows_c), val=np.concatenate(rows_v), days=days)
