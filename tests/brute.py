"""Brute-force dense semiring products for tiny inputs (test helper).

Every matrix is a dense array plus a presence mask; an absent entry takes no
part in the additive reduction.  The O(n^3) form is evaluated with numpy
broadcasting, entirely independent of the oracle's sparse row loop.
"""

import numpy as np

INT_INF = (2 ** 31 - 1) // 2


def csr_to_dense(csr, fill, dtype):
    D = np.full((csr.nrows, csr.ncols), fill, dtype=dtype)
    M = np.zeros((csr.nrows, csr.ncols), dtype=bool)
    for i in range(csr.nrows):
        c, v = csr.row(i)
        D[i, c] = v
        M[i, c] = True
    return D, M


def dense_product(semiring, dtype, A, MA, B, MB):
    """Returns (C, MC): C_ij over all k with MA[i,k] and MB[k,j]."""
    P = MA[:, :, None] & MB[None, :, :]          # (i, k, j) term present
    MC = P.any(axis=1)
    if semiring == "plus_times":
        a = A.astype(np.float64)
        b = B.astype(np.float64)
        C = np.where(P, a[:, :, None] * b[None, :, :], 0.0).sum(axis=1)
        return C, MC
    if semiring == "min_plus":
        if dtype == "i32":
            t = A.astype(np.int64)[:, :, None] + B.astype(np.int64)[None, :, :]
            t = np.where(P, t, np.int64(INT_INF))
            C = np.minimum(t.min(axis=1, initial=INT_INF), INT_INF)
            return C, MC & (C < INT_INF)
        t = (A.astype(np.float32)[:, :, None] + B.astype(np.float32)[None, :, :])
        t = np.where(P, t, np.float32(np.inf))
        C = t.min(axis=1, initial=np.float32(np.inf))
        return C, MC & np.isfinite(C)
    if semiring == "max_times":
        t = A[:, :, None] * B[None, :, :]            # rounded in the stored type
        t = np.where(P, t, np.zeros((), dtype=t.dtype))
        C = t.max(axis=1, initial=np.zeros((), dtype=t.dtype))
        return C, MC & (C != 0)
    if semiring == "or_and":
        return P.any(axis=1).astype(np.uint8), MC
    raise ValueError(semiring)
