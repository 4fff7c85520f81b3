"""CPU oracle for the semiring sparse contraction -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product path (the HIP library and its binding) never
imports, links or calls anything here, and this package imports nothing from
the product.  The heavy loops live in plain C (``oracle.c``, built with gcc
and OpenMP); this module marshals numpy arrays to it and holds the few
numpy-level definitions (mode folding of tensor keys).

Semiring names: ``plus_times``, ``min_plus``, ``or_and``, ``max_times``.
Value types: ``f64``, ``f32``, ``i32``, ``bool`` (uint8 0/1).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SEMIRINGS = {"plus_times": 0, "min_plus": 1, "or_and": 2, "max_times": 3}
DTYPES = {"f64": 0, "f32": 1, "i32": 2, "bool": 3}
NP_DTYPES = {"f64": np.float64, "f32": np.float32, "i32": np.int32, "bool": np.uint8}

# Tropical additive identity on int32: half of INT_MAX (Section 3.1).
INT_INF = (2 ** 31 - 1) // 2


def default_add_id(semiring: str, dtype: str):
    """Additive identity used when the caller gives none (Section 3.1 for
    (+,x) and (min,+) int; +inf for float (min,+); 0 for (max,x) on the
    non-negative domain; false for (or,and))."""
    if semiring == "plus_times":
        return 0.0
    if semiring == "min_plus":
        return INT_INF if dtype == "i32" else float("inf")
    if semiring == "max_times":
        return 0.0
    return 0


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` to ``liboracle.so`` with gcc (-O2, OpenMP,
    no floating-point contraction so the error-free transformations stay
    exact)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-shared", "-fPIC", _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        L.orc_num_threads.restype = I
        L.orc_set_threads.argtypes = [I]
        L.orc_fold.argtypes = [I, I, P, I64, P, P, P, I64, P, P, P, P]
        L.orc_spgemm_rows.argtypes = [I, I, I, P, I64, P, P, P, P, P, P, P, P, P, P, I64, P, P, P, P]
        L.orc_spmm.argtypes = [I, I, P, I64, I64, P, P, P, P, I, P, P]
        L.orc_bellman_ford.argtypes = [I, I, P, I64, I64, P, P, P, P, I64, P]
        L.orc_bfs.argtypes = [I64, P, P, P, I64, P]
        L.orc_dijkstra.argtypes = [I64, P, P, P, P, I64, I64, P]
        L.orc_floyd_warshall.argtypes = [I64, P, I64]
        L.orc_apsp_tiskin.argtypes = [I64, P, P, P, I64, P, P, P, P]
        for f in ("orc_fold", "orc_spgemm_rows", "orc_spmm", "orc_bellman_ford", "orc_bfs",
                  "orc_dijkstra", "orc_floyd_warshall", "orc_apsp_tiskin"):
            getattr(L, f).restype = I
        _lib = L
    return _lib


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _id_buf(semiring, dtype, add_id):
    if add_id is None:
        add_id = default_add_id(semiring, dtype)
    return np.array([add_id], dtype=NP_DTYPES[dtype])


class CSR:
    """Host CSR matrix: int64 rowptr, int32 col, values (numpy)."""

    def __init__(self, rowptr, col, val, nrows, ncols):
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val)
        self.nrows = int(nrows)
        self.ncols = int(ncols)

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def row(self, i):
        a, b = self.rowptr[i], self.rowptr[i + 1]
        return self.col[a:b], self.val[a:b]


def fold(semiring, dtype, rows, cols, vals, nrows, ncols, add_id=None) -> CSR:
    """Index-value pairs -> CSR: stable sort by (row, col), duplicates
    combined with the additive operator in input order, identity entries
    dropped (Section 3.2 index-value pairs; readings in ``oracle.c``)."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=NP_DTYPES[dtype])
    nnz = rows.size
    rp = np.zeros(nrows + 1, dtype=np.int64)
    oc = np.zeros(max(nnz, 1), dtype=np.int32)
    ov = np.zeros(max(nnz, 1), dtype=NP_DTYPES[dtype])
    on = np.zeros(1, dtype=np.int64)
    idb = _id_buf(semiring, dtype, add_id)
    rc = lib().orc_fold(SEMIRINGS[semiring], DTYPES[dtype], _p(idb), nnz, _p(rows), _p(cols),
                        _p(vals), nrows, _p(rp), _p(oc), _p(ov), _p(on))
    if rc != 0:
        raise MemoryError("oracle fold failed")
    k = int(on[0])
    return CSR(rp, oc[:k].copy(), ov[:k].copy(), nrows, ncols)


def mode_split(keys, dims):
    """Per-mode indices of linearized keys (last mode fastest)."""
    keys = np.asarray(keys, dtype=np.int64)
    out = []
    rem = keys.copy()
    for d in reversed(dims):
        out.append(rem % d)
        rem //= d
    return list(reversed(out))


def linearize(idx_list, dims):
    """Linear key of per-mode indices (last mode fastest)."""
    key = np.zeros_like(idx_list[0]) if idx_list else np.zeros(0, dtype=np.int64)
    for i, d in zip(idx_list, dims):
        key = key * d + i
    return key


def fold_tensor(semiring, dtype, keys, vals, dims, idx, row_idx, col_idx, add_id=None) -> CSR:
    """Fold an order-d COO tensor to a matrix: rows linearize the modes named
    by ``row_idx`` (in that order), columns those named by ``col_idx``.  A
    contraction maps three groups of indices onto the three indices of a
    matrix product (Section 5.1)."""
    modes = mode_split(keys, dims)
    pos = {c: t for t, c in enumerate(idx)}
    rdims = [dims[pos[c]] for c in row_idx]
    cdims = [dims[pos[c]] for c in col_idx]
    rows = linearize([modes[pos[c]] for c in row_idx], rdims)
    cols = linearize([modes[pos[c]] for c in col_idx], cdims)
    return fold(semiring, dtype, rows, cols, vals, int(np.prod(rdims, dtype=np.int64)),
                int(np.prod(cdims, dtype=np.int64)), add_id)


def spgemm(semiring, dtype, A: CSR, B: CSR, add_id=None, rows=None, C_old: CSR = None,
           threads=None):
    """Rows of C = A (x) B [(+) C_old] by the contraction's definition.

    Returns a CSR over the selected rows (``rows`` = None means all rows, in
    order).  (+,x) values are fp64 (Dot2 accumulation); other semirings keep
    the stored type.
    """
    if threads:
        set_threads(threads)
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    sel = np.arange(A.nrows, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    idb = _id_buf(semiring, dtype, add_id)
    sr, dt = SEMIRINGS[semiring], DTYPES[dtype]
    counts = np.zeros(max(sel.size, 1), dtype=np.int64)
    va = np.ascontiguousarray(A.val, dtype=NP_DTYPES[dtype])
    vb = np.ascontiguousarray(B.val, dtype=NP_DTYPES[dtype])
    rc_ = cc_ = vc_ = None
    if C_old is not None:
        rc_, cc_ = C_old.rowptr, C_old.col
        vc_ = np.ascontiguousarray(C_old.val, dtype=NP_DTYPES[dtype])
    L = lib()
    args = (sr, dt, _p(idb), B.ncols, _p(A.rowptr), _p(A.col), _p(va), _p(B.rowptr), _p(B.col),
            _p(vb), _p(rc_), _p(cc_), _p(vc_), _p(sel), sel.size)
    if L.orc_spgemm_rows(0, *args, _p(counts), None, None, None) != 0:
        raise MemoryError("oracle spgemm failed")
    counts = counts[: sel.size]
    rp = np.zeros(sel.size + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    total = int(rp[-1])
    oc = np.zeros(max(total, 1), dtype=np.int32)
    odt = np.float64 if semiring == "plus_times" else NP_DTYPES[dtype]
    ov = np.zeros(max(total, 1), dtype=odt)
    offs = np.ascontiguousarray(rp[:-1])
    if L.orc_spgemm_rows(1, *args, None, _p(offs), _p(oc), _p(ov)) != 0:
        raise MemoryError("oracle spgemm failed")
    return CSR(rp, oc[:total], ov[:total], sel.size, B.ncols)


def dense_plus_times(A, B):
    """Dense (+,x) product C = A B in fp64: the contraction's definition
    over full operands (the dense case of Section 3.3.1), one library matmul."""
    return np.asarray(A, dtype=np.float64) @ np.asarray(B, dtype=np.float64)


def spgemm_masked(semiring, dtype, A: CSR, B: CSR, M: CSR, add_id=None) -> CSR:
    """C = M (.) (A (x) B): the entries of the product whose position is in
    M's pattern (an output with predefined sparsity, Sections 1 and 7);
    M's values are ignored.  The full product by its definition, then the
    positions outside M removed."""
    if M.nrows != A.nrows or M.ncols != B.ncols:
        raise ValueError("mask shape")
    C = spgemm(semiring, dtype, A, B, add_id=add_id)
    crow = np.repeat(np.arange(C.nrows, dtype=np.int64), np.diff(C.rowptr))
    mrow = np.repeat(np.arange(M.nrows, dtype=np.int64), np.diff(M.rowptr))
    keep = np.isin(crow * C.ncols + C.col.astype(np.int64), mrow * M.ncols + M.col.astype(np.int64))
    rp = np.zeros(C.nrows + 1, dtype=np.int64)
    np.cumsum(np.bincount(crow[keep], minlength=C.nrows), out=rp[1:])
    return CSR(rp, C.col[keep], C.val[keep], C.nrows, C.ncols)


def spmm(semiring, dtype, A: CSR, X, add_id=None, self_term=False):
    """Y = [X (+)] A (x) X for dense row-major X (n x s).  Returns (Y, changed).
    (+,x) gives fp64; other semirings keep the stored type."""
    X = np.ascontiguousarray(X, dtype=NP_DTYPES[dtype])
    s = X.shape[1] if X.ndim == 2 else 1
    odt = np.float64 if semiring == "plus_times" else NP_DTYPES[dtype]
    Y = np.zeros((A.nrows, s), dtype=odt)
    ch = np.zeros(1, dtype=np.int32)
    idb = _id_buf(semiring, dtype, add_id)
    va = np.ascontiguousarray(A.val, dtype=NP_DTYPES[dtype])
    lib().orc_spmm(SEMIRINGS[semiring], DTYPES[dtype], _p(idb), A.nrows, s, _p(A.rowptr),
                   _p(A.col), _p(va), _p(X), int(self_term), _p(Y), _p(ch))
    return Y, bool(ch[0])


def bellman_ford(semiring, dtype, A: CSR, P0, add_id=None, max_iters=None):
    """Bellman-Ford fixpoint P <- P (+) A (x) P (Section 4.2).
    Returns (P, iterations, converged)."""
    P = np.array(P0, dtype=NP_DTYPES[dtype], copy=True, order="C")
    if P.ndim == 1:
        P = P[:, None]
    n, s = P.shape
    if max_iters is None:
        max_iters = n
    it = np.zeros(1, dtype=np.int64)
    idb = _id_buf(semiring, dtype, add_id)
    va = np.ascontiguousarray(A.val, dtype=NP_DTYPES[dtype])
    rc = lib().orc_bellman_ford(SEMIRINGS[semiring], DTYPES[dtype], _p(idb), n, s, _p(A.rowptr),
                                _p(A.col), _p(va), _p(P), int(max_iters), _p(it))
    if rc < 0:
        raise ValueError("oracle bellman-ford failed")
    return P, int(it[0]), rc == 0


def bfs_levels(A: CSR, sources):
    """Queue BFS levels over edges j -> i (A[i][j] stored); -1 = unreachable."""
    src = np.ascontiguousarray(sources, dtype=np.int64)
    lev = np.zeros((A.nrows, src.size), dtype=np.int32)
    lib().orc_bfs(A.nrows, _p(A.rowptr), _p(A.col), _p(src), src.size, _p(lev))
    return lev


def dijkstra(A: CSR, sources, inf_value=INT_INF):
    """Dijkstra distances (int64) from each source; unreachable = inf_value."""
    src = np.ascontiguousarray(sources, dtype=np.int64)
    w = np.ascontiguousarray(A.val, dtype=np.int32)
    d = np.zeros((A.nrows, src.size), dtype=np.int64)
    lib().orc_dijkstra(A.nrows, _p(A.rowptr), _p(A.col), _p(w), _p(src), src.size,
                       int(inf_value), _p(d))
    return d


def floyd_warshall(D, inf_value=INT_INF):
    """All-pairs distances from a dense n x n matrix (D[i][j] = w(j -> i))."""
    D = np.array(D, dtype=np.int64, copy=True, order="C")
    lib().orc_floyd_warshall(D.shape[0], _p(D), int(inf_value))
    return D


def apsp_tiskin(A: CSR, inf_value=INT_INF):
    """Tiskin's path doubling over (weight, hops) paths (Section 4.2): P
    starts as I (+) A with every edge a 1-hop path; round l = 1, 2, 4, ...
    (l < n) forms P <- P (+) P_l (x) P with P_l the paths of exactly l hops.
    Equal weights keep the path with fewer hops.  Returns (D, H, rounds,
    pl_nnz): D[i, j] = weight of the lightest path j -> i (inf_value where
    none), H = its hops (-1 where none), rounds = rounds whose P_l had
    entries, pl_nnz = entries of P_l per round of the loop."""
    n = int(A.nrows)
    w = np.ascontiguousarray(A.val, dtype=np.int32)
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    D = np.zeros((n, n), dtype=np.int64)
    H = np.zeros((n, n), dtype=np.int64)
    r = np.zeros(1, dtype=np.int32)
    pl = np.zeros(64, dtype=np.int64)
    rc = lib().orc_apsp_tiskin(n, _p(rp), _p(col), _p(w), int(inf_value), _p(D), _p(H), _p(r), _p(pl))
    if rc < 0:
        raise ValueError("negative edge weight")
    nr = 0
    l = 1
    while l < n:
        nr += 1
        l <<= 1
    return D, H, int(r[0]), pl[:nr].tolist()


def path_product(Aw, Ah, Bw, Bh, inf_value=INT_INF):
    """Dense product over (weight, hops) paths: C[i, j] = the lightest of
    A[i, k] (x) B[k, j] (weights and hops added), fewer hops on equal
    weights; operand entries with weight >= inf_value are absent, and so are
    products that reach it.  Returns (Cw, Ch): inf_value / -1 where none."""
    Aw = np.asarray(Aw, dtype=np.int64)
    Ah = np.asarray(Ah, dtype=np.int64)
    Bw = np.asarray(Bw, dtype=np.int64)
    Bh = np.asarray(Bh, dtype=np.int64)
    m, kk = Aw.shape
    n = Bw.shape[1]
    Cw = np.full((m, n), inf_value, dtype=np.int64)
    Ch = np.full((m, n), -1, dtype=np.int64)
    for k in range(kk):
        a_ok = Aw[:, k] < inf_value
        b_ok = Bw[k, :] < inf_value
        cw = Aw[:, k][:, None] + Bw[k, :][None, :]
        ch = Ah[:, k][:, None] + Bh[k, :][None, :]
        ok = a_ok[:, None] & b_ok[None, :] & (cw < inf_value)
        better = ok & ((cw < Cw) | ((cw == Cw) & (ch < Ch)))
        Cw = np.where(better, cw, Cw)
        Ch = np.where(better, ch, Ch)
    return Cw, Ch


_NP_SEMIRING = {
    # (multiply, add reduction) of each semiring over numpy arrays
    "plus_times": (np.multiply, np.add.reduce),
    "min_plus": (np.add, np.minimum.reduce),
    "or_and": (np.bitwise_and, np.bitwise_or.reduce),
    "max_times": (np.multiply, np.maximum.reduce),
}


def contract(semiring, dtype, ia: str, A, ib: str, B, ic: str, add_id=None):
    """C[ic] = (+) over the letters not in ic of A[ia] (x) B[ib], written out
    on dense operands (Section 3.3.1): both operands are broadcast over every
    letter and the letters outside C are reduced.  Entries equal to the
    additive identity are absent (their products are the identity).  (+,x)
    runs in fp64 with numpy's einsum (the same sum of products); (min,+)
    int32 sums in int64 and clamps results at the identity (Section 3.1).
    Returns a dense array in C's letter order."""
    A = np.asarray(A)
    B = np.asarray(B)
    if semiring == "plus_times":
        return np.einsum(f"{ia},{ib}->{ic}", A.astype(np.float64), B.astype(np.float64))
    ident = default_add_id(semiring, dtype) if add_id is None else add_id
    extra = []
    for ch in ia + ib:
        if ch not in ic and ch not in extra:
            extra.append(ch)
    full = ic + "".join(extra)
    ext = {}
    for s_, T in ((ia, A), (ib, B)):
        for ch, e in zip(s_, T.shape):
            ext[ch] = e

    def spread(T, idx):
        # T's axes moved to their places in `full`, size 1 elsewhere
        T = np.transpose(T, [idx.index(ch) for ch in full if ch in idx])
        return T.reshape([ext[ch] if ch in idx else 1 for ch in full])

    mul, red = _NP_SEMIRING[semiring]
    wide = np.int64 if dtype == "i32" else NP_DTYPES[dtype]
    a = spread(A, ia).astype(wide)
    b = spread(B, ib).astype(wide)
    absent = (spread(A, ia) == ident) | (spread(B, ib) == ident)
    if semiring == "min_plus" and dtype == "i32":
        p = np.minimum(mul(a, b), ident)
    else:
        p = mul(a, b)
    p = np.where(absent, np.asarray(ident, dtype=p.dtype), p)
    p = np.broadcast_to(p, [ext[ch] for ch in full])
    axes = tuple(range(len(ic), len(full)))
    out = red(p, axis=axes) if axes else np.array(p)
    if semiring == "min_plus" and dtype == "i32":
        out = np.minimum(out, ident)
    return out.astype(NP_DTYPES[dtype])


def jacobi(A: CSR, b, x0, tol, max_iters=10000, dtype="f64"):
    """Jacobi iteration for A x = b (Section 4.1, the listing read as
    intended: the row sum skips the diagonal and the residual is b - A x):
    x^{l+1} = (b - (A - diag) x^l) / diag, stored in the value type, until
    |b - A x^l|_2 <= tol for some l >= 1.  Returns (x^l, l, |r|, converged);
    without convergence x^max_iters and its residual."""
    npt = NP_DTYPES[dtype]
    b = np.asarray(b, dtype=npt)
    x = np.array(x0, dtype=npt, copy=True)
    n = A.nrows
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    d = np.zeros(n, dtype=np.float64)
    np.add.at(d, rows[A.col == rows], np.asarray(A.val, dtype=np.float64)[A.col == rows])
    if np.any(d == 0):
        raise ValueError("a row has no nonzero diagonal entry")
    for l in range(1, max_iters + 1):
        Ax, _ = spmm("plus_times", dtype, A, x[:, None])
        s = Ax[:, 0] - d * x.astype(np.float64)
        x = ((b.astype(np.float64) - s) / d).astype(npt)
        Ax, _ = spmm("plus_times", dtype, A, x[:, None])
        r = float(np.sqrt(np.sum((b.astype(np.float64) - Ax[:, 0]) ** 2)))
        if r <= tol:
            return x, l, r, True
    return x, max_iters, r, False


TRANSFORMS = ("recip", "scale", "add", "fma", "div_sum")


def transform(op, alpha, ia, A, ib, B, ic, C):
    """Elementwise transform of dense C (returns the new C): recip c =
    alpha / c, scale c = alpha c, add c = c + alpha a, fma c = c + alpha a b,
    div_sum c = c / (a + b), with a = A[ia] and b = B[ib] read at C's letters
    (broadcast along letters they lack), Section 3.4."""
    C = np.array(C, copy=True)

    def at_c(T, idx):
        T = np.asarray(T)
        T = np.transpose(T, [idx.index(ch) for ch in ic if ch in idx])
        return T.reshape([C.shape[q] if ch in idx else 1 for q, ch in enumerate(ic)])

    if op == "recip":
        return (C.dtype.type(alpha) / C).astype(C.dtype)
    if op == "scale":
        return (C.dtype.type(alpha) * C).astype(C.dtype)
    a = at_c(A, ia).astype(C.dtype)
    if op == "add":
        return (C + C.dtype.type(alpha) * a).astype(C.dtype)
    b = at_c(B, ib).astype(C.dtype)
    if op == "fma":
        return (C + C.dtype.type(alpha) * a * b).astype(C.dtype)
    return (C / (a + b)).astype(C.dtype)


def _bit_length(x):
    """Bit length of non-negative integers (0 for 0): floor(log2 x) + 1."""
    x = np.asarray(x, dtype=np.int64)
    _, e = np.frexp(x.astype(np.float64))  # x = f 2^e with 0.5 <= f < 1, exact below 2^53
    return np.where(x > 0, e, 0).astype(np.int64)


def features(semiring, A: CSR, B: CSR):
    """The 32 schedule features of the product A (x) B, from their
    definitions (the inputs of the schedule choice; Section 5.1 picks among
    mappings with performance models driven by sizes and nonzero counts).
    With m rows and w_i = sum over the entries (i, k) of A of the length of
    B's row k (the products of row i):
      0..9    fraction of rows of A whose length has bit length b (b >= 9: 9)
      10..19  fraction of rows with (bit length of w_i + 1) // 2 = b (w_i = 0:
              bin 0; b >= 9: 19)
      20..23  log2(m + 1), log2(columns of B + 1), log2(nnz(A) + 1),
              log2(sum w + 1)
      24      log2 of sum w / sum outputs over the rows floor(t m / s),
              t < s = min(512, m); an output is a distinct column reached
              from the row (by structure); 1 if no output was sampled
      25, 26  log2(max w + 1), log2(longest row of A + 1)
      27      population standard deviation of w over its mean (0 if the
              mean is 0)
      28..31  one-hot of the semiring.
    Returns float32[32]."""
    out = np.zeros(32, dtype=np.float32)
    m = A.nrows
    mm = float(max(m, 1))
    nz = np.diff(A.rowptr).astype(np.int64)
    blen = np.diff(B.rowptr).astype(np.int64)
    w = np.zeros(m, dtype=np.int64)
    if A.nnz:
        np.add.at(w, np.repeat(np.arange(m, dtype=np.int64), nz), blen[A.col[:A.nnz]])
    bn = np.minimum(9, _bit_length(nz))
    bw = np.where(w == 0, 0, np.minimum(9, (_bit_length(w) + 1) // 2))
    for b in range(10):
        out[b] = np.float32(int(np.count_nonzero(bn == b)) / mm)
        out[10 + b] = np.float32(int(np.count_nonzero(bw == b)) / mm)
    ns = min(512, m)
    cr = 1.0
    if ns > 0 and A.nnz > 0 and B.nnz > 0:
        sw_s, sn_s = 0, 0
        for t in range(ns):
            i = (t * m) // ns
            ks = A.col[A.rowptr[i]:A.rowptr[i + 1]]
            cols = [B.col[B.rowptr[k]:B.rowptr[k + 1]] for k in ks]
            sw_s += int(w[i])
            if cols:
                sn_s += int(np.unique(np.concatenate(cols)).size)
        if sn_s > 0:
            cr = sw_s / sn_s
    sw = int(w.sum())
    sq = int(np.sum(w.astype(object) * w.astype(object))) if m else 0
    mean = sw / mm
    var = max(0.0, float(sq) / mm - mean * mean)
    out[20] = np.float32(np.log2(m + 1.0))
    out[21] = np.float32(np.log2(B.ncols + 1.0))
    out[22] = np.float32(np.log2(A.nnz + 1.0))
    out[23] = np.float32(np.log2(sw + 1.0))
    out[24] = np.float32(np.log2(cr))
    out[25] = np.float32(np.log2(float(w.max() if m else 0) + 1.0))
    out[26] = np.float32(np.log2(float(nz.max() if m else 0) + 1.0))
    out[27] = np.float32(np.sqrt(var) / mean if mean > 0 else 0.0)
    out[28 + SEMIRINGS[semiring]] = 1.0
    return out
