"""Pins for the CPU oracle: each check ties it to something other than its own
code -- brute force on tiny inputs, closed forms, library routines (scipy),
and invariants of the algebra.  CPU only."""

import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
from hypothesis import given, settings, strategies as st

import oracle
from gen import synth
from brute import INT_INF, csr_to_dense, dense_product

PAIRS = [("plus_times", "f64"), ("plus_times", "f32"), ("min_plus", "i32"),
         ("min_plus", "f32"), ("or_and", "bool"), ("max_times", "f32"),
         ("max_times", "f64")]


def rand_matrix(semiring, dtype, m, n, density, seed, tag):
    key = synth.stream_key(seed, tag)
    u = synth.uniform_f64(key, m * n)
    mask = u < density
    rows, cols = np.nonzero(mask.reshape(m, n))
    k = rows.size
    if dtype == "i32":
        vals = synth.randint(synth.stream_key(seed, tag + 1), k, -20, 100).astype(np.int32)
        if semiring == "min_plus":
            vals = np.abs(vals).astype(np.int32) + 1
    elif dtype == "bool":
        vals = np.ones(k, dtype=np.uint8)
    elif dtype == "f32":
        vals = synth.uniform_f32(synth.stream_key(seed, tag + 1), k) + np.float32(0.0625)
    else:
        vals = synth.uniform_f64(synth.stream_key(seed, tag + 1), k) + 0.0625
    return oracle.fold(semiring, dtype, rows, cols, vals, m, n)


def identity_fill(semiring, dtype):
    if semiring == "min_plus":
        return INT_INF if dtype == "i32" else np.inf
    return 0


@pytest.mark.parametrize("semiring,dtype", PAIRS)
@settings(max_examples=12, deadline=None)
@given(m=st.integers(0, 24), k=st.integers(0, 24), n=st.integers(0, 24),
       density=st.floats(0.0, 0.9), seed=st.integers(0, 2 ** 32))
def test_spgemm_matches_brute_force(semiring, dtype, m, k, n, density, seed):
    A = rand_matrix(semiring, dtype, m, k, density, seed, 1)
    B = rand_matrix(semiring, dtype, k, n, density, seed, 7)
    C = oracle.spgemm(semiring, dtype, A, B)
    npdt = oracle.NP_DTYPES[dtype]
    fill = identity_fill(semiring, dtype)
    DA, MA = csr_to_dense(A, fill, npdt)
    DB, MB = csr_to_dense(B, fill, npdt)
    DC, MC = dense_product(semiring, dtype, DA, MA, DB, MB)
    got = np.zeros((m, n), dtype=np.float64)
    gm = np.zeros((m, n), dtype=bool)
    for i in range(m):
        c, v = C.row(i)
        assert np.all(np.diff(c) > 0), "columns ascending"
        got[i, c] = v
        gm[i, c] = True
    assert np.array_equal(gm, MC)
    if semiring == "plus_times":
        np.testing.assert_allclose(got[MC], DC[MC], rtol=1e-14)
    else:
        assert np.array_equal(got[MC], DC[MC].astype(np.float64))


def test_fold_duplicates_and_identity():
    # brute force with a dict over a tiny COO list
    rows = np.array([2, 0, 2, 1, 2, 0, 1, 1])
    cols = np.array([1, 0, 1, 3, 1, 0, 0, 3])
    vals_f = np.array([1.0, 2.0, 4.0, 0.0, 8.0, -2.0, 5.0, 3.0])
    A = oracle.fold("plus_times", "f64", rows, cols, vals_f, 3, 4)
    # (0,0): 2 + -2 = 0 -> dropped; (1,3): 0 is absent, 3 kept; (2,1): 13
    assert A.rowptr.tolist() == [0, 0, 2, 3]
    assert A.col.tolist() == [0, 3, 1]
    assert A.val.tolist() == [5.0, 3.0, 13.0]
    vals_i = np.array([7, 3, 5, INT_INF, 9, 4, 1, 2], dtype=np.int32)
    T = oracle.fold("min_plus", "i32", rows, cols, vals_i, 3, 4)
    assert T.col.tolist() == [0, 0, 3, 1]
    assert T.val.tolist() == [3, 1, 2, 5]
    assert T.rowptr.tolist() == [0, 1, 3, 4]


def test_fold_matches_scipy_sum_duplicates():
    src, dst = synth.rmat_edges(10, 8, 0.57, 0.19, 0.19, seed=11)
    vals = synth.edge_values("i32", src.size, 11, lo=1, hi=9).astype(np.float64)
    A = oracle.fold("plus_times", "f64", dst, src, vals, 1024, 1024)
    S = sp.coo_matrix((vals, (dst, src)), shape=(1024, 1024)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    assert np.array_equal(A.rowptr, S.indptr)
    assert np.array_equal(A.col, S.indices)
    assert np.array_equal(A.val, S.data)   # small integers: sums are exact


def test_fold_tensor_modes():
    dims = (5, 6, 7)
    keys = synth.bernoulli_keys(dims, 0.2, seed=3)
    vals = synth.uniform_f32(synth.stream_key(3, 1), keys.size)
    F = oracle.fold_tensor("plus_times", "f32", keys, vals, dims, "ijk", "ki", "j")
    i, j, k = np.unravel_index(keys, dims)
    D = np.zeros((7 * 5, 6), dtype=np.float32)
    D[k * 5 + i, j] = vals
    G = np.zeros_like(D)
    for r in range(F.nrows):
        c, v = F.row(r)
        G[r, c] = v
    assert np.array_equal(D, G)


def test_plus_times_matches_scipy_and_dot2():
    src, dst = synth.er_edges(300, 6, seed=5)
    v = synth.uniform_f64(synth.stream_key(5, 9), src.size)
    A = oracle.fold("plus_times", "f64", dst, src, v, 300, 300)
    C = oracle.spgemm("plus_times", "f64", A, A)
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(300, 300))
    R = (S @ S).tocsr()
    R.sort_indices()
    R.eliminate_zeros()
    assert np.array_equal(C.rowptr, R.indptr) and np.array_equal(C.col, R.indices)
    np.testing.assert_allclose(C.val, R.data, rtol=1e-13)
    # Dot2: 1e16 + 1 - 1e16 is 1 exactly, which plain fp64 summation loses
    A1 = oracle.fold("plus_times", "f64", [0, 0, 0], [0, 1, 2], [1e16, 1.0, -1e16], 1, 3)
    B1 = oracle.fold("plus_times", "f64", [0, 1, 2], [0, 0, 0], [1.0, 1.0, 1.0], 3, 1)
    assert oracle.spgemm("plus_times", "f64", A1, B1).val.tolist() == [1.0]


def path_graph(n, w):
    src = np.arange(n - 1)
    dst = src + 1
    return oracle.fold("min_plus", "i32", dst, src, w, n, n)


def test_path_graph_closed_forms():
    n = 40
    w = synth.randint(synth.stream_key(9, 1), n - 1, 1, 100).astype(np.int32)
    A = path_graph(n, w)
    C = oracle.spgemm("min_plus", "i32", A, A)
    # (A (x) A)[i+2, i] = w_i + w_{i+1}; nothing else
    assert C.nnz == n - 2
    for i in range(n - 2):
        c, v = C.row(i + 2)
        assert c.tolist() == [i] and v.tolist() == [w[i] + w[i + 1]]
    P0 = np.full((n, 1), INT_INF, dtype=np.int32)
    P0[0, 0] = 0
    P, iters, conv = oracle.bellman_ford("min_plus", "i32", A, P0)
    assert conv and iters == n          # n-1 relaxations plus one unchanged step
    assert np.array_equal(P[:, 0], np.concatenate([[0], np.cumsum(w)]))
    lev = oracle.bfs_levels(A, [0])
    assert np.array_equal(lev[:, 0], np.arange(n))
    # boolean A^k is a shift by k
    Ab = oracle.fold("or_and", "bool", np.arange(1, n), np.arange(n - 1), np.ones(n - 1, np.uint8), n, n)
    Pk = Ab
    for k in range(2, 6):
        Pk = oracle.spgemm("or_and", "bool", Pk, Ab)
        assert Pk.nnz == n - k
        assert all(Pk.row(i + k)[0].tolist() == [i] for i in range(n - k))


def test_bf_not_converged_cap():
    n = 10
    A = path_graph(n, np.ones(n - 1, np.int32))
    P0 = np.full((n, 1), INT_INF, dtype=np.int32)
    P0[0, 0] = 0
    _, iters, conv = oracle.bellman_ford("min_plus", "i32", A, P0, max_iters=5)
    assert not conv and iters == 5


def test_star_closed_form():
    L = 50
    hub = np.zeros(L, dtype=np.int64)
    leaves = np.arange(1, L + 1)
    rows = np.concatenate([hub, leaves])
    cols = np.concatenate([leaves, hub])
    A = oracle.fold("plus_times", "f64", rows, cols, np.ones(2 * L), L + 1, L + 1)
    C = oracle.spgemm("plus_times", "f64", A, A)
    assert C.nnz == L * L + 1
    assert C.row(0)[0].tolist() == [0] and C.row(0)[1].tolist() == [float(L)]
    for i in range(1, L + 1):
        c, v = C.row(i)
        assert c.tolist() == list(range(1, L + 1)) and np.all(v == 1.0)
    T = oracle.fold("min_plus", "i32", rows, cols, np.ones(2 * L, np.int32), L + 1, L + 1)
    CT = oracle.spgemm("min_plus", "i32", T, T)
    assert CT.nnz == L * L + 1 and np.all(CT.val == 2)


@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_identity_matrix_is_neutral(semiring, dtype):
    A = rand_matrix(semiring, dtype, 30, 30, 0.2, 77, 3)
    one = {"plus_times": 1, "min_plus": 0, "or_and": 1, "max_times": 1}[semiring]
    I = oracle.fold(semiring, dtype, np.arange(30), np.arange(30),
                    np.full(30, one, dtype=oracle.NP_DTYPES[dtype]), 30, 30)
    for C in (oracle.spgemm(semiring, dtype, I, A), oracle.spgemm(semiring, dtype, A, I)):
        assert np.array_equal(C.rowptr, A.rowptr) and np.array_equal(C.col, A.col)
        assert np.array_equal(C.val.astype(np.float64), A.val.astype(np.float64))


def test_all_ones_square():
    n = 33
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    J = oracle.fold("plus_times", "f32", r.ravel(), c.ravel(), np.ones(n * n, np.float32), n, n)
    C = oracle.spgemm("plus_times", "f32", J, J)
    assert C.nnz == n * n and np.all(C.val == n)
    E = oracle.spgemm("plus_times", "f32", oracle.fold("plus_times", "f32", [], [], [], n, n), J)
    assert E.nnz == 0


def test_stencil27_square_closed_form():
    g = 7
    src, dst = synth.stencil27_edges(g)
    N = g ** 3
    A = oracle.fold("plus_times", "f64", dst, src, np.ones(src.size), N, N)
    C = oracle.spgemm("plus_times", "f64", A, A)
    cnt = {0: 3, 1: 2, 2: 1}
    ctr = (3 * g + 3) * g + 3          # interior point (3,3,3)
    c, v = C.row(ctr)
    assert c.size == 125
    for col, val in zip(c, v):
        x, y, z = col // (g * g), (col // g) % g, col % g
        assert val == cnt[abs(x - 3)] * cnt[abs(y - 3)] * cnt[abs(z - 3)]
    T = oracle.fold("min_plus", "i32", dst, src, np.ones(src.size, np.int32), N, N)
    assert np.all(oracle.spgemm("min_plus", "i32", T, T, rows=[ctr]).val[
        oracle.spgemm("min_plus", "i32", T, T, rows=[ctr]).col != ctr] == 2)
    lev = oracle.bfs_levels(T, [0])[:, 0]
    xs, ys, zs = np.unravel_index(np.arange(N), (g, g, g))
    assert np.array_equal(lev, np.maximum(np.maximum(xs, ys), zs))


def er_weighted(n, d, seed):
    src, dst = synth.er_edges(n, d, seed)
    w = synth.edge_values("i32", src.size, seed, lo=1, hi=100)
    return oracle.fold("min_plus", "i32", dst, src, w, n, n), src, dst, w


def test_apsp_floyd_warshall_equals_path_doubling_and_scipy():
    n = 64
    A, src, dst, w = er_weighted(n, 8, synth.SEED_CFG0)
    D = np.full((n, n), INT_INF, dtype=np.int64)
    D[A.rowptr.searchsorted(np.arange(A.nnz), side="right") - 1, A.col] = A.val
    np.fill_diagonal(D, 0)
    FW = oracle.floyd_warshall(D)
    # scipy: graph[u, v] = weight of u -> v, i.e. the transpose of D
    G = sp.csr_matrix((A.val.astype(np.float64), A.col,
                       A.rowptr), shape=(n, n)).T
    ref = csg.floyd_warshall(G, directed=True).T
    fin = np.isfinite(ref)
    assert np.array_equal(FW[fin], ref[fin].astype(np.int64)) and np.all(FW[~fin] == INT_INF)
    # path doubling: A <- A (+) A (x) A, ceil(log2 n) rounds, from I (+) A
    I = oracle.fold("min_plus", "i32", np.arange(n), np.arange(n), np.zeros(n, np.int32), n, n)
    P = oracle.spgemm("min_plus", "i32", I, I, C_old=A)   # (I (+) A)
    rounds = 0
    l = 1
    while l < n:
        P = oracle.spgemm("min_plus", "i32", P, P, C_old=P)
        l <<= 1
        rounds += 1
    assert rounds == 6
    Dp = np.full((n, n), INT_INF, dtype=np.int64)
    for i in range(n):
        c, v = P.row(i)
        Dp[i, c] = v
    assert np.array_equal(Dp, FW)


def test_sssp_bellman_ford_equals_dijkstra_and_scipy():
    n = 2000
    A, src, dst, w = er_weighted(n, 6, 17)
    sources = synth.pick_sources(n, src, 8, 17)
    P0 = np.full((n, sources.size), INT_INF, dtype=np.int32)
    P0[sources, np.arange(sources.size)] = 0
    P, iters, conv = oracle.bellman_ford("min_plus", "i32", A, P0)
    assert conv
    Dj = oracle.dijkstra(A, sources)
    assert np.array_equal(P.astype(np.int64), Dj)
    G = sp.csr_matrix((A.val.astype(np.float64), A.col, A.rowptr), shape=(n, n)).T.tocsr()
    ref = csg.dijkstra(G, directed=True, indices=sources).T
    fin = np.isfinite(ref)
    assert np.array_equal(Dj[fin], ref[fin].astype(np.int64)) and np.all(Dj[~fin] == INT_INF)
    # BFS levels vs scipy unweighted shortest paths
    lev = oracle.bfs_levels(A, sources)
    hop = csg.shortest_path(G, directed=True, unweighted=True, indices=sources).T
    fin = np.isfinite(hop)
    assert np.array_equal(lev[fin], hop[fin].astype(np.int32)) and np.all(lev[~fin] == -1)


def test_bf_iterates_are_hop_bounded_distances():
    # After r BSP steps P holds shortest distances over paths of <= r edges;
    # checked against Dijkstra on the layered (hop, vertex) graph.
    n, s = 300, 3
    A, src, dst, w = er_weighted(n, 3, 23)
    sources = synth.pick_sources(n, src, s, 23)
    P0 = np.full((n, s), INT_INF, dtype=np.int32)
    P0[sources, np.arange(s)] = 0
    for r in (1, 2, 3, 5):
        P, it, _ = oracle.bellman_ford("min_plus", "i32", A, P0, max_iters=r)
        # layered graph: node (h, v), edges (h, u) -> (h+1, v) weight w, (h, v) -> (h+1, v) weight 0
        L = r + 1
        rr, cc, ww = [], [], []
        rows_of = np.repeat(np.arange(n), np.diff(A.rowptr))
        for h in range(r):
            rr += list(h * n + A.col); cc += list((h + 1) * n + rows_of); ww += list(A.val)
            rr += list(h * n + np.arange(n)); cc += list((h + 1) * n + np.arange(n)); ww += [0] * n
        G = sp.csr_matrix((np.array(ww, float) + 1e-9, (rr, cc)), shape=(L * n, L * n))
        ref = csg.dijkstra(G, directed=True, indices=sources)[:, r * n:(r + 1) * n].T
        fin = np.isfinite(ref)
        assert np.array_equal(P[fin].astype(np.int64), np.rint(ref[fin]).astype(np.int64))
        assert np.all(P[~fin] == INT_INF)


def test_algebraic_invariants():
    for semiring, dtype in (("min_plus", "i32"), ("or_and", "bool")):
        A = rand_matrix(semiring, dtype, 20, 15, 0.2, 5, 1)
        B = rand_matrix(semiring, dtype, 15, 25, 0.2, 5, 3)
        C = rand_matrix(semiring, dtype, 25, 10, 0.2, 5, 5)
        L = oracle.spgemm(semiring, dtype, oracle.spgemm(semiring, dtype, A, B), C)
        R = oracle.spgemm(semiring, dtype, A, oracle.spgemm(semiring, dtype, B, C))
        assert np.array_equal(L.rowptr, R.rowptr) and np.array_equal(L.col, R.col)
        assert np.array_equal(L.val, R.val)

    def transpose(M, semiring, dtype):
        rows = np.repeat(np.arange(M.nrows), np.diff(M.rowptr))
        return oracle.fold(semiring, dtype, M.col, rows, M.val, M.ncols, M.nrows)

    for semiring, dtype in (("min_plus", "i32"), ("min_plus", "f32"), ("or_and", "bool"),
                            ("max_times", "f32")):
        A = rand_matrix(semiring, dtype, 20, 15, 0.3, 8, 1)
        B = rand_matrix(semiring, dtype, 15, 25, 0.3, 8, 3)
        L = transpose(oracle.spgemm(semiring, dtype, A, B), semiring, dtype)
        R = oracle.spgemm(semiring, dtype, transpose(B, semiring, dtype), transpose(A, semiring, dtype))
        assert np.array_equal(L.col, R.col) and np.array_equal(L.val, R.val)
    # same pattern across semirings for positive values
    src, dst = synth.er_edges(200, 5, 31)
    pats = []
    for semiring, dtype, v in (("or_and", "bool", np.ones(src.size, np.uint8)),
                               ("min_plus", "i32", np.ones(src.size, np.int32)),
                               ("plus_times", "f64", np.ones(src.size))):
        A = oracle.fold(semiring, dtype, dst, src, v, 200, 200)
        C = oracle.spgemm(semiring, dtype, A, A)
        pats.append((C.rowptr, C.col))
        prods = int(sum(np.diff(A.rowptr)[A.col]))
        assert C.nnz <= prods
    for p in pats[1:]:
        assert np.array_equal(p[0], pats[0][0]) and np.array_equal(p[1], pats[0][1])


@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_spmm_matches_brute_force(semiring, dtype):
    A = rand_matrix(semiring, dtype, 23, 19, 0.3, 41, 1)
    X = rand_matrix(semiring, dtype, 19, 5, 0.6, 41, 3)
    fill = identity_fill(semiring, dtype)
    npdt = oracle.NP_DTYPES[dtype]
    DX, MX = csr_to_dense(X, fill, npdt)
    Y, _ = oracle.spmm(semiring, dtype, A, DX)
    DA, MA = csr_to_dense(A, fill, npdt)
    DC, MC = dense_product(semiring, dtype, DA, MA, DX, MX)
    idv = fill if semiring != "or_and" else 0
    exp = np.where(MC, DC, idv)
    if semiring == "plus_times":
        np.testing.assert_allclose(Y, exp, rtol=1e-14)
    else:
        assert np.array_equal(Y.astype(np.float64), exp.astype(np.float64))


def test_mlp_oracle_gradient_matches_finite_differences():
    from oracle import mlp
    K = 8
    rng = np.random.default_rng(3)
    p = rng.normal(0, 0.3, mlp.num_params(K))
    X = rng.normal(0, 1, (7, 32))
    T = rng.normal(0, 1, (7, K))
    loss, g = mlp.loss_grad(p, X, T, K)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_grad(p + e, X, T, K)[0] - mlp.loss_grad(p - e, X, T, K)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9
    # a network with zero weights outputs its last bias exactly
    z = np.zeros(mlp.num_params(K))
    z[-K:] = np.arange(K)
    y, _ = mlp.forward(z, X, K)
    assert np.array_equal(y, np.tile(np.arange(K, dtype=float), (7, 1)))


def test_dense_plus_times_pins():
    # explicit triple loop on a small case, and the all-ones closed form
    a = synth.uniform_f64(synth.stream_key(31, 0), 5 * 7).reshape(5, 7)
    b = synth.uniform_f64(synth.stream_key(31, 1), 7 * 3).reshape(7, 3)
    ref = np.zeros((5, 3))
    for i in range(5):
        for j in range(3):
            for k in range(7):
                ref[i, j] += a[i, k] * b[k, j]
    assert np.allclose(oracle.dense_plus_times(a, b), ref, rtol=1e-15, atol=0)
    n = 37
    assert np.array_equal(oracle.dense_plus_times(np.ones((n, n)), np.ones((n, n))), np.full((n, n), float(n)))


@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_spgemm_masked_pins(semiring, dtype):
    # brute force with a dense mask; the identity pattern keeps the
    # diagonal; a mask covering the product changes nothing
    m, k, n = 23, 19, 21
    A = rand_matrix(semiring, dtype, m, k, 0.3, 77, 1)
    B = rand_matrix(semiring, dtype, k, n, 0.3, 77, 7)
    M = rand_matrix("or_and", "bool", m, n, 0.4, 77, 13)
    C = oracle.spgemm_masked(semiring, dtype, A, B, M)
    fill = identity_fill(semiring, dtype)
    npdt = oracle.NP_DTYPES[dtype]
    DA, MA = csr_to_dense(A, fill, npdt)
    DB, MB = csr_to_dense(B, fill, npdt)
    DC, MC = dense_product(semiring, dtype, DA, MA, DB, MB)
    _, MM = csr_to_dense(M, 0, np.uint8)
    want = MC & MM
    got = np.zeros((m, n), dtype=bool)
    for i in range(m):
        c, v = C.row(i)
        got[i, c] = True
        if semiring == "plus_times":
            np.testing.assert_allclose(v, DC[i, c], rtol=1e-14)
        else:
            assert np.array_equal(v.astype(np.float64), DC[i, c].astype(np.float64))
    assert np.array_equal(got, want)
    sq = rand_matrix(semiring, dtype, 30, 30, 0.2, 78, 1)
    I = oracle.fold("or_and", "bool", np.arange(30), np.arange(30), np.ones(30, np.uint8), 30, 30)
    full = oracle.spgemm(semiring, dtype, sq, sq)
    diag = oracle.spgemm_masked(semiring, dtype, sq, sq, I)
    for i in range(30):
        c, v = diag.row(i)
        fc, fv = full.row(i)
        assert c.tolist() == ([i] if i in fc.tolist() else [])
        if c.size:
            assert v[0] == fv[fc.tolist().index(i)]
    cover = oracle.fold("or_and", "bool", np.repeat(np.arange(30), 30), np.tile(np.arange(30), 30),
                        np.ones(900, np.uint8), 30, 30)
    again = oracle.spgemm_masked(semiring, dtype, sq, sq, cover)
    assert np.array_equal(again.rowptr, full.rowptr) and np.array_equal(again.col, full.col)
    assert np.array_equal(again.val, full.val)


# ------------------------------------------------- Tiskin path doubling --

def hop_layered_distances(A, n, inf=INT_INF):
    """Lightest path weights with at most h hops for h = 0 .. n-1 (textbook
    hop-bounded Bellman-Ford on a dense matrix; orientation as A)."""
    W = np.full((n, n), np.inf)
    for i in range(n):
        c, v = A.row(i)
        W[i, c] = np.minimum(W[i, c], v.astype(np.float64))
    Dh = np.full((n, n), np.inf)
    np.fill_diagonal(Dh, 0.0)
    layers = [Dh]
    for _ in range(1, max(n, 1)):
        Dh = np.minimum(Dh, (W[:, :, None] + Dh[None, :, :]).min(axis=1))
        layers.append(Dh)
    return layers


def min_hops_from_layers(layers, D):
    """H[i, j] = fewest hops of a lightest path = first layer reaching D."""
    n = D.shape[0]
    H = np.full((n, n), -1, dtype=np.int64)
    for h, L in enumerate(layers):
        hit = (H < 0) & np.isfinite(L) & (L == D)
        H[hit] = h
    return H


@pytest.mark.parametrize("n,d,lo,hi,seed", [(2, 1, 0, 5, 1), (17, 3, 0, 4, 2), (40, 4, 0, 3, 3), (64, 8, 1, 100, 4),
                                            (33, 0.5, 1, 9, 5)])
def test_tiskin_matches_scipy_and_fewest_hops(n, d, lo, hi, seed):
    src, dst = synth.er_edges(n, d, seed)
    w = synth.edge_values("i32", src.size, seed, lo=lo, hi=hi)
    A = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    D, H, rounds, pl = oracle.apsp_tiskin(A)
    G = sp.csr_matrix((A.val.astype(np.float64), A.col, A.rowptr), shape=(n, n)).T
    ref = csg.floyd_warshall(G, directed=True).T
    fin = np.isfinite(ref)
    assert np.array_equal(D[fin], ref[fin].astype(np.int64)) and np.all(D[~fin] == INT_INF)
    layers = hop_layered_distances(A, n)
    assert np.array_equal(np.where(fin, ref, np.inf), layers[-1])
    assert np.array_equal(H, min_hops_from_layers(layers, np.where(fin, ref, np.inf)))
    # rounds with entries are a prefix of the loop, and the last one
    # reaches the largest hop count
    assert all(x > 0 for x in pl[:rounds]) and all(x == 0 for x in pl[rounds:])
    if H.max() > 0:
        assert 1 << (rounds - 1) <= H.max() <= 1 << rounds


def test_tiskin_path_graph_closed_form():
    n = 37
    w = synth.randint(synth.stream_key(11, 1), n - 1, 1, 50).astype(np.int32)
    A = path_graph(n, w)
    D, H, rounds, pl = oracle.apsp_tiskin(A)
    cs = np.concatenate([[0], np.cumsum(w)])
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert np.array_equal(D, np.where(i >= j, cs[i] - cs[np.minimum(i, j)], INT_INF))
    assert np.array_equal(H, np.where(i >= j, i - j, -1))
    # round l keeps the n - l pairs exactly l hops apart
    assert pl == [n - (1 << r) for r in range(6)] and rounds == 6


def test_tiskin_ties_keep_fewer_hops_and_diagonal():
    # 0 -> 1 (5), 0 -> 2 (5), 2 -> 1 (0), 1 -> 3 (0), 3 -> 1 (0), 2 -> 2 (3),
    # 3 -> 0 (7); entry (i, j) = edge j -> i
    edges = [(0, 1, 5), (0, 2, 5), (2, 1, 0), (1, 3, 0), (3, 1, 0), (2, 2, 3), (3, 0, 7)]
    n = 4
    src = np.array([e[0] for e in edges])
    dst = np.array([e[1] for e in edges])
    w = np.array([e[2] for e in edges], dtype=np.int32)
    A = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    D, H, rounds, _ = oracle.apsp_tiskin(A)
    assert D[1, 0] == 5 and H[1, 0] == 1          # direct edge beats 0 -> 2 -> 1
    assert D[3, 0] == 5 and H[3, 0] == 2          # 0 -> 1 -> 3
    assert np.all(np.diag(D) == 0) and np.all(np.diag(H) == 0)   # closure of I (+) A
    assert D[0, 1] == 7 and H[0, 1] == 2          # 1 -> 3 -> 0
    assert D[0, 2] == 7 and H[0, 2] == 3          # 2 -> 1 -> 3 -> 0


def test_tiskin_degenerate_graphs():
    for n in (0, 1, 5):
        A = oracle.fold("min_plus", "i32", np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int32),
                        n, n)
        D, H, rounds, pl = oracle.apsp_tiskin(A)
        assert rounds == 0 and all(x == 0 for x in pl)
        assert np.array_equal(D, np.where(np.eye(n, dtype=bool), 0, INT_INF))
        assert np.array_equal(H, np.where(np.eye(n, dtype=bool), 0, -1))
    # complete graph of equal weights: every lightest path is one edge
    n = 9
    src, dst, _ = synth.dense_graph(n, 1)
    A = oracle.fold("min_plus", "i32", dst, src, np.full(src.size, 4, np.int32), n, n)
    D, H, rounds, pl = oracle.apsp_tiskin(A)
    assert rounds == 1 and pl[0] == n * (n - 1)
    assert np.array_equal(H, 1 - np.eye(n, dtype=np.int64)) and np.array_equal(D, 4 * H)
    with pytest.raises(ValueError):
        oracle.apsp_tiskin(oracle.fold("min_plus", "i32", np.array([1]), np.array([0]), np.array([-1], np.int32), 2, 2))


def test_tiskin_dense_workload_shape():
    n = 48
    src, dst, w = synth.dense_graph(n, 7)
    assert w.min() >= 1 and w.max() <= n * n and src.size == n * (n - 1)
    A = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    D, H, rounds, pl = oracle.apsp_tiskin(A)
    G = sp.csr_matrix((A.val.astype(np.float64), A.col, A.rowptr), shape=(n, n)).T
    assert np.array_equal(D, csg.floyd_warshall(G, directed=True).T.astype(np.int64))
    # the sparsified products do less work than dense doubling's n^3 per round
    assert pl[0] == n * (n - 1) and sum(pl) * n < rounds * n ** 3


def test_path_product_pins():
    inf = INT_INF
    # 1 x 1: a single product adds weights and hops
    Cw, Ch = oracle.path_product([[3]], [[2]], [[4]], [[5]])
    assert Cw.tolist() == [[7]] and Ch.tolist() == [[7]]
    # equal weights: fewer hops wins, whatever the order of k
    Cw, Ch = oracle.path_product([[2, 1]], [[4, 1]], [[3], [4]], [[0], [1]])
    assert Cw.tolist() == [[5]] and Ch.tolist() == [[2]]
    Cw, Ch = oracle.path_product([[1, 2]], [[1, 4]], [[4], [3]], [[1], [0]])
    assert Cw.tolist() == [[5]] and Ch.tolist() == [[2]]
    # absent operands and products that reach the identity are no path
    Cw, Ch = oracle.path_product([[inf, inf - 1]], [[0, 1]], [[1], [1]], [[1], [1]])
    assert Cw.tolist() == [[inf]] and Ch.tolist() == [[-1]]
    # with every hop count 0 the weights are the plain (min,+) product
    rng = np.random.default_rng(3)
    Aw = rng.integers(0, 50, (7, 5))
    Bw = rng.integers(0, 50, (5, 6))
    Cw, Ch = oracle.path_product(Aw, 0 * Aw, Bw, 0 * Bw)
    assert np.array_equal(Cw, (Aw[:, :, None] + Bw[None, :, :]).min(axis=1)) and np.all(Ch == 0)


# ------------------------------------------------------ tensor contraction --

def dense_of_csr(M: "oracle.CSR", fill):
    D = np.full((M.nrows, M.ncols), fill, dtype=np.asarray(M.val).dtype)
    for i in range(M.nrows):
        c, v = M.row(i)
        D[i, c] = v
    return D


@pytest.mark.parametrize("semiring,dtype", [("plus_times", "f64"), ("min_plus", "i32"), ("or_and", "bool"),
                                            ("max_times", "f64")])
def test_contract_matrix_case_matches_spgemm(semiring, dtype):
    # C["ij"] = A["ik"] B["kj"] is the matrix product of the oracle's SpGEMM
    A = rand_matrix(semiring, dtype, 13, 9, 0.3, 5, 1)
    B = rand_matrix(semiring, dtype, 9, 11, 0.3, 5, 2)
    fill = identity_fill(semiring, dtype)
    Ad, Bd = dense_of_csr(A, fill), dense_of_csr(B, fill)
    C = oracle.contract(semiring, dtype, "ik", Ad, "kj", Bd, "ij")
    ref = dense_of_csr(oracle.spgemm(semiring, dtype, A, B), fill)
    if semiring == "plus_times":
        assert np.allclose(C, ref, rtol=1e-14, atol=0)
    else:
        assert np.array_equal(C, ref)
    # letter order is notation only: the transposed form gives C^T
    Ct = oracle.contract(semiring, dtype, "kj", Bd, "ik", Ad, "ji")
    assert np.array_equal(Ct, C.T) if semiring != "plus_times" else np.allclose(Ct, C.T, rtol=1e-14, atol=0)


def test_contract_tensor_forms():
    rng = np.random.default_rng(11)
    V = rng.random((3, 4, 5, 2))
    T = rng.random((5, 4, 4, 3))
    # an interleaved output order, brute force over every index
    Z = oracle.contract("plus_times", "f64", "amei", V, "ebmj", T, "abij")
    ref = np.zeros((3, 4, 2, 3))
    for a in range(3):
        for b in range(4):
            for i in range(2):
                for j in range(3):
                    ref[a, b, i, j] = sum(V[a, m, e, i] * T[e, b, m, j] for m in range(4) for e in range(5))
    assert np.allclose(Z, ref, rtol=1e-14, atol=0)
    # a letter in all three tensors is a batch: the Hadamard product
    H = oracle.contract("plus_times", "f64", "abij", V[:, :, :2, :2], "abij", T[:3, :, :2, :2], "abij")
    assert np.array_equal(H, V[:, :, :2, :2] * T[:3, :, :2, :2])
    # no letter in C: the full contraction (a scalar)
    E = oracle.contract("plus_times", "f64", "abcd", V, "abcd", V, "")
    assert E.shape == () and np.isclose(E, (V * V).sum(), rtol=1e-14)
    # (min,+) int32 with absent entries and clamping at the identity
    W = np.array([[1, INT_INF], [INT_INF - 1, 2]], dtype=np.int32)
    P = oracle.contract("min_plus", "i32", "ik", W, "kj", W, "ij")
    assert P.tolist() == [[2, INT_INF], [INT_INF, 4]]


# ------------------------------------------------- Jacobi and transforms --

def test_jacobi_closed_forms():
    # diagonal A: one update solves it exactly
    n = 5
    d = np.arange(1, n + 1, dtype=np.float64)
    A = oracle.fold("plus_times", "f64", np.arange(n), np.arange(n), d, n, n)
    x, l, r, ok = oracle.jacobi(A, np.ones(n), np.zeros(n), 1e-14)
    assert ok and l == 1 and r == 0.0 and np.array_equal(x, 1.0 / d)
    # 2 x 2 by hand: A = [[4, 1], [2, 5]], b = [1, 2], x0 = 0
    A = oracle.fold("plus_times", "f64", [0, 0, 1, 1], [0, 1, 0, 1], np.array([4.0, 1, 2, 5]), 2, 2)
    x1, l1, _, ok1 = oracle.jacobi(A, [1.0, 2.0], [0.0, 0.0], 0.0, max_iters=1)
    x2, l2, _, ok2 = oracle.jacobi(A, [1.0, 2.0], [0.0, 0.0], 0.0, max_iters=2)
    assert not ok1 and not ok2 and l1 == 1 and l2 == 2
    assert np.allclose(x1, [0.25, 0.4], rtol=1e-15) and np.allclose(x2, [0.15, 0.3], rtol=1e-15)
    with pytest.raises(ValueError):
        oracle.jacobi(oracle.fold("plus_times", "f64", [0], [1], np.array([1.0]), 2, 2), [1.0, 1.0], [0.0, 0.0], 1e-6)


def test_jacobi_converges_to_the_solution():
    g = 6
    src, dst = synth.stencil27_edges(g)
    n = g ** 3
    vals = np.where(src == dst, 27.0, -1.0)
    A = oracle.fold("plus_times", "f64", dst, src, vals, n, n)
    b = synth.uniform_f64(synth.stream_key(3, 1), n)
    x, l, r, ok = oracle.jacobi(A, b, np.zeros(n), 1e-10)
    Ad = np.zeros((n, n))
    Ad[dst, src] = vals
    assert ok and r <= 1e-10 and np.allclose(x, np.linalg.solve(Ad, b), rtol=0, atol=1e-10)
    # the residual decreases by at most the Jacobi iteration's contraction
    assert l > 1


def test_transform_pins():
    rng = np.random.default_rng(5)
    C = rng.random((3, 4, 2, 5)) + 1.0
    Ei = rng.random(2)
    Ea = rng.random(3)
    # D["abij"] += Ei["i"]; D["abij"] -= Ea["a"] as nested loops
    D1 = oracle.transform("add", 1.0, "i", Ei, "", None, "abij", C)
    D2 = oracle.transform("add", -1.0, "a", Ea, "", None, "abij", D1)
    ref = C.copy()
    for a in range(3):
        for bb in range(4):
            for i in range(2):
                for j in range(5):
                    ref[a, bb, i, j] = C[a, bb, i, j] + Ei[i] - Ea[a]
    assert np.allclose(D2, ref, rtol=1e-15)
    # C["ij"] = C["ij"] / (A["i"] + B["j"])
    M = rng.random((4, 6)) + 1
    va, vb = rng.random(4), rng.random(6)
    out = oracle.transform("div_sum", 0.0, "i", va, "j", vb, "ij", M)
    assert np.array_equal(out, M / (va[:, None] + vb[None, :]))
    assert np.array_equal(oracle.transform("recip", 2.0, "", None, "", None, "ij", M), 2.0 / M)
    assert np.array_equal(oracle.transform("fma", 0.5, "ji", M.T, "ij", M, "ij", M), M + 0.5 * M * M)


# ------------------------------------------------- schedule features pins --
def _bin_of_len(x):
    # row-length bin from its definition: the bit length, capped at 9
    return min(9, int(x).bit_length())


def test_features_path_graph_closed_form():
    # path 0 -> 1 -> ... -> n-1: row 0 of A is empty, row i >= 1 holds (i, i-1);
    # w_0 = w_1 = 0 and w_i = 1 (i >= 2); every product reaches its own column
    n = 40
    A = oracle.fold("min_plus", "i32", np.arange(1, n), np.arange(0, n - 1), np.ones(n - 1, np.int32), n, n)
    f = oracle.features("min_plus", A, A)
    exp = np.zeros(32)
    exp[0], exp[1] = 1 / n, (n - 1) / n          # one empty row, n-1 rows of length 1
    exp[10], exp[11] = 2 / n, (n - 2) / n        # two rows without products
    exp[20], exp[21], exp[22] = np.log2(n + 1), np.log2(n + 1), np.log2(n)
    exp[23] = np.log2(n - 1)                     # sum w = n - 2
    exp[24] = 0.0                                # one output per product
    exp[25], exp[26] = 1.0, 1.0                  # log2(1 + 1)
    exp[27] = np.sqrt(2.0 / (n - 2))             # CV of n-2 ones and 2 zeros
    exp[29] = 1.0                                # (min,+)
    np.testing.assert_allclose(f, exp.astype(np.float32), rtol=1e-6, atol=1e-7)


def test_features_star_closed_form():
    # bidirectional star with L leaves: every row has L products; row 0 reaches
    # only column 0, a leaf reaches all L leaves: CR = L(L+1) / (L^2 + 1)
    L = 100
    rows = np.concatenate([np.zeros(L, np.int64), np.arange(1, L + 1)])
    cols = np.concatenate([np.arange(1, L + 1), np.zeros(L, np.int64)])
    A = oracle.fold("plus_times", "f64", rows, cols, np.ones(2 * L), L + 1, L + 1)
    f = oracle.features("plus_times", A, A)
    m = L + 1
    assert f[_bin_of_len(L)] == np.float32(1 / m) and f[1] == np.float32(L / m)   # 100 -> bit length 7
    assert f[10 + (L.bit_length() + 1) // 2] == np.float32(1.0)                   # w = 100: bin 4
    assert f[24] == np.float32(np.log2(L * (L + 1) / (L * L + 1)))
    assert f[27] == 0.0                                                           # every w equal
    assert f[25] == np.float32(np.log2(L + 1)) and f[26] == np.float32(np.log2(L + 1))
    assert f[23] == np.float32(np.log2(L * (L + 1) + 1))
    assert list(f[28:]) == [1, 0, 0, 0]


def test_features_identity_and_empty():
    n = 700
    I = oracle.fold("or_and", "bool", np.arange(n), np.arange(n), np.ones(n, np.uint8), n, n)
    f = oracle.features("or_and", I, I)
    assert f[1] == 1.0 and f[11] == 1.0 and f[24] == 0.0 and f[27] == 0.0
    assert list(f[28:]) == [0, 0, 1, 0]
    E = oracle.fold("or_and", "bool", np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.uint8), 5, 5)
    g = oracle.features("or_and", E, E)
    assert g[0] == 1.0 and g[10] == 1.0 and g[24] == 0.0 and g[27] == 0.0 and g[23] == 0.0


def test_features_compression_ratio_samples_stride_rows():
    # m = 1024 rows, s = 512 samples: rows floor(t * 1024 / 512) = 2t, the
    # even rows.  Even rows reach 4 columns through 8 products (CR 2), odd rows
    # 8 columns through 8 products (CR 1): the estimate must be exactly 2.
    m = 1024
    # B: 2 rows per "kind"; B row 0 = cols {0,1,2,3}, row 1 = cols {0,1,2,3},
    # row 2 = {4..7}, row 3 = {8..11}
    brows = np.repeat(np.arange(4), 4)
    bcols = np.array([0, 1, 2, 3, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11])
    B = oracle.fold("plus_times", "f64", brows, bcols, np.ones(16), 4, 12)
    even = np.arange(0, m, 2)
    odd = np.arange(1, m, 2)
    arows = np.concatenate([np.repeat(even, 2), np.repeat(odd, 2)])
    acols = np.concatenate([np.tile([0, 1], even.size), np.tile([2, 3], odd.size)])
    A = oracle.fold("plus_times", "f64", arows, acols, np.ones(arows.size), m, 4)
    f = oracle.features("plus_times", A, B)
    assert f[24] == np.float32(1.0)  # log2(2)
    assert f[23] == np.float32(np.log2(8 * m + 1))


# ----------------------------------------------------------- Adam pins --
def test_adam_first_step_closed_form():
    # with zero moments the bias corrections cancel exactly: the first step
    # moves every parameter by -lr g / (|g| + eps)
    from oracle import mlp
    rng = np.random.default_rng(5)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 0.01, 1e-8
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr, 0.9, 0.999, eps)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_two_steps_by_hand():
    # beta1 = 1/2, beta2 = 3/4, lr = 1/10, eps = 0, p0 = 1, g1 = 2, g2 = 1:
    # step 1: p1 = 1 - 0.1 * 2 / 2 = 0.9; m = 1, v = 1
    # step 2: m = 0.5 + 0.5 = 1, mh = 1 / (1 - 1/4) = 4/3;
    #         v = 0.75 + 0.25 = 1, vh = 1 / (1 - 9/16) = 16/7;
    #         p2 = 0.9 - 0.1 * (4/3) / (4 / sqrt 7) = 0.9 - sqrt(7) / 30
    from oracle import mlp
    p1, m, v = mlp.adam_step(np.array([1.0]), np.array([2.0]), np.zeros(1), np.zeros(1), 1, 0.1, 0.5, 0.75, 0.0)
    assert abs(p1[0] - 0.9) < 1e-15 and abs(m[0] - 1.0) < 1e-15 and abs(v[0] - 1.0) < 1e-15
    p2, m, v = mlp.adam_step(p1, np.array([1.0]), m, v, 2, 0.1, 0.5, 0.75, 0.0)
    assert abs(p2[0] - (0.9 - np.sqrt(7.0) / 30.0)) < 1e-15


def _golden_semirings():
    path = os.path.join(os.path.dirname(__file__), "golden", "semiring_identities.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            sr, dt, add_id, mul_id = line.split()
            rows.append((sr, dt, float(add_id) if dt == "f64" else int(add_id),
                         float(mul_id) if dt == "f64" else int(mul_id)))
    return rows


@pytest.mark.parametrize("semiring,dtype,add_id,mul_id", _golden_semirings())
def test_semiring_identities_as_the_paper_defines_them(semiring, dtype, add_id, mul_id):
    """The oracle's default identities are the ones Section 3.1 prints, and
    they act as identities: an entry equal to the additive one is absent
    (dropped by the fold), the multiplicative one leaves a product's other
    factor unchanged, and two additive identities combined by the product
    stay representable (the reason the paper halves INT_MAX)."""
    assert oracle.default_add_id(semiring, dtype) == add_id
    np_dt = oracle.NP_DTYPES[dtype]
    vals = np.array([add_id, 5, 7], dtype=np_dt)
    F = oracle.fold(semiring, dtype, np.array([0, 0, 1]), np.array([0, 1, 1]), vals, 2, 2)
    assert F.col.tolist() == [1, 1] and F.rowptr.tolist() == [0, 1, 2]
    # [mul_id] x [x] = [x]
    I = oracle.fold(semiring, dtype, np.array([0]), np.array([0]), np.array([mul_id], dtype=np_dt), 1, 1)
    for x in (3, 11):
        X = oracle.fold(semiring, dtype, np.array([0]), np.array([0]), np.array([x], dtype=np_dt), 1, 1)
        assert oracle.spgemm(semiring, dtype, I, X).val.tolist() == [x]
    if dtype == "i32":
        assert 2 * add_id <= np.iinfo(np.int32).max
