"""Full-size parity of the measured workloads (GPU only).

* R-MAT scale 18, edge factor 16, A.A over (+,x) in fp64 and fp32, in every
  SpGEMM schedule, compared on sampled rows (the 300 heaviest rows and a
  seeded 1% of all rows) with the oracle computing just those rows; the
  order-3 tensor contraction of the same workload in full.
* R-MAT scale 21, edge factor 16, A.A in full, streamed in row panels as the
  benchmark runs it, in (+,x) fp64 and fp32 and (min,+) int32, on sampled
  rows (the heaviest and a seeded random sample).
* R-MAT scale 20: 64-source Bellman-Ford fixpoint and BFS in full.
* 512 uneven ER instances, batched against per-instance and the oracle.
"""

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import check_csr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmat18():
    src, dst = synth.rmat_edges(18, 16, 0.57, 0.19, 0.19, synth.SEED_CFG1)
    return src, dst


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rmat18_square_sampled_rows(rmat18, dtype):
    src, dst = rmat18
    n = 1 << 18
    ctx = srtc.Context(0)
    v = synth.edge_values(dtype, src.size, synth.SEED_CFG1, 0 if dtype == "f64" else 1)
    keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
    A = ctx.fold("plus_times", srtc.COO(keys, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
    O = oracle.fold("plus_times", dtype, dst, src, v, n, n)
    rn = np.diff(O.rowptr)
    w = np.zeros(n, dtype=np.int64)
    np.add.at(w, np.repeat(np.arange(n), rn), rn[O.col])
    # the 300 heaviest rows (the dense-window and ranked-group paths carry
    # nearly all of C) and a seeded 1% of all rows
    heavy = np.argsort(w)[-300:]
    rnd = synth.permutation(synth.stream_key(synth.SEED_CFG1, 99), n)[:n // 100]
    rows = np.unique(np.concatenate([heavy, rnd]))
    exp = oracle.spgemm("plus_times", dtype, O, O, rows=rows)
    for sch in range(srtc.NUM_SCHEDULES):
        say("rmat18", dtype, "schedule", sch)
        C = ctx.contract("plus_times", "ik", A, "kj", A, "ij", schedule=sch)
        check_csr(C, exp, "plus_times", dtype, rows=rows)
        del C
        torch.cuda.empty_cache()


def test_tensor512_contraction_full():
    dims = (512, 512, 512)
    keys = synth.bernoulli_keys(dims, 1e-3, seed=synth.SEED_CFG1, tag=1)
    tv = synth.uniform_f32(synth.stream_key(synth.SEED_CFG1, 11), keys.size)
    M = synth.uniform_f32(synth.stream_key(synth.SEED_CFG1, 12), 512 * 64).reshape(512, 64)
    ctx = srtc.Context(0)
    T = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(tv, device="cuda"), dims)
    C = torch.empty((512, 512, 64), dtype=torch.float32, device="cuda")
    ctx.contract("plus_times", "ijk", T, "kl", torch.as_tensor(M, device="cuda"), "ijl", C=C)
    F = oracle.fold_tensor("plus_times", "f32", keys, tv, dims, "ijk", "ij", "k")
    exp, _ = oracle.spmm("plus_times", "f32", F, M)
    got = C.cpu().numpy().reshape(-1, 64).astype(np.float64)
    assert np.all(np.abs(got - exp) <= 1e-5 * np.abs(exp))


def test_rmat20_multi_source_sssp_and_bfs():
    # R-MAT 20, edge factor 16, int32 weights [1,255], 64 sources: the
    # Bellman-Ford fixpoint as a (min,+) SpMM with graph-captured steps and
    # the bit-packed BFS.  All 64 distance columns and the step count are
    # checked against the oracle's Bellman-Ford, a seeded sample of 4 sources
    # also against Dijkstra; BFS levels of all 64 sources against the
    # oracle's queue BFS.
    scale = 20
    n = 1 << scale
    src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, synth.SEED_CFG2)
    w = synth.edge_values("i32", src.size, synth.SEED_CFG2, lo=1, hi=255)
    ctx = srtc.Context(0)
    keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
    G = ctx.fold("min_plus", srtc.COO(keys, torch.as_tensor(w, device="cuda"), (n, n)), "ij", "i", "j")
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    sources = synth.pick_sources(n, src, 64, synth.SEED_CFG2)
    P0 = np.full((n, 64), oracle.INT_INF, np.int32)
    P0[sources, np.arange(64)] = 0
    X = torch.as_tensor(P0, device="cuda")
    say("rmat20 BF fixpoint")
    it = ctx.fixpoint("min_plus", G, X, steps_per_check=4)
    got = X.cpu().numpy()
    Pexp, it_exp, conv = oracle.bellman_ford("min_plus", "i32", O, P0)
    assert conv and it == it_exp
    assert np.array_equal(got, Pexp)
    pick = np.sort(synth.permutation(synth.stream_key(synth.SEED_CFG2, 5), 64)[:4])
    assert np.array_equal(Pexp[:, pick].astype(np.int64), oracle.dijkstra(O, sources[pick]))
    X2 = torch.as_tensor(P0, device="cuda")
    assert ctx.fixpoint("min_plus", G, X2, steps_per_check=4, changed_rows_only=True) == it_exp
    assert torch.equal(X2, X)
    say("rmat20 BFS")
    lev, depth = ctx.bfs_levels(G, sources)
    exp = oracle.bfs_levels(O, sources)
    assert np.array_equal(lev.cpu().numpy(), exp) and depth == exp.max()


def test_batch512_matches_per_instance_and_oracle():
    # 512 ER instances, n log-uniform in [1e3,1e5], degree uniform in
    # [4,32], int32 weights [1,100]: (min,+) A.A and an 8-source
    # Bellman-Ford each.  Batched results equal per-instance results bit
    # for bit on every instance; six sampled instances (the largest among
    # them) are checked against the oracle.
    ninst, nsrc = 512, 8
    ns, ds = synth.er_batch_params(ninst, synth.SEED_CFG3)
    ctx = srtc.Context(0)
    As, X0s, host = [], [], []
    for b in range(ninst):
        n = int(ns[b])
        src, dst = synth.er_edges(n, float(ds[b]), synth.SEED_CFG3, tag=b)
        w = synth.edge_values("i32", src.size, synth.SEED_CFG3, tag=b, lo=1, hi=100)
        keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
        As.append(ctx.fold("min_plus", srtc.COO(keys, torch.as_tensor(w, device="cuda"), (n, n)), "ij", "i", "j"))
        sources = synth.pick_sources(n, src, nsrc, synth.SEED_CFG3, tag=b)
        P0 = np.full((n, nsrc), oracle.INT_INF, np.int32)
        P0[sources, np.arange(sources.size)] = 0
        X0s.append(P0)
        host.append((src, dst, w))
    say("batch512 batched")
    Cs = ctx.batch_contract("min_plus", As, As)
    Xs = [torch.as_tensor(p, device="cuda") for p in X0s]
    its = ctx.batch_fixpoint("min_plus", As, Xs, steps_per_check=4)
    say("batch512 per instance")
    for b in range(ninst):
        C = ctx.contract("min_plus", "ik", As[b], "kj", As[b], "ij")
        assert C.nnz == Cs[b].nnz, b
        assert torch.equal(C.rowptr, Cs[b].rowptr) and torch.equal(C.col, Cs[b].col) and torch.equal(C.val, Cs[b].val), b
        X = torch.as_tensor(X0s[b], device="cuda")
        assert ctx.fixpoint("min_plus", As[b], X, steps_per_check=4) == its[b], b
        assert torch.equal(X, Xs[b]), b
        del C, X
    say("batch512 oracle samples")
    pick = set(synth.permutation(synth.stream_key(synth.SEED_CFG3, 7), ninst)[:5].tolist()) | {int(np.argmax(ns))}
    for b in sorted(pick):
        src, dst, w = host[b]
        n = int(ns[b])
        O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
        check_csr(Cs[b], oracle.spgemm("min_plus", "i32", O, O), "min_plus", "i32")
        exp, it_exp, conv = oracle.bellman_ford("min_plus", "i32", O, X0s[b])
        assert conv and its[b] == it_exp
        assert np.array_equal(Xs[b].cpu().numpy(), exp)


def test_apsp_tiskin_dense2048_sampled():
    """The dense APSP workload (n = 2,048, weights U[1, n^2]) in the bench's
    call: distance columns of sampled sources against the oracle's Dijkstra;
    every hop count is one more than the fewest hops of a predecessor on a
    lightest path (and 0 on the diagonal)."""
    n = 2048
    say("apsp dense", n)
    src, dst, w = synth.dense_graph(n, synth.SEED_CFG0)
    ctx = srtc.Context(0)
    coo = srtc.COO(torch.as_tensor(dst * n + src, device="cuda"), torch.as_tensor(w, device="cuda"), (n, n))
    rn = []
    D, H, rounds = ctx.apsp_tiskin(coo, round_nnz=rn)
    D = D.cpu().numpy().astype(np.int64)
    H = H.cpu().numpy().astype(np.int64)
    say("rounds", rounds, rn)
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    cols = synth.permutation(synth.stream_key(synth.SEED_CFG0, 77), n)[:8]
    ref = oracle.dijkstra(O, cols)
    assert np.array_equal(D[:, cols], ref)
    W = np.full((n, n), np.iinfo(np.int64).max // 4, np.int64)
    W[dst, src] = w
    for j in cols:
        cand = W + D[:, j][None, :]              # cand[i, k] = A[i, k] + D[k, j]
        on = cand == D[:, j][:, None]
        hk = np.where(on, H[:, j][None, :], np.iinfo(np.int64).max)
        exp = 1 + hk.min(axis=1)
        exp[j] = 0
        assert np.array_equal(H[:, j], exp)
    assert rounds == len(rn) and rn[0] == n * (n - 1) and 1 << (rounds - 1) <= H.max() <= 1 << rounds


@pytest.mark.parametrize("semiring,dtype", [("min_plus", "i32"), ("plus_times", "f64")])
def test_spgemm_wide_matrix_multiwindow_symbolic(semiring, dtype):
    """2.5M columns: heavy rows count their outputs over several LDS bitmap
    windows (each walking only its own products through the window table)
    and accumulate over several dense windows; every schedule, all rows."""
    n, m = 2_500_000, 48
    say("wide spgemm", semiring, dtype)
    src, dst = synth.er_edges(n, 4, seed=88)
    wB = synth.edge_values("i32" if dtype == "i32" else dtype, src.size, 88, lo=1, hi=100)
    ka = synth.bernoulli_keys((m, n), 3000 / n, seed=89)
    wA = synth.edge_values("i32" if dtype == "i32" else dtype, ka.size, 89, lo=1, hi=100)
    ctx = srtc.Context(0)
    B = ctx.fold(semiring, srtc.COO(torch.as_tensor(dst * n + src, device="cuda"), torch.as_tensor(wB, device="cuda"),
                                    (n, n)), "ij", "i", "j")
    A = ctx.fold(semiring, srtc.COO(torch.as_tensor(ka, device="cuda"), torch.as_tensor(wA, device="cuda"), (m, n)),
                 "ij", "i", "j")
    Bo = oracle.fold(semiring, dtype, dst, src, wB, n, n)
    Ao = oracle.fold(semiring, dtype, ka // n, ka % n, wA, m, n)
    exp = oracle.spgemm(semiring, dtype, Ao, Bo)
    for sched in range(srtc.NUM_SCHEDULES):
        say("  schedule", sched)
        C = ctx.contract(semiring, "ik", A, "kj", B, "ij", schedule=sched)
        check_csr(C, exp, semiring, dtype)


@pytest.fixture(scope="module")
def rmat21():
    src, dst = synth.rmat_edges(21, 16, 0.57, 0.19, 0.19, synth.SEED_CFG4, tag=21)
    return src, dst


@pytest.mark.parametrize("semiring,dtype,heavy,frac", [("plus_times", "f64", 300, 1e-2),
                                                         ("plus_times", "f32", 300, 1e-2),
                                                         ("min_plus", "i32", 300, 1e-2)])
def test_rmat21_square_in_panels_sampled_rows(rmat21, semiring, dtype, heavy, frac):
    """R-MAT scale 21 (edge factor 16) A.A in full, streamed in row panels
    of at most 8e9 products as the benchmark runs it (schedule chosen by the
    library); the 300 heaviest rows and a seeded 1% random sample of rows
    are checked against the oracle computing just those rows."""
    src, dst = rmat21
    n = 1 << 21
    v = synth.edge_values(dtype, src.size, synth.SEED_CFG4, tag=21, lo=1, hi=100)
    ctx = srtc.Context(0)
    keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
    A = ctx.fold(semiring, srtc.COO(keys, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
    del keys
    O = oracle.fold(semiring, dtype, dst, src, v, n, n)
    rn = np.diff(O.rowptr)
    w = np.zeros(n, dtype=np.int64)
    np.add.at(w, np.repeat(np.arange(n), rn), rn[O.col])
    rows = np.unique(np.concatenate([np.argsort(w)[-heavy:],
                                     synth.permutation(synth.stream_key(synth.SEED_CFG4, 98), n)[:int(n * frac)]]))
    got = {}

    def take(r0, P):
        r1 = r0 + P.shape[0]
        sel = rows[(rows >= r0) & (rows < r1)]
        if sel.size == 0:
            return
        rp = P.rowptr.cpu().numpy()
        for r in sel:
            a, b = int(rp[r - r0]), int(rp[r - r0 + 1])
            got[int(r)] = (P.col[a:b].cpu().numpy(), P.val[a:b].cpu().numpy())

    say("rmat21", semiring, dtype, "streaming")
    count = ctx.contract_panels(semiring, "ik", A, "kj", A, "ij", take, panel_products=8_000_000_000)
    say("rmat21 panels", count, "oracle rows", rows.size)
    assert count >= int(w.sum() // 8_000_000_000)
    exp = oracle.spgemm(semiring, dtype, O, O, rows=rows)
    rp = np.concatenate([[0], np.cumsum([got[int(r)][0].size if int(r) in got else 0 for r in rows])])
    col = np.concatenate([got[int(r)][0] for r in rows if int(r) in got])
    val = np.concatenate([got[int(r)][1] for r in rows if int(r) in got])
    G = srtc.CSR(torch.as_tensor(rp), torch.as_tensor(col), torch.as_tensor(val), (rows.size, n))
    check_csr(G, exp, semiring, dtype)
