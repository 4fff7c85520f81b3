"""Parity of the packed-path (min,+) semiring and Tiskin's path doubling
with the CPU oracle (GPU only).  Distances, hop counts and the number of
products formed are compared exactly."""

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import gpu_fold, say

pytestmark = pytest.mark.gpu
INF = oracle.INT_INF


@pytest.fixture(scope="module")
def ctx():
    return srtc.Context(0)


def graph(n, src, dst, w):
    """(GPU COO, oracle CSR) of edges src -> dst (entry (dst, src))."""
    keys = np.asarray(dst, np.int64) * n + np.asarray(src, np.int64)
    coo = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(np.asarray(w, np.int32), device="cuda"), (n, n))
    return coo, oracle.fold("min_plus", "i32", dst, src, np.asarray(w, np.int32), n, n)


def check_apsp(ctx, n, src, dst, w, add_id=None, what=""):
    say("apsp", what, "n =", n, "edges =", len(src))
    G, O = graph(n, src, dst, w)
    rn = []
    D, H, rounds = ctx.apsp_tiskin(G, add_id=add_id, round_nnz=rn)
    torch.cuda.synchronize()
    Do, Ho, ro, pl = oracle.apsp_tiskin(O, inf_value=INF if add_id is None else add_id)
    assert np.array_equal(D.cpu().numpy().astype(np.int64), Do), "distances differ"
    assert np.array_equal(H.cpu().numpy().astype(np.int64), Ho), "hop counts differ"
    assert rounds == ro and rn == pl[:ro]
    return D, H, rounds


@pytest.mark.parametrize("n,d,lo,hi,seed", [(1, 1, 1, 9, 1), (2, 1, 0, 5, 2), (65, 4, 0, 9, 3), (300, 3, 0, 9, 4),
                                            (301, 12, 1, 1000, 5), (129, 0.7, 1, 20, 6)])
def test_tiskin_er_graphs(ctx, n, d, lo, hi, seed):
    src, dst = synth.er_edges(n, d, seed)
    w = synth.edge_values("i32", src.size, seed, lo=lo, hi=hi)
    check_apsp(ctx, n, src, dst, w, what=f"er d={d} w=[{lo},{hi}]")


@pytest.mark.parametrize("n", [200, 257, 384])
def test_tiskin_dense_graph(ctx, n):
    # rounds whose sparse factor is dense run on dense tiles (ragged edges
    # at 200 and 257)
    src, dst, w = synth.dense_graph(n, 8)
    _, _, rounds = check_apsp(ctx, n, src, dst, w, what="dense")
    assert rounds >= 2


def test_tiskin_dense_rounds_value_widths(ctx):
    # heavy weights leave no room for the 32-bit tile form (64-bit dense
    # rounds); a small identity cuts sums off inside a 32-bit round
    n = 260
    src, dst, _ = synth.dense_graph(n, 9)
    w = synth.randint(synth.stream_key(9, 5), src.size, 1, 1 << 28).astype(np.int32)
    check_apsp(ctx, n, src, dst, w, add_id=(1 << 30) - 1, what="dense wide weights")
    w = synth.randint(synth.stream_key(9, 6), src.size, 1, 90).astype(np.int32)
    check_apsp(ctx, n, src, dst, w, add_id=100, what="dense small identity")


def test_tiskin_dense_rounds_with_ties(ctx):
    # many equal weights: the fewest-hops rule decides most entries
    n = 333
    src, dst = synth.er_edges(n, 120, 13)
    w = synth.edge_values("i32", src.size, 13, lo=0, hi=3)
    check_apsp(ctx, n, src, dst, w, what="dense ties")


def test_tiskin_path_graph_and_unreachable(ctx):
    n = 130
    w = synth.randint(synth.stream_key(12, 1), n - 1, 1, 50).astype(np.int32)
    src = np.arange(n - 1)
    _, H, rounds = check_apsp(ctx, n, src, src + 1, w, what="path")
    assert rounds == 8 and int(H.max()) == n - 1
    # two components, self-loops and zero weights
    src = np.array([0, 1, 2, 2, 5, 6, 7, 7, 3])
    dst = np.array([1, 2, 0, 2, 6, 7, 5, 7, 4])
    w = np.array([0, 0, 0, 4, 3, 0, 2, 1, 6])
    check_apsp(ctx, 9, src, dst, w, what="components")
    check_apsp(ctx, 7, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int32), what="no edges")


def test_tiskin_duplicates_custom_identity_and_csr_input(ctx):
    n = 150
    src, dst = synth.er_edges(n, 5, 9)
    w = synth.edge_values("i32", src.size, 9, lo=1, hi=60)
    # repeated edges: the lightest counts
    w2 = synth.edge_values("i32", src.size, 9, tag=1, lo=1, hi=60)
    s2, d2, ww = np.concatenate([src, src]), np.concatenate([dst, dst]), np.concatenate([w, w2])
    check_apsp(ctx, n, s2, d2, ww, what="duplicates")
    # an identity that cuts off long paths: weights reaching it are no path
    check_apsp(ctx, n, src, dst, w, add_id=150, what="identity 150")
    # CSR input gives the same result as COO
    G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
    Dc, Hc, rc = ctx.apsp_tiskin(G)
    Dk, Hk, rk = ctx.apsp_tiskin(graph(n, src, dst, w)[0])
    assert torch.equal(Dc, Dk) and torch.equal(Hc, Hk) and rc == rk


def test_tiskin_errors(ctx):
    G, _ = graph(3, np.array([0]), np.array([1]), np.array([-2]))
    with pytest.raises(srtc.SrtcError):
        ctx.apsp_tiskin(G)
    R = srtc.COO(torch.zeros(0, dtype=torch.int64, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"),
                 (3, 4))
    with pytest.raises(srtc.SrtcError):
        ctx.apsp_tiskin(R)
    F = srtc.COO(torch.zeros(1, dtype=torch.int64, device="cuda"), torch.ones(1, dtype=torch.float32, device="cuda"),
                 (3, 3))
    with pytest.raises(srtc.SrtcError):
        ctx.apsp_tiskin(F)


def path_coo(n, m, rows, cols, w, h):
    keys = np.asarray(rows, np.int64) * m + np.asarray(cols, np.int64)
    val = srtc.pack_path(torch.as_tensor(np.asarray(w, np.int64)), torch.as_tensor(np.asarray(h, np.int64)))
    return srtc.COO(torch.as_tensor(keys, device="cuda"), val.cuda(), (n, m))


def dense_of(rows, cols, w, h, m, n):
    """Dense (weight, hops) of an entry list; repeated entries keep the
    lighter path, fewer hops on equal weights."""
    Dw = np.full((m, n), INF, np.int64)
    Dh = np.full((m, n), -1, np.int64)
    for r, c, a, b in zip(rows, cols, w, h):
        if a < Dw[r, c] or (a == Dw[r, c] and b < Dh[r, c]):
            Dw[r, c], Dh[r, c] = a, b
    return Dw, Dh


@pytest.mark.parametrize("n,dens,heavy", [(97, 0.05, 0), (600, 0.01, 0), (800, 0.004, 3)])
def test_path_semiring_contraction(ctx, n, dens, heavy):
    say("path contraction", n, dens, heavy)
    rows_l, cols_l = [], []
    for t in range(2):
        k = synth.bernoulli_keys((n, n), dens, seed=50 + t)
        r, c = k // n, k % n
        if heavy:
            # a few rows of A that reach most of B's rows (dense windows)
            hr = np.repeat(np.arange(heavy) * 7, n // 2)
            hc = np.tile(np.arange(0, n, 2), heavy)
            r, c = np.concatenate([r, hr]), np.concatenate([c, hc])
        rows_l.append(r)
        cols_l.append(c)
    # repeated entries in A to check the fold's lexicographic combine
    ra, ca = np.concatenate([rows_l[0], rows_l[0][:50]]), np.concatenate([cols_l[0], cols_l[0][:50]])
    wa = synth.randint(synth.stream_key(60, 1), ra.size, 0, 6)
    ha = synth.randint(synth.stream_key(60, 2), ra.size, 0, 5)
    rb, cb = rows_l[1], cols_l[1]
    wb = synth.randint(synth.stream_key(60, 3), rb.size, 0, 6)
    hb = synth.randint(synth.stream_key(60, 4), rb.size, 0, 5)
    A = ctx.fold("min_plus", path_coo(n, n, ra, ca, wa, ha), "ij", "i", "j")
    B = ctx.fold("min_plus", path_coo(n, n, rb, cb, wb, hb), "ij", "i", "j")
    Aw, Ah = dense_of(ra, ca, wa, ha, n, n)
    Bw, Bh = dense_of(rb, cb, wb, hb, n, n)
    Cw, Ch = oracle.path_product(Aw, Ah, Bw, Bh)
    # every schedule when some rows are heavy (8-byte dense windows)
    for sched in (range(srtc.NUM_SCHEDULES) if heavy else [-1]):
        say("  schedule", sched)
        C = ctx.contract("min_plus", "ik", A, "kj", B, "ij", validate=True, schedule=sched)
        rp, col, val = C.to_host()
        val = val.astype(np.int64)
        Gw = np.full((n, n), INF, np.int64)
        Gh = np.full((n, n), -1, np.int64)
        rr = np.repeat(np.arange(n), np.diff(rp))
        Gw[rr, col] = val >> 32
        Gh[rr, col] = val & 0xFFFFFFFF
        assert C.nnz == int((Cw < INF).sum())
        assert np.array_equal(Gw, Cw) and np.array_equal(Gh, Ch)
        assert all(np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0) for i in range(n))
