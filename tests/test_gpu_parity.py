"""Parity of the HIP library with the CPU oracle (GPU only).

Every input comes from the seeded generators; the library folds it with its
own kernels and the oracle with its own code, then the results are compared
element by element: bit-exact for (min,+), (or,and), (max,x); within the
stated relative bounds for (+,x) (1e-12 fp64, 1e-5 fp32 against fp64)."""

import os

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import EXACT, PAIRS, RTOL, TORCH, check_csr, gpu_fold, pair_inputs, say, values

pytestmark = pytest.mark.gpu
INF = oracle.INT_INF


@pytest.fixture(scope="module")
def ctx():
    return srtc.Context(0)


# ------------------------------------------------------------------- fold --
@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_fold_duplicates_and_identities(ctx, semiring, dtype):
    say("fold", semiring, dtype)
    src, dst = synth.rmat_edges(12, 8, 0.57, 0.19, 0.19, seed=101)   # ~32k pairs, duplicates
    v = values(semiring, dtype, src.size, 101)
    # sprinkle explicit identity entries (absent by definition)
    idv = oracle.default_add_id(semiring, dtype)
    v = v.copy()
    v[::97] = idv
    n = 1 << 12
    G = gpu_fold(ctx, semiring, dtype, dst, src, v, n, n)
    O = oracle.fold(semiring, dtype, dst, src, v, n, n)
    # fold combines duplicates in input order on both sides: bit-exact
    rp, col, val = G.to_host()
    assert np.array_equal(rp, O.rowptr) and np.array_equal(col, O.col)
    assert np.array_equal(val, O.val)


def test_fold_edge_cases(ctx):
    say("fold edge cases")
    e = gpu_fold(ctx, "min_plus", "i32", [], [], np.zeros(0, np.int32), 5, 7)
    assert e.nnz == 0 and e.rowptr.cpu().tolist() == [0] * 6
    one = gpu_fold(ctx, "min_plus", "i32", [4], [6], np.array([3], np.int32), 5, 7)
    assert one.rowptr.cpu().tolist() == [0, 0, 0, 0, 0, 1] and one.col.cpu().tolist() == [6]
    # all entries identity -> empty
    z = gpu_fold(ctx, "plus_times", "f64", [0, 1], [1, 0], np.zeros(2), 2, 2)
    assert z.nnz == 0


def test_fold_transpose_and_tensor_modes(ctx):
    say("fold transpose / tensor modes")
    src, dst = synth.er_edges(3000, 5, seed=55)
    v = values("plus_times", "f64", src.size, 55)
    G = gpu_fold(ctx, "plus_times", "f64", dst, src, v, 3000, 3000)
    T = ctx.fold("plus_times", G, "ij", "j", "i")              # transpose of a CSR
    O = oracle.fold("plus_times", "f64", src, dst, v, 3000, 3000)
    rp, col, val = T.to_host()
    assert np.array_equal(rp, O.rowptr) and np.array_equal(col, O.col) and np.array_equal(val, O.val)
    dims = (37, 41, 29)
    keys = synth.bernoulli_keys(dims, 0.05, seed=9)
    tv = synth.uniform_f32(synth.stream_key(9, 1), keys.size)
    coo = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(tv, device="cuda"), dims)
    F = ctx.fold("plus_times", coo, "ijk", "ki", "j")
    OF = oracle.fold_tensor("plus_times", "f32", keys, tv, dims, "ijk", "ki", "j")
    rp, col, val = F.to_host()
    assert np.array_equal(rp, OF.rowptr) and np.array_equal(col, OF.col) and np.array_equal(val, OF.val)


# ----------------------------------------------------------------- spgemm --
CASES = {
    "er500": lambda: (synth.er_edges(500, 6, seed=3), 500),
    "rmat11": lambda: (synth.rmat_edges(11, 8, 0.57, 0.19, 0.19, seed=7), 1 << 11),
    "rmat15w": lambda: (synth.rmat_edges(15, 4, 0.57, 0.19, 0.19, seed=7), 1 << 15),  # several windows
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_spgemm_parity(ctx, semiring, dtype, case):
    (src, dst), n = CASES[case]()
    say("spgemm", semiring, dtype, case)
    G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, 11)
    exp = oracle.spgemm(semiring, dtype, O, O)
    scheds = range(srtc.NUM_SCHEDULES) if (semiring, dtype) in EXACT and case != "rmat15w" else (0, 2, 4)
    for sch in scheds:
        say("  schedule", sch)
        C = ctx.contract(semiring, "ik", G, "kj", G, "ij", schedule=sch)
        check_csr(C, exp, semiring, dtype)


def test_spgemm_heavy_rows_all_schedules(ctx):
    # R-MAT 14, edge factor 16: >1000 rows above 4096 outputs (dense windows)
    src, dst = synth.rmat_edges(14, 16, 0.57, 0.19, 0.19, seed=7)
    n = 1 << 14
    for semiring, dtype in (("min_plus", "i32"), ("plus_times", "f64")):
        G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, 12)
        exp = oracle.spgemm(semiring, dtype, O, O)
        for sch in range(srtc.NUM_SCHEDULES):
            say("heavy", semiring, dtype, "schedule", sch)
            check_csr(ctx.contract(semiring, "ik", G, "kj", G, "ij", schedule=sch), exp, semiring, dtype)


def window_structured_pair(semiring, dtype, seed, cancel=False):
    """A (15 x 2048) times B (2048 x 65,659): B's rows are dense in some
    8192-column windows, sparse in others and empty in windows 4-5 (the last
    window ragged); A's rows range from 1 to 500 entries, one avoids B's 16
    dense rows and one hits them (its product is dense in most windows), one
    is empty.  Rows of the product therefore mix dense windows, runs of
    sparse windows, skipped empty windows, A rows longer than a block and
    rows with several tiles per window."""
    rng = np.random.default_rng(seed)
    k, n, W = 2048, 65536 + 123, 8192
    b_rows, b_cols = [], []
    for r in range(k):
        parts = []
        for w, c in ((0, 40), (1, 6000 if r < 16 else 5), (2, 6000 if r < 16 else 5), (3, 6000 if r < 16 else 5),
                     (6, 200 if r % 7 == 0 else 3), (7, 2), (8, 2)):
            lo, hi = w * W, min(n, w * W + W)
            parts.append(lo + rng.choice(hi - lo, size=min(c, hi - lo), replace=False))
        cols = np.unique(np.concatenate(parts))
        b_rows.append(np.full(cols.size, r)), b_cols.append(cols)
    a_rows, a_cols = [], []
    sizes = [1, 3, 10, 60, 100, 300, 40, 7, 2, 20, 500, 5, 260]
    for i, c in enumerate(sizes):
        cols = np.sort(16 + rng.choice(k - 16, size=c, replace=False))
        a_rows.append(np.full(c, i)), a_cols.append(cols)
    heavy = np.unique(np.concatenate([np.arange(16), rng.choice(k, size=300, replace=False)]))
    a_rows.append(np.full(heavy.size, len(sizes))), a_cols.append(heavy)
    m = len(sizes) + 2                                   # the last row stays empty
    ar, ac = np.concatenate(a_rows), np.concatenate(a_cols)
    br, bc = np.concatenate(b_rows), np.concatenate(b_cols)
    if cancel:
        av = rng.choice([-1.0, 1.0], ar.size).astype(oracle.NP_DTYPES[dtype])
        bv = rng.choice([-1.0, 1.0], br.size).astype(oracle.NP_DTYPES[dtype])
    else:
        av, bv = values(semiring, dtype, ar.size, seed, 1), values(semiring, dtype, br.size, seed, 2)
    return (ar, ac, av, m, k), (br, bc, bv, k, n)


@pytest.mark.parametrize("semiring,dtype,cancel", [("plus_times", "f64", False), ("plus_times", "f64", True),
                                                   ("plus_times", "f32", False), ("min_plus", "i32", False),
                                                   ("max_times", "f64", False), ("or_and", "bool", False)])
def test_spgemm_window_groups_all_schedules(ctx, semiring, dtype, cancel):
    """Dense rows over many column windows: dense windows, ranked groups of
    sparse windows, skipped empty windows, chunked long A rows, identity
    results (exact cancellations) dropped; every schedule."""
    say("window groups", semiring, dtype, cancel)
    (ar, ac, av, m, k), (br, bc, bv, _, n) = window_structured_pair(semiring, dtype, 61, cancel)
    GA = gpu_fold(ctx, semiring, dtype, ar, ac, av, m, k)
    GB = gpu_fold(ctx, semiring, dtype, br, bc, bv, k, n)
    exp = oracle.spgemm(semiring, dtype, oracle.fold(semiring, dtype, ar, ac, av, m, k),
                        oracle.fold(semiring, dtype, br, bc, bv, k, n))
    if cancel:
        # some sums cancel to exactly zero (absent): fewer entries than the pattern
        ones_a, ones_b = np.ones(ar.size, np.uint8), np.ones(br.size, np.uint8)
        pat = oracle.spgemm("or_and", "bool", oracle.fold("or_and", "bool", ar, ac, ones_a, m, k),
                            oracle.fold("or_and", "bool", br, bc, ones_b, k, n))
        assert exp.rowptr[-1] < pat.rowptr[-1]
    for sch in range(srtc.NUM_SCHEDULES):
        check_csr(ctx.contract(semiring, "ik", GA, "kj", GB, "ij", schedule=sch), exp, semiring, dtype)


@pytest.mark.parametrize("case", ["f32_cancel", "f64_cancel_column_blocks", "i32_clamp"])
def test_spgemm_ranked_groups_with_identity_results(ctx, case):
    """Identity results inside the ranked groups of dense rows (exact
    cancellations of +-1 products, (min,+) sums clamped at the identity)
    are written in place with column -1 and dropped by the compaction that
    follows the numeric pass, also when B is cut into column blocks (the
    heavy rows' blocks are then compacted segment by segment); every
    schedule."""
    semiring, dtype = ("min_plus", "i32") if case == "i32_clamp" else ("plus_times", case[:3])
    say("ranked identity results", case)
    (ar, ac, av, m, k), (br, bc, bv, _, n) = window_structured_pair(semiring, dtype, 63, cancel=case != "i32_clamp")
    if case == "i32_clamp":
        # two-hop sums of 5e8..7e8 weights mostly reach the identity
        av = synth.edge_values("i32", ar.size, 63, 3, lo=500_000_000, hi=700_000_000)
        bv = synth.edge_values("i32", br.size, 63, 4, lo=500_000_000, hi=700_000_000)
    GA = gpu_fold(ctx, semiring, dtype, ar, ac, av, m, k)
    GB = gpu_fold(ctx, semiring, dtype, br, bc, bv, k, n)
    exp = oracle.spgemm(semiring, dtype, oracle.fold(semiring, dtype, ar, ac, av, m, k),
                        oracle.fold(semiring, dtype, br, bc, bv, k, n))
    ones_a, ones_b = np.ones(ar.size, np.uint8), np.ones(br.size, np.uint8)
    pat = oracle.spgemm("or_and", "bool", oracle.fold("or_and", "bool", ar, ac, ones_a, m, k),
                        oracle.fold("or_and", "bool", br, bc, ones_b, k, n))
    assert exp.rowptr[-1] < pat.rowptr[-1]
    c = ctx
    if case == "f64_cancel_column_blocks":
        old = os.environ.get("SRTC_COL_BLOCKS")
        os.environ["SRTC_COL_BLOCKS"] = "3"
        try:
            c = srtc.Context(0)
        finally:
            if old is None:
                os.environ.pop("SRTC_COL_BLOCKS", None)
            else:
                os.environ["SRTC_COL_BLOCKS"] = old
    for sch in range(srtc.NUM_SCHEDULES):
        say("  schedule", sch)
        check_csr(c.contract(semiring, "ik", GA, "kj", GB, "ij", schedule=sch), exp, semiring, dtype)


def wide_window_pair(semiring, dtype, seed):
    """A (8 x 1024) times B (1024 x 1,310,928): every B row holds one entry in
    each 8192-column stretch (160 of them, the last ragged), so a row of the
    product spreads its products thinly over 40 to 320 dense windows
    depending on the window width -- more than a ranked group may span (at
    most 32 windows).  A's rows of 1, 5, 40 and 200 entries make runs that end
    at the span limit, at the product cap of a group, or hold one product per
    window; a row of 600 entries (longer than a block) and an empty row take
    the other paths."""
    rng = np.random.default_rng(seed)
    k, n, S = 1024, 160 * 8192 + 208, 8192
    b_rows, b_cols = [], []
    for r in range(k):
        cols = np.arange(160) * S + (r * 37 + np.arange(160) * 11) % S
        cols = np.unique(np.append(cols, n - 1 - (r % 200)))
        b_rows.append(np.full(cols.size, r)), b_cols.append(cols)
    a_rows, a_cols = [], []
    sizes = [1, 5, 40, 200, 600, 0, 3, 120]
    for i, c in enumerate(sizes):
        cols = np.sort(rng.choice(k, size=c, replace=False))
        a_rows.append(np.full(c, i)), a_cols.append(cols)
    ar, ac = np.concatenate(a_rows), np.concatenate(a_cols)
    br, bc = np.concatenate(b_rows), np.concatenate(b_cols)
    av, bv = values(semiring, dtype, ar.size, seed, 1), values(semiring, dtype, br.size, seed, 2)
    return (ar, ac, av, len(sizes), k), (br, bc, bv, k, n)


@pytest.mark.parametrize("semiring,dtype", [("plus_times", "f64"), ("plus_times", "f32"), ("min_plus", "i32"),
                                            ("max_times", "f64"), ("or_and", "bool")])
def test_spgemm_groups_past_the_span_limit(ctx, semiring, dtype):
    """Ranked groups cut at their window-span limit and at their product
    cap, then continued, over more than 30 windows of the widest window;
    every schedule."""
    say("wide windows", semiring, dtype)
    (ar, ac, av, m, k), (br, bc, bv, _, n) = wide_window_pair(semiring, dtype, 62)
    GA = gpu_fold(ctx, semiring, dtype, ar, ac, av, m, k)
    GB = gpu_fold(ctx, semiring, dtype, br, bc, bv, k, n)
    exp = oracle.spgemm(semiring, dtype, oracle.fold(semiring, dtype, ar, ac, av, m, k),
                        oracle.fold(semiring, dtype, br, bc, bv, k, n))
    assert np.diff(exp.rowptr).max() > 30 * 1000
    for sch in range(srtc.NUM_SCHEDULES):
        check_csr(ctx.contract(semiring, "ik", GA, "kj", GB, "ij", schedule=sch), exp, semiring, dtype)


def test_spgemm_star_and_identity(ctx):
    say("star / identity")
    L = 3000
    hub = np.zeros(L, np.int64)
    leaves = np.arange(1, L + 1)
    rows = np.concatenate([hub, leaves])
    cols = np.concatenate([leaves, hub])
    G = gpu_fold(ctx, "plus_times", "f64", rows, cols, np.ones(2 * L), L + 1, L + 1)
    C = ctx.contract("plus_times", "ik", G, "kj", G, "ij", schedule=0)
    rp, col, val = C.to_host()
    assert C.nnz == L * L + 1 and col[0] == 0 and val[0] == L and np.all(val[1:] == 1.0)
    # identity (x) A == A, bit-exact even for fp (one term per entry)
    src, dst = synth.er_edges(700, 7, seed=21)
    A, _ = pair_inputs(ctx, "plus_times", "f32", src, dst, 700, 21)
    I = gpu_fold(ctx, "plus_times", "f32", np.arange(700), np.arange(700), np.ones(700, np.float32), 700, 700)
    for X in (ctx.contract("plus_times", "ik", I, "kj", A, "ij"), ctx.contract("plus_times", "ik", A, "kj", I, "ij")):
        for a, b in zip(X.to_host(), A.to_host()):
            assert np.array_equal(a, b)


def test_spgemm_empty_and_rectangular(ctx):
    say("empty / rectangular")
    E = gpu_fold(ctx, "min_plus", "i32", [], [], np.zeros(0, np.int32), 40, 30)
    B = gpu_fold(ctx, "min_plus", "i32", [0, 5, 29], [1, 2, 3], np.array([1, 2, 3], np.int32), 30, 50)
    C = ctx.contract("min_plus", "ik", E, "kj", B, "ij")
    assert C.nnz == 0 and C.shape == (40, 50)
    key = synth.stream_key(31, 0)
    r = synth.randint(key, 900, 0, 59)
    c = synth.randint(synth.stream_key(31, 1), 900, 0, 16)
    v = values("min_plus", "i32", 900, 31)
    A = gpu_fold(ctx, "min_plus", "i32", r, c, v, 60, 17)
    OA = oracle.fold("min_plus", "i32", r, c, v, 60, 17)
    r2 = synth.randint(synth.stream_key(31, 2), 300, 0, 16)
    c2 = synth.randint(synth.stream_key(31, 3), 300, 0, 99)
    v2 = values("min_plus", "i32", 300, 32)
    B = gpu_fold(ctx, "min_plus", "i32", r2, c2, v2, 17, 100)
    OB = oracle.fold("min_plus", "i32", r2, c2, v2, 17, 100)
    check_csr(ctx.contract("min_plus", "ik", A, "kj", B, "ij"), oracle.spgemm("min_plus", "i32", OA, OB),
              "min_plus", "i32")


def test_spgemm_drops_identity_results(ctx):
    # (+,x): a row whose two products cancel to exactly 0 is dropped
    say("identity results dropped")
    A = gpu_fold(ctx, "plus_times", "f64", [0, 0, 1], [0, 1, 1], np.array([1.0, 1.0, 2.0]), 2, 2)
    B = gpu_fold(ctx, "plus_times", "f64", [0, 1], [0, 0], np.array([3.0, -3.0]), 2, 1)
    for sch in range(srtc.NUM_SCHEDULES):
        C = ctx.contract("plus_times", "ik", A, "kj", B, "ij", schedule=sch)
        rp, col, val = C.to_host()
        assert rp.tolist() == [0, 0, 1] and col.tolist() == [0] and val.tolist() == [-6.0]


def test_spgemm_drops_identities_with_empty_rows(ctx):
    # Most output rows are empty (in no bin) and many results cancel to 0, so
    # the compaction after the numeric pass must see 0 outputs for every
    # empty row, whatever the recycled scratch memory held before.
    say("identity drops with empty rows")
    n = 3000
    rng_rows = np.arange(1, n, 2)
    rows = np.repeat(rng_rows, 2)
    cols = np.tile([0, 1], rng_rows.size)
    vals = np.tile([1.0, 1.0], rng_rows.size)
    A = gpu_fold(ctx, "plus_times", "f64", rows, cols, vals, n, n)
    Ah = oracle.fold("plus_times", "f64", rows, cols, vals, n, n)
    # B: rows 0 and 1 cancel on columns 0..99 and agree on 100..149
    bc = np.concatenate([np.arange(150), np.arange(150)])
    br = np.concatenate([np.zeros(150, np.int64), np.ones(150, np.int64)])
    bv = np.concatenate([np.full(150, 3.0), np.concatenate([np.full(100, -3.0), np.full(50, 2.0)])])
    B = gpu_fold(ctx, "plus_times", "f64", br, bc, bv, n, n)
    Bh = oracle.fold("plus_times", "f64", br, bc, bv, n, n)
    exp = oracle.spgemm("plus_times", "f64", Ah, Bh)
    assert exp.rowptr[-1] == 50 * rng_rows.size
    for sch in range(srtc.NUM_SCHEDULES):
        junk = [torch.full((n * 8,), 0x55, dtype=torch.uint8, device="cuda") for _ in range(8)]
        del junk
        check_csr(ctx.contract("plus_times", "ik", A, "kj", B, "ij", schedule=sch), exp, "plus_times", "f64")


def test_spgemm_accumulate_path_doubling(ctx):
    # APSP of the 64-vertex instance: (I (+) A)^n by ceil(log2 n) rounds of
    # P (+)= P (x) P, against Floyd-Warshall
    say("path doubling")
    n = 64
    src, dst = synth.er_edges(n, 8, synth.SEED_CFG0)
    w = synth.edge_values("i32", src.size, synth.SEED_CFG0, lo=1, hi=100)
    rows = np.concatenate([dst, np.arange(n)])
    cols = np.concatenate([src, np.arange(n)])
    vals = np.concatenate([w, np.zeros(n, np.int32)]).astype(np.int32)
    P = gpu_fold(ctx, "min_plus", "i32", rows, cols, vals, n, n)
    l = 1
    while l < n:
        Q = srtc.CSR(P.rowptr.clone(), P.col.clone(), P.val.clone(), P.dims, 1)
        P = ctx.contract("min_plus", "ik", Q, "kj", Q, "ij", C=P, accumulate=True)
        l <<= 1
    D = np.full((n, n), INF, dtype=np.int64)
    np.minimum.at(D, (dst, src), w.astype(np.int64))
    np.fill_diagonal(D, 0)
    FW = oracle.floyd_warshall(D)
    rp, col, val = P.to_host()
    got = np.full((n, n), INF, dtype=np.int64)
    for i in range(n):
        got[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    assert np.array_equal(got, FW)


# ------------------------------------------------------------ cfg0 (ER 4096) --
def test_er4096_tropical_square_and_bellman_ford(ctx):
    say("ER 4096 (min,+)")
    n = 4096
    src, dst = synth.er_edges(n, 8, synth.SEED_CFG0)
    w = synth.edge_values("i32", src.size, synth.SEED_CFG0, lo=1, hi=100)
    G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    for sch in range(srtc.NUM_SCHEDULES):
        check_csr(ctx.contract("min_plus", "ik", G, "kj", G, "ij", schedule=sch), oracle.spgemm("min_plus", "i32", O, O),
                  "min_plus", "i32")
    # one Bellman-Ford relaxation step from vertex 0: P1 = P0 (+) A (x) P0
    P0 = np.full((n, 1), INF, np.int32)
    P0[0] = 0
    X = torch.as_tensor(P0, device="cuda")
    Y = X.clone()
    ctx.contract("min_plus", "ij", G, "jk", X, "ik", C=Y, accumulate=True)
    exp, _ = oracle.spmm("min_plus", "i32", O, P0, self_term=True)
    assert np.array_equal(Y.cpu().numpy(), exp)
    # the fixpoint: iterates and count as the oracle, distances as Dijkstra
    X = torch.as_tensor(P0, device="cuda")
    iters = ctx.fixpoint("min_plus", G, X, steps_per_check=4)
    Pexp, it_exp, conv = oracle.bellman_ford("min_plus", "i32", O, P0)
    assert conv and iters == it_exp
    assert np.array_equal(X.cpu().numpy(), Pexp)
    Dj = oracle.dijkstra(O, [0])
    assert np.array_equal(X.cpu().numpy().astype(np.int64), Dj)


# ------------------------------------------------------------------ SpMM --
@pytest.mark.parametrize("semiring,dtype", PAIRS)
@pytest.mark.parametrize("width", [1, 8, 64, 100, 300])
def test_spmm_parity(ctx, semiring, dtype, width):
    say("spmm", semiring, dtype, width)
    src, dst = synth.rmat_edges(12, 16, 0.57, 0.19, 0.19, seed=77)   # rows up to ~1k nonzeros (split items)
    n = 1 << 12
    G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, 77)
    key = synth.stream_key(77, 5)
    X = values(semiring, dtype, n * width, 78).reshape(n, width)
    absent = synth.uniform_f64(key, n * width).reshape(n, width) < 0.3
    X = np.where(absent, np.asarray(oracle.default_add_id(semiring, dtype), dtype=X.dtype), X)
    Xd = torch.as_tensor(np.ascontiguousarray(X), device="cuda")
    Y = torch.empty_like(Xd)
    ctx.contract(semiring, "ik", G, "kj", Xd, "ij", C=Y)
    exp, _ = oracle.spmm(semiring, dtype, O, X)
    got = Y.cpu().numpy()
    if (semiring, dtype) in RTOL:
        err = np.abs(got.astype(np.float64) - exp)
        assert np.all(err <= RTOL[(semiring, dtype)] * np.abs(exp))
    else:
        assert np.array_equal(got, exp)


def test_tensor_fold_contraction(ctx):
    # T["ijk"] * M["kl"] -> C["ijl"] with T sparse COO (folded on the fly)
    for dims, p, L in (((40, 30, 50), 0.02, 16), ((512, 512, 512), 1e-3, 64)):
        say("tensor contraction", dims)
        keys = synth.bernoulli_keys(dims, p, seed=synth.SEED_CFG1, tag=1)
        tv = synth.uniform_f32(synth.stream_key(synth.SEED_CFG1, 11), keys.size)
        M = synth.uniform_f32(synth.stream_key(synth.SEED_CFG1, 12), dims[2] * L).reshape(dims[2], L)
        T = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(tv, device="cuda"), dims)
        C = torch.empty((dims[0], dims[1], L), dtype=torch.float32, device="cuda")
        ctx.contract("plus_times", "ijk", T, "kl", torch.as_tensor(M, device="cuda"), "ijl", C=C)
        F = oracle.fold_tensor("plus_times", "f32", keys, tv, dims, "ijk", "ij", "k")
        exp, _ = oracle.spmm("plus_times", "f32", F, M)
        got = C.cpu().numpy().reshape(dims[0] * dims[1], L).astype(np.float64)
        assert np.all(np.abs(got - exp) <= 1e-5 * np.abs(exp))


# ------------------------------------------------------- fixpoints / BFS --
def test_multi_source_bellman_ford_and_bfs(ctx):
    say("multi-source BF / BFS")
    scale = 14
    n = 1 << scale
    src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, seed=synth.SEED_CFG2)
    w = synth.edge_values("i32", src.size, synth.SEED_CFG2, lo=1, hi=255)
    G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    sources = synth.pick_sources(n, src, 64, synth.SEED_CFG2)
    P0 = np.full((n, 64), INF, np.int32)
    P0[sources, np.arange(64)] = 0
    X = torch.as_tensor(P0, device="cuda")
    it = ctx.fixpoint("min_plus", G, X, steps_per_check=4)
    Pexp, it_exp, conv = oracle.bellman_ford("min_plus", "i32", O, P0)
    assert conv and it == it_exp
    assert np.array_equal(X.cpu().numpy(), Pexp)
    assert np.array_equal(Pexp.astype(np.int64), oracle.dijkstra(O, sources))
    # gathers from changed rows only: same iterates, same result
    X2 = torch.as_tensor(P0, device="cuda")
    assert ctx.fixpoint("min_plus", G, X2, steps_per_check=4, changed_rows_only=True) == it_exp
    assert np.array_equal(X2.cpu().numpy(), Pexp)
    for cap in (1, 3, 6):
        Xc = torch.as_tensor(P0, device="cuda")
        with pytest.raises(srtc.NotConverged):
            ctx.fixpoint("min_plus", G, Xc, max_iters=cap, steps_per_check=4, changed_rows_only=True)
        expc, _, _ = oracle.bellman_ford("min_plus", "i32", O, P0, max_iters=cap)
        assert np.array_equal(Xc.cpu().numpy(), expc), cap
    lev, depth = ctx.bfs_levels(G, sources)
    exp = oracle.bfs_levels(O, sources)
    assert np.array_equal(lev.cpu().numpy(), exp) and depth == exp.max()


def test_fixpoint_not_converged_and_cap(ctx):
    say("negative cycle / cap")
    # 0 -> 1 -> 2 -> 0 with total weight -3: never settles
    A = gpu_fold(ctx, "min_plus", "i32", [1, 2, 0], [0, 1, 2], np.array([1, 1, -5], np.int32), 3, 3)
    X = torch.as_tensor(np.array([[0], [INF], [INF]], np.int32), device="cuda")
    with pytest.raises(srtc.NotConverged) as e:
        ctx.fixpoint("min_plus", A, X)
    assert e.value.iters == 3
    X = torch.as_tensor(np.array([[0], [INF], [INF]], np.int32), device="cuda")
    with pytest.raises(srtc.NotConverged) as e:
        ctx.fixpoint("min_plus", A, X, changed_rows_only=True)
    assert e.value.iters == 3
    # path graph with a cap below its n steps
    n = 50
    P = gpu_fold(ctx, "min_plus", "i32", np.arange(1, n), np.arange(n - 1), np.ones(n - 1, np.int32), n, n)
    X = torch.full((n, 1), INF, dtype=torch.int32, device="cuda")
    X[0] = 0
    with pytest.raises(srtc.NotConverged):
        ctx.fixpoint("min_plus", P, X, max_iters=7, steps_per_check=4)
    O = oracle.fold("min_plus", "i32", np.arange(1, n), np.arange(n - 1), np.ones(n - 1, np.int32), n, n)
    X0 = np.full((n, 1), INF, np.int32)
    X0[0] = 0
    exp, _, _ = oracle.bellman_ford("min_plus", "i32", O, X0, max_iters=7)
    assert np.array_equal(X.cpu().numpy(), exp)
    X = torch.full((n, 1), INF, dtype=torch.int32, device="cuda")
    X[0] = 0
    assert ctx.fixpoint("min_plus", P, X, steps_per_check=6) == n


# ------------------------------------------------------------- MFMA tile --
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dense_mfma(ctx, dtype):
    say("dense mfma", dtype)
    for (M, N, K) in ((16, 16, 4), (100, 70, 300), (257, 129, 1000), (640, 384, 517), (128, 128, 16)):
        a = synth.uniform_f64(synth.stream_key(5, M), M * K).reshape(M, K)
        b = synth.uniform_f64(synth.stream_key(6, N), K * N).reshape(K, N)
        if dtype == "f32":
            a, b = a.astype(np.float32), b.astype(np.float32)
        C = torch.zeros((M, N), dtype=TORCH[dtype], device="cuda")
        ctx.contract("plus_times", "ik", torch.as_tensor(a, device="cuda"), "kj", torch.as_tensor(b, device="cuda"),
                     "ij", C=C)
        ref = oracle.dense_plus_times(a, b)   # non-negative terms
        tol = 1e-12 if dtype == "f64" else 1e-5
        assert np.all(np.abs(C.cpu().numpy().astype(np.float64) - ref) <= tol * ref)
        # accumulate: the old C joins the sum
        ctx.contract("plus_times", "ik", torch.as_tensor(a, device="cuda"), "kj", torch.as_tensor(b, device="cuda"),
                     "ij", C=C, accumulate=True)
        assert np.all(np.abs(C.cpu().numpy().astype(np.float64) - 2 * ref) <= 2 * tol * ref)


# ----------------------------------------------------------------- batch --
def test_batch_contract_and_fixpoint(ctx):
    say("batch")
    ns = [1, 200, 1500, 64, 3000, 0 + 1, 900]
    As, Os, srcs = [], [], []
    for b, n in enumerate(ns):
        src, dst = synth.er_edges(n, 6, seed=1000 + b)
        w = synth.edge_values("i32", src.size, 1000 + b, lo=1, hi=100)
        As.append(gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n))
        Os.append(oracle.fold("min_plus", "i32", dst, src, w, n, n))
        srcs.append(src)
    Cs = ctx.batch_contract("min_plus", As, As)
    for C, O in zip(Cs, Os):
        check_csr(C, oracle.spgemm("min_plus", "i32", O, O), "min_plus", "i32")
    Xs, P0s = [], []
    for b, n in enumerate(ns):
        P0 = np.full((n, 8), INF, np.int32)
        s = synth.pick_sources(n, srcs[b], 8, 2000 + b)
        P0[s, np.arange(s.size)] = 0
        P0s.append(P0)
        Xs.append(torch.as_tensor(P0, device="cuda"))
    iters = ctx.batch_fixpoint("min_plus", As, Xs, steps_per_check=4)
    for X, O, P0, it in zip(Xs, Os, P0s, iters):
        exp, it_exp, conv = oracle.bellman_ford("min_plus", "i32", O, P0)
        assert conv and it == it_exp
        assert np.array_equal(X.cpu().numpy(), exp)


def test_batch_autotune_one_schedule_for_the_batch():
    """The batch tuner times every schedule on the whole batch (as
    batch_contract forms it with one schedule) and caches the winner: a
    later batch_contract of the same batch without schedules takes it, and
    its results equal the oracle's and those of the winner given
    explicitly (bit-exact over (min,+)); malformed batches are refused."""
    say("batch autotune")
    c = srtc.Context(0)
    ns = [300, 2500, 40, 1200, 4000, 900, 64, 1800]
    As, Os = [], []
    for b, n in enumerate(ns):
        src, dst = synth.er_edges(n, 8, seed=3000 + b)
        w = synth.edge_values("i32", src.size, 3000 + b, lo=1, hi=100)
        As.append(gpu_fold(c, "min_plus", "i32", dst, src, w, n, n))
        Os.append(oracle.fold("min_plus", "i32", dst, src, w, n, n))
    best, times = c.batch_autotune("min_plus", As, As, reps=3)
    say("  batch schedule", best, "times", np.round(times, 3))
    assert 0 <= best < srtc.NUM_SCHEDULES
    assert (times > 0).all() and times[best] == times.min()
    chosen = c.batch_contract("min_plus", As, As)
    given = c.batch_contract("min_plus", As, As, schedules=[best] * len(As))
    for C, G, O in zip(chosen, given, Os):
        check_csr(C, oracle.spgemm("min_plus", "i32", O, O), "min_plus", "i32")
        assert torch.equal(C.rowptr, G.rowptr) and torch.equal(C.col, G.col) and torch.equal(C.val, G.val)
    with pytest.raises(srtc.SrtcError):
        c.batch_autotune("min_plus", As, As, ia="ik", ib="kj", ic="ik")


# -------------------------------------------------------------------- MLP --
def test_batch_index_strings_and_per_instance_schedules(ctx):
    """Batched C_b = A_b (x) B_b with one schedule per instance (every
    schedule id, and -1 = choose) is bit-identical to per-instance calls
    with those schedules and matches the oracle; A given transposed as COO
    ("ki","kj","ij") folds per instance to the same result."""
    ninst = 20
    As, ATs, Os, want = [], [], [], []
    scheds = [(b % (srtc.NUM_SCHEDULES + 1)) - 1 for b in range(ninst)]
    for b in range(ninst):
        n = 300 + 137 * b
        src, dst = synth.er_edges(n, 3.0 + b, 0x5EEDBA7C, tag=b)
        w = synth.edge_values("i32", src.size, 0x5EEDBA7C, tag=b, lo=1, hi=100)
        G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
        As.append(G)
        # A^T stored as (k, i) index-value pairs
        ATs.append(srtc.COO(torch.as_tensor(src.astype(np.int64) * n + dst, device="cuda"),
                            torch.as_tensor(w, device="cuda"), (n, n)))
        O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
        Os.append(oracle.spgemm("min_plus", "i32", O, O))
        want.append(ctx.contract("min_plus", "ik", G, "kj", G, "ij", schedule=max(scheds[b], 0)))
    Cs = ctx.batch_contract("min_plus", As, As, schedules=scheds)
    Ct = ctx.batch_contract("min_plus", ATs, As, ia="ki", ib="kj", ic="ij", schedule=5)
    for b in range(ninst):
        for got in (Cs[b], Ct[b]):
            g, e = got.to_host(), want[b].to_host()
            assert all(np.array_equal(x, y) for x, y in zip(g, e)), b
            check_csr(got, Os[b], "min_plus", "i32")
    with pytest.raises(srtc.SrtcError):
        ctx.batch_contract("min_plus", As[:2], As[:2], schedules=[0])
    for ia, ib, ic in (("ik", "kj", "ik"), ("ik", "kj", "ji"), ("ik", "jl", "ij"), ("ii", "kj", "ij")):
        with pytest.raises(srtc.SrtcError) as e:
            ctx.batch_contract("min_plus", As[:2], As[:2], ia=ia, ib=ib, ic=ic)
        assert e.value.status == -2


def test_mlp_gradients_match_oracle(ctx):
    say("mlp gradients")
    from oracle import mlp
    K = srtc.NUM_SCHEDULES
    P = mlp.num_params(K)
    assert P == srtc.mlp_num_params()
    key = synth.stream_key(44, 0)
    p = (synth.uniform_f64(key, P) - 0.5) * 0.4
    X = synth.uniform_f64(synth.stream_key(44, 1), 50 * 32).reshape(50, 32) * 2 - 1
    T = synth.uniform_f64(synth.stream_key(44, 2), 50 * K).reshape(50, K)
    p32, X32, T32 = p.astype(np.float32), X.astype(np.float32), T.astype(np.float32)
    loss, g = ctx.mlp_loss_grad(torch.as_tensor(p32, device="cuda"), torch.as_tensor(X32, device="cuda"),
                                torch.as_tensor(T32, device="cuda"))
    lref, gref = mlp.loss_grad(p32.astype(np.float64), X32.astype(np.float64), T32.astype(np.float64), K)
    gg = g.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - lref) <= 1e-4 * abs(lref)
    assert np.linalg.norm(gg - gref) <= 1e-4 * np.linalg.norm(gref)
    Y = ctx.mlp_forward(torch.as_tensor(p32, device="cuda"), torch.as_tensor(X32, device="cuda")).cpu().numpy()
    yref, _ = mlp.forward(p32.astype(np.float64), X32.astype(np.float64), K)
    assert np.abs(Y - yref).max() <= 1e-4 * max(1.0, np.abs(yref).max())
    z = np.zeros(P, np.float32)
    z[-K:] = np.arange(K)
    Yz = ctx.mlp_forward(torch.as_tensor(z, device="cuda"), torch.as_tensor(X32, device="cuda")).cpu().numpy()
    assert np.array_equal(Yz, np.tile(np.arange(K, dtype=np.float32), (50, 1)))


def test_selector_overfits_tiny_set(ctx, tmp_path):
    say("selector overfit")
    c2 = srtc.Context(0)
    X = synth.uniform_f32(synth.stream_key(45, 0), 16 * 32).reshape(16, 32)
    best = synth.randint(synth.stream_key(45, 1), 16, 0, srtc.NUM_SCHEDULES - 1)
    T = np.ones((16, srtc.NUM_SCHEDULES), np.float32)
    T[np.arange(16), best] = -1.0
    loss = c2.selector_train(X, T, epochs=1500, batch=16, lr=3e-3, seed=1)
    assert loss < 1e-3
    picks = [c2.select(X[i]) for i in range(16)]
    assert picks == best.tolist()
    path = str(tmp_path / "sel.bin")
    c2.selector_save(path)
    c3 = srtc.Context(0)
    c3.selector_load(path)
    assert [c3.select(X[i]) for i in range(16)] == picks


# ----------------------------------------------------------------- errors --
def test_error_statuses(ctx):
    say("error statuses")
    A = gpu_fold(ctx, "min_plus", "i32", [0], [1], np.array([1], np.int32), 3, 4)
    B = gpu_fold(ctx, "min_plus", "i32", [0], [1], np.array([1], np.int32), 4, 5)
    cases = [
        (dict(ia="ik", ib="kj", ic="ii"), -2),           # repeated index
        (dict(ia="ik", ib="kj", ic="ixj"), -2),           # length / index only in output
        (dict(ia="ik", ib="lj", ic="ij"), -2),            # index only in one operand (reduction)
        (dict(ia="ik", ib="jk", ic="ij"), -3),            # extents of k differ
    ]
    for kw, st in cases:
        with pytest.raises(srtc.SrtcError) as e:
            ctx.contract("min_plus", kw["ia"], A, kw["ib"], B, kw["ic"])
        assert e.value.status == st, kw
    # a column letter before a row letter in C is folded back, not refused
    Ct = ctx.contract("min_plus", "ik", A, "kj", B, "ji")
    assert tuple(Ct.dims) == (5, 3) and Ct.nnz == ctx.contract("min_plus", "ik", A, "kj", B, "ij").nnz
    # ... but the masked form keeps C's rows first
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract_masked("min_plus", "ik", A, "kj", B, "ji", Ct)
    assert e.value.status == -9
    F = gpu_fold(ctx, "plus_times", "f32", [0], [1], np.array([1], np.float32), 3, 4)
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract("min_plus", "ik", F, "kj", B, "ij")  # mixed value types
    assert e.value.status == -4
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract("or_and", "ik", A, "kj", B, "ij")    # int32 not defined for (or,and)
    assert e.value.status == -4
    X = torch.zeros((4, 5), dtype=torch.int32, device="cuda")
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract("min_plus", "ik", A, "kj", X, "ij", C=X[:3])   # C is a view of B
    assert e.value.status == -6


def test_validate_rejects_malformed_operands(ctx):
    # With validate=True every malformed sparse operand is reported as
    # SRTC_ERR_FORMAT before any kernel uses it (malformed operands are
    # never passed without it).
    say("validation")
    good = gpu_fold(ctx, "min_plus", "i32", [0, 0, 1, 2], [0, 2, 1, 0], np.array([1, 2, 3, 4], np.int32), 3, 3)
    C = ctx.contract("min_plus", "ik", good, "kj", good, "ij", validate=True)
    assert C.nnz > 0

    def csr(rp, col, val, dims=(3, 3)):
        return srtc.CSR(torch.tensor(rp, dtype=torch.int64, device="cuda"),
                        torch.tensor(col, dtype=torch.int32, device="cuda"),
                        torch.tensor(val, device="cuda"), dims, 1)

    bad = [
        csr([1, 2, 3, 4], [0, 1, 2, 0], np.array([1, 1, 1, 1], np.int32)),   # rowptr[0] != 0
        csr([0, 3, 2, 4], [0, 1, 2, 0], np.array([1, 1, 1, 1], np.int32)),   # rowptr decreases
        csr([0, 1, 2, 3], [0, 1, 2, 0], np.array([1, 1, 1, 1], np.int32)),   # rowptr[m] != nnz
        csr([0, 2, 3, 4], [0, 5, 2, 0], np.array([1, 1, 1, 1], np.int32)),   # column out of range
        csr([0, 2, 3, 4], [2, 0, 1, 0], np.array([1, 1, 1, 1], np.int32)),   # row not ascending
        csr([0, 2, 3, 4], [1, 1, 1, 0], np.array([1, 1, 1, 1], np.int32)),   # repeated column
    ]
    for b in bad:
        with pytest.raises(srtc.SrtcError) as e:
            ctx.contract("min_plus", "ik", b, "kj", good, "ij", validate=True)
        assert e.value.status == -5
    keys = torch.tensor([0, 4, 9], dtype=torch.int64, device="cuda")   # 9 is outside 3 x 3
    coo = srtc.COO(keys, torch.tensor([1, 1, 1], dtype=torch.int32, device="cuda"), (3, 3))
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract("min_plus", "ik", coo, "kj", good, "ij", validate=True)
    assert e.value.status == -5
    fgood = gpu_fold(ctx, "min_plus", "f32", [0, 1], [1, 0], np.array([1.0, 2.0], np.float32), 2, 2)
    fnan = csr([0, 1, 2], [1, 0], np.array([np.nan, 2.0], np.float32), (2, 2))
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract("min_plus", "ik", fnan, "kj", fgood, "ij", validate=True)
    assert e.value.status == -5


# ----------------------------------------------------------------- masked --
@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_masked_contraction(ctx, semiring, dtype):
    say("masked", semiring, dtype)
    for case, dens in (("er500", 0.02), ("rmat11", 0.01), ("rmat11", 0.2)):
        (src, dst), n = CASES[case]()
        G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, 21)
        mk = synth.bernoulli_keys((n, n), dens, seed=31, tag=len(case))
        Mo = oracle.fold("or_and", "bool", mk // n, mk % n, np.ones(mk.size, np.uint8), n, n)
        M = srtc.COO(torch.as_tensor(mk, device="cuda"), torch.ones(mk.size, dtype=torch.uint8, device="cuda"), (n, n))
        C = ctx.contract_masked(semiring, "ik", G, "kj", G, "ij", M, validate=True)
        check_csr(C, oracle.spgemm_masked(semiring, dtype, O, O, Mo), semiring, dtype)


def test_masked_contraction_edge_cases(ctx):
    say("masked edge cases")
    n = 6000
    src, dst = synth.er_edges(n, 4, seed=41)
    w = synth.edge_values("i32", src.size, 41, lo=1, hi=100)
    G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    # rows longer than one LDS chunk, duplicate mask keys, zero mask values
    long_rows = np.concatenate([r * n + np.arange(n) for r in (0, 5, 4321)])
    mk = np.concatenate([synth.bernoulli_keys((n, n), 0.002, seed=42), long_rows, long_rows[:100]])
    mv = np.zeros(mk.size, np.uint8)
    M = srtc.COO(torch.as_tensor(mk, device="cuda"), torch.as_tensor(mv, device="cuda"), (n, n))
    Mo = oracle.fold("or_and", "bool", mk // n, mk % n, np.ones(mk.size, np.uint8), n, n)
    check_csr(ctx.contract_masked("min_plus", "ik", G, "kj", G, "ij", M), oracle.spgemm_masked("min_plus", "i32", O, O, Mo),
              "min_plus", "i32")
    # an empty mask gives an empty C; a mask covering the product changes nothing
    E = srtc.COO(torch.zeros(0, dtype=torch.int64, device="cuda"), torch.zeros(0, dtype=torch.uint8, device="cuda"), (n, n))
    assert ctx.contract_masked("min_plus", "ik", G, "kj", G, "ij", E).nnz == 0
    full = ctx.contract("min_plus", "ik", G, "kj", G, "ij")
    again = ctx.contract_masked("min_plus", "ik", G, "kj", G, "ij", full)
    assert torch.equal(again.rowptr, full.rowptr) and torch.equal(again.col, full.col) and torch.equal(again.val, full.val)
