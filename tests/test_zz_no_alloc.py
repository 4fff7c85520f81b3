"""The contraction that allocates nothing (srtc_contract_noalloc) against the
allocating srtc_contract on the same inputs, and both against the oracle.

The two entry points run the same sparse x dense kernels; only where the
work-item plan lives differs (the library's fixed per-device buffer instead
of allocator memory), so their outputs must agree bit for bit.  Every test
makes two calls in a row, the second with a smaller input, so the second
plan is laid over the first one's leftovers in the shared buffer."""

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import PAIRS, RTOL, pair_inputs, say, values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return srtc.Context(0)


def _dense(semiring, dtype, rows, width, seed):
    X = values(semiring, dtype, rows * width, seed).reshape(rows, width)
    absent = synth.uniform_f64(synth.stream_key(seed, 5), rows * width).reshape(rows, width) < 0.3
    return np.where(absent, np.asarray(oracle.default_add_id(semiring, dtype), dtype=X.dtype), X)


def _check_oracle(got, exp, semiring, dtype):
    if (semiring, dtype) in RTOL:
        err = np.abs(got.astype(np.float64) - exp)
        assert np.all(err <= RTOL[(semiring, dtype)] * np.abs(exp))
    else:
        assert np.array_equal(got, exp.astype(got.dtype))


@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_noalloc_matches_contract_twice(ctx, semiring, dtype):
    # first call: R-MAT 12 (rows up to ~1k nonzeros, split into several work
    # items) times 100 columns (two column chunks); second: R-MAT 10 times 8
    for scale, width, seed in ((12, 100, 91), (10, 8, 92)):
        say("noalloc", semiring, dtype, "scale", scale, "width", width)
        n = 1 << scale
        src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, seed=seed)
        G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, seed)
        X = _dense(semiring, dtype, n, width, seed + 100)
        Xd = torch.as_tensor(np.ascontiguousarray(X), device="cuda")
        Y0 = torch.empty_like(Xd)
        Y1 = torch.full_like(Xd, 7)  # stale values the call must overwrite
        ctx.contract(semiring, "ik", G, "kj", Xd, "ij", C=Y0)
        before = ctx.allocations
        ctx.contract_noalloc(semiring, "ik", G, "kj", Xd, "ij", Y1)
        assert ctx.allocations == before, "the no-allocation call asked the allocator for memory"
        torch.cuda.synchronize()
        assert torch.equal(Y0, Y1)
        exp, _ = oracle.spmm(semiring, dtype, O, X)
        _check_oracle(Y1.cpu().numpy(), exp, semiring, dtype)
        # accumulate: C (+)= A (x) X on a C that already holds values
        Cinit = _dense(semiring, dtype, n, width, seed + 200)
        Z0 = torch.as_tensor(np.ascontiguousarray(Cinit), device="cuda")
        Z1 = Z0.clone()
        ctx.contract(semiring, "ik", G, "kj", Xd, "ij", C=Z0, accumulate=True)
        ctx.contract_noalloc(semiring, "ik", G, "kj", Xd, "ij", Z1, accumulate=True)
        torch.cuda.synchronize()
        assert torch.equal(Z0, Z1)


def test_noalloc_letter_orders_and_empty_rows(ctx):
    # order-3 A (rows "ab", inner "k") and a B with two column letters
    semiring, dtype = "min_plus", "i32"
    dims = (24, 40, 300)
    keys = synth.bernoulli_keys(dims, 0.05, seed=synth.SEED_CFG1, tag=7)
    v = synth.edge_values("i32", keys.size, synth.SEED_CFG1, tag=7, lo=1, hi=100)
    T = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(v, device="cuda"), dims)
    A = ctx.fold(semiring, T, "abk", "ab", "k")
    Bh = _dense(semiring, dtype, 300, 6 * 5, 93).reshape(300, 6, 5)
    B = torch.as_tensor(np.ascontiguousarray(Bh), device="cuda")
    C0 = torch.empty((24, 40, 6, 5), dtype=torch.int32, device="cuda")
    C1 = torch.empty_like(C0)
    ctx.contract(semiring, "abk", A, "kcd", B, "abcd", C=C0)
    ctx.contract_noalloc(semiring, "abk", A, "kcd", B, "abcd", C1)
    torch.cuda.synchronize()
    assert torch.equal(C0, C1)
    F = oracle.fold_tensor(semiring, dtype, keys, v, dims, "abk", "ab", "k")
    exp, _ = oracle.spmm(semiring, dtype, F, Bh.reshape(300, 30))
    assert np.array_equal(C1.cpu().numpy().reshape(24 * 40, 30), exp.astype(np.int32))
    # no entries at all: every output is the additive identity, and with
    # accumulate C is left as it was
    E = srtc.csr_from_host(np.zeros(17, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), (16, 9))
    Xe = torch.ones((9, 3), dtype=torch.float32, device="cuda")
    Ye = torch.zeros((16, 3), dtype=torch.float32, device="cuda")
    ctx.contract_noalloc("min_plus", "ik", E, "kj", Xe, "ij", Ye)
    torch.cuda.synchronize()
    assert torch.all(torch.isinf(Ye))
    Ye.fill_(2.5)
    ctx.contract_noalloc("min_plus", "ik", E, "kj", Xe, "ij", Ye, accumulate=True)
    torch.cuda.synchronize()
    assert torch.all(Ye == 2.5)


def test_noalloc_rejections(ctx):
    src, dst = synth.rmat_edges(8, 8, 0.57, 0.19, 0.19, seed=94)
    G, _ = pair_inputs(ctx, "plus_times", "f64", src, dst, 256, 94)
    X = torch.ones((256, 4), dtype=torch.float64, device="cuda")
    Y = torch.empty((256, 4), dtype=torch.float64, device="cuda")
    # layouts that need a rearrangement (scratch) are left to srtc_contract
    for ia, ib, ic, Bt, Ct in (("ki", "kj", "ij", X, Y), ("ik", "jk", "ij", X.t().contiguous(), Y),
                               ("ik", "kj", "ji", X, Y.t().contiguous())):
        with pytest.raises(srtc.SrtcError) as e:
            ctx.contract_noalloc("plus_times", ia, G, ib, Bt, ic, Ct)
        assert e.value.status == -9, (ia, ib, ic)
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract_noalloc("plus_times", "ik", G, "kj", X, "ij", X)
    assert e.value.status == -6
    # a plan larger than the fixed buffer: 2^21 rows need about 120 MB
    m = 1 << 21
    Big = srtc.CSR(torch.zeros(m + 1, dtype=torch.int64, device="cuda"), torch.zeros(0, dtype=torch.int32,
                   device="cuda"), torch.zeros(0, dtype=torch.float32, device="cuda"), (m, 4))
    Xb = torch.ones((4, 1), dtype=torch.float32, device="cuda")
    Yb = torch.empty((m, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract_noalloc("plus_times", "ik", Big, "kj", Xb, "ij", Yb)
    assert e.value.status == -11 and "fixed buffer" in e.value.message
    # the context is still usable after a rejection
    ctx.contract_noalloc("plus_times", "ik", G, "kj", X, "ij", Y)
    Y2 = torch.empty_like(Y)
    ctx.contract("plus_times", "ik", G, "kj", X, "ij", C=Y2)
    torch.cuda.synchronize()
    assert torch.equal(Y, Y2)


def test_noalloc_replayed_from_a_graph(ctx):
    """Captured into a HIP graph (where nothing may be allocated) and
    replayed three times, with eager work between the replays: every replay
    equals the eager result."""
    semiring, dtype = "max_times", "f32"
    n = 1 << 11
    src, dst = synth.rmat_edges(11, 16, 0.57, 0.19, 0.19, seed=95)
    G, _ = pair_inputs(ctx, semiring, dtype, src, dst, n, 95)
    X = torch.as_tensor(np.ascontiguousarray(_dense(semiring, dtype, n, 16, 96)), device="cuda")
    Y_eager = torch.empty_like(X)
    ctx.contract_noalloc(semiring, "ik", G, "kj", X, "ij", Y_eager)
    torch.cuda.synchronize()
    Y = torch.zeros_like(X)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        before = ctx.allocations
        with torch.cuda.graph(g, stream=s):
            ctx.contract_noalloc(semiring, "ik", G, "kj", X, "ij", Y)
        assert ctx.allocations == before
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        Y.zero_()
        # eager use of the same buffer between replays
        Z = torch.empty_like(X)
        ctx.contract_noalloc(semiring, "ik", G, "kj", X[:, :8].contiguous(), "ij", Z[:, :8].contiguous())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, Y_eager), rep
