"""Semiring edge semantics and failure paths on the GPU, against the oracle.

* Tropical sums reaching the additive identity (Section 3.1: the identity is
  INT_MAX/2 so that two identities add without overflow): int32 weights
  near 6e8 make most two-hop sums cross INT32_MAX/2; they are absent in a
  sparse result and stored as the identity in a dense one, in SpGEMM (every
  schedule), SpMM and the Bellman-Ford fixpoint.
* Identities other than the default: (max,x) with -inf on signed values,
  (min,+) int32 with a small identity.
* C (+)= A (x) B with the old C seeding the accumulators, every pair.
* fp32 dense x dense on the matrix cores with signed data, against the error
  model of 128-term fp32 partial sums.
* Failure paths forced from the host: an allocator that runs dry
  (SRTC_ERR_OOM, nothing leaked), a small SRTC_LDS_BUDGET (identical
  results), SRTC_FORCE_SCHEDULE, SRTC_VALIDATE and malformed switches.
"""

import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import PAIRS, check_csr, gpu_fold, pair_inputs, say, values

pytestmark = pytest.mark.gpu

SEED = 0x5EED2000
ID = oracle.INT_INF


@pytest.fixture(scope="module")
def ctx():
    return srtc.Context(0)


def heavy_weight_graph(n, d, tag):
    src, dst = synth.er_edges(n, d, SEED, tag=tag)
    w = synth.edge_values("i32", src.size, SEED, tag, lo=500_000_000, hi=700_000_000)
    return src, dst, w


def test_tropical_sums_reaching_the_identity_spgemm(ctx):
    n = 3000
    src, dst, w = heavy_weight_graph(n, 12.0, 1)
    G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    exp = oracle.spgemm("min_plus", "i32", O, O)
    full = np.diff(O.rowptr)
    products = int(full[O.col].sum())
    # most two-hop sums are >= the identity: they must all be absent
    say("tropical clamp: products", products, "kept", exp.nnz)
    assert 0 < exp.nnz < products // 2
    for sch in range(srtc.NUM_SCHEDULES):
        say("  schedule", sch)
        check_csr(ctx.contract("min_plus", "ik", G, "kj", G, "ij", schedule=sch), exp, "min_plus", "i32")


@pytest.mark.parametrize("width", [1, 8, 64])
def test_tropical_sums_reaching_the_identity_spmm(ctx, width):
    n = 3000
    src, dst, w = heavy_weight_graph(n, 12.0, 2)
    G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    X = synth.edge_values("i32", n * width, SEED, 3, lo=300_000_000, hi=700_000_000).reshape(n, width)
    X[synth.permutation(synth.stream_key(SEED, 4), n)[: n // 3]] = ID
    Y = torch.empty((n, width), dtype=torch.int32, device="cuda")
    ctx.contract("min_plus", "ik", G, "kj", torch.as_tensor(X, device="cuda"), "ij", C=Y)
    exp, _ = oracle.spmm("min_plus", "i32", O, X)
    got = Y.cpu().numpy()
    assert got.max() <= ID and (got == ID).any() and (got < ID).any()
    assert np.array_equal(got, exp)


def test_tropical_sums_reaching_the_identity_fixpoint(ctx):
    n = 3000
    src, dst, w = heavy_weight_graph(n, 6.0, 5)
    G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
    sources = synth.pick_sources(n, src, 8, SEED, tag=5)
    P0 = np.full((n, 8), ID, np.int32)
    P0[sources, np.arange(8)] = 0
    X = torch.as_tensor(P0, device="cuda")
    it = ctx.fixpoint("min_plus", G, X, steps_per_check=4)
    Pexp, it_exp, conv = oracle.bellman_ford("min_plus", "i32", O, P0)
    assert conv and it == it_exp
    got = X.cpu().numpy()
    # one hop is below the identity, some two-hop paths are, no longer one is
    assert got.max() == ID and np.array_equal(got, Pexp)


def test_non_default_identities(ctx):
    # (max,x) with -inf on signed values in [-1, 1): negative products are
    # ordinary values, only -inf is absent
    n = 400
    src, dst = synth.er_edges(n, 10.0, SEED, tag=7)
    for dt in ("f32", "f64"):
        v = (synth.edge_values(dt, src.size, SEED, 8) * 2 - 1).astype(oracle.NP_DTYPES[dt])
        keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
        G = ctx.fold("max_times", srtc.COO(keys, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j",
                     add_id=-np.inf)
        O = oracle.fold("max_times", dt, dst, src, v, n, n, add_id=-np.inf)
        assert np.array_equal(G.to_host()[2], O.val)
        exp = oracle.spgemm("max_times", dt, O, O, add_id=-np.inf)
        assert (exp.val < 0).any()
        for sch in range(srtc.NUM_SCHEDULES):
            say("(max,x) -inf", dt, "schedule", sch)
            check_csr(ctx.contract("max_times", "ik", G, "kj", G, "ij", schedule=sch, add_id=-np.inf), exp,
                      "max_times", dt)
        X = (synth.edge_values(dt, n * 8, SEED, 9) * 2 - 1).astype(oracle.NP_DTYPES[dt]).reshape(n, 8)
        X[::5] = -np.inf
        Y = torch.empty((n, 8), dtype=srtc._DT_TO_TORCH[srtc.F64 if dt == "f64" else srtc.F32], device="cuda")
        ctx.contract("max_times", "ik", G, "kj", torch.as_tensor(X, device="cuda"), "ij", C=Y, add_id=-np.inf)
        ey, _ = oracle.spmm("max_times", dt, O, X, add_id=-np.inf)
        assert np.array_equal(Y.cpu().numpy(), ey.astype(oracle.NP_DTYPES[dt]))
    # (min,+) int32 with identity 1000 and weights in [1, 600]: sums of 1000
    # or more are absent
    w = synth.edge_values("i32", src.size, SEED, 10, lo=1, hi=600)
    G = gpu_fold(ctx, "min_plus", "i32", dst, src, w, n, n)
    O = oracle.fold("min_plus", "i32", dst, src, w, n, n, add_id=1000)
    exp = oracle.spgemm("min_plus", "i32", O, O, add_id=1000)
    assert exp.val.max() < 1000
    for sch in (0, 4, 5):
        check_csr(ctx.contract("min_plus", "ik", G, "kj", G, "ij", schedule=sch, add_id=1000), exp, "min_plus", "i32")
    # identities outside the allowed range are refused
    for bad in (0, -5, 2 ** 30 + 5):
        with pytest.raises(srtc.SrtcError) as e:
            ctx.contract("min_plus", "ik", G, "kj", G, "ij", add_id=bad)
        assert e.value.status == -1


@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_accumulate_seeds_the_product(ctx, semiring, dtype):
    # C_new = C_old (+) A (x) B with C_old overlapping the product's pattern
    # in part; rectangular, some empty rows
    m, k, n = 300, 200, 250
    src, dst = synth.er_edges(max(m, k), 6.0, SEED, tag=20)
    sel = (dst < m) & (src < k)
    A = (dst[sel], src[sel], values(semiring, dtype, int(sel.sum()), SEED, 21))
    src2, dst2 = synth.er_edges(max(k, n), 6.0, SEED, tag=22)
    sel2 = (dst2 < k) & (src2 < n)
    B = (dst2[sel2], src2[sel2], values(semiring, dtype, int(sel2.sum()), SEED, 23))
    src3, dst3 = synth.er_edges(max(m, n), 4.0, SEED, tag=24)
    sel3 = (dst3 < m) & (src3 < n) & (dst3 % 7 != 3)
    Cv = (dst3[sel3], src3[sel3], values(semiring, dtype, int(sel3.sum()), SEED, 25))
    GA = gpu_fold(ctx, semiring, dtype, *A, m, k)
    GB = gpu_fold(ctx, semiring, dtype, *B, k, n)
    OA = oracle.fold(semiring, dtype, *A, m, k)
    OB = oracle.fold(semiring, dtype, *B, k, n)
    OC = oracle.fold(semiring, dtype, *Cv, m, n)
    exp = oracle.spgemm(semiring, dtype, OA, OB, C_old=OC)
    for sch in (0, 2, 4, 5):
        GC = gpu_fold(ctx, semiring, dtype, *Cv, m, n)
        say("accumulate", semiring, dtype, "schedule", sch)
        R = ctx.contract(semiring, "ik", GA, "kj", GB, "ij", C=GC, accumulate=True, schedule=sch)
        check_csr(R, exp, semiring, dtype)


def test_mfma_fp32_signed_error_model(ctx):
    # fp32 dense x dense: partial sums of at most 128 k-terms in fp32 added to
    # an fp64 total, so |c - c_exact| <= 128 * 2^-24 * sum_k |a_ik b_kj|
    M, N, K = 257, 190, 1500
    a = (synth.uniform_f32(synth.stream_key(SEED, 30), M * K) * 2 - 1).reshape(M, K)
    b = (synth.uniform_f32(synth.stream_key(SEED, 31), K * N) * 2 - 1).reshape(K, N)
    C = torch.empty((M, N), dtype=torch.float32, device="cuda")
    ctx.contract("plus_times", "ik", torch.as_tensor(a, device="cuda"), "kj", torch.as_tensor(b, device="cuda"), "ij",
                 C=C)
    exact = oracle.dense_plus_times(a, b)
    mag = oracle.dense_plus_times(np.abs(a), np.abs(b))
    err = np.abs(C.cpu().numpy().astype(np.float64) - exact)
    bound = 128 * 2.0 ** -24 * mag + 2.0 ** -24 * np.abs(exact)
    assert np.all(err <= bound), f"worst ratio {np.max(err / bound):.3f}"


# ------------------------------------------------------------- failure paths --
class _Env:
    def __init__(self, **kv):
        self.kv = kv
        self.old = {}

    def __enter__(self):
        for k, v in self.kv.items():
            self.old[k] = os.environ.get(k)
            os.environ[k] = v

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_lds_budget_gives_identical_results(ctx):
    # a 48 KB budget rules out the 4096- and 8192-slot hash bins, the 16384-slot
    # symbolic table and the 8K/16K dense windows: their rows take the 4K
    # windows; results are unchanged
    n = 1 << 13
    src, dst = synth.rmat_edges(13, 16, 0.57, 0.19, 0.19, SEED, tag=40)
    with _Env(SRTC_LDS_BUDGET=str(48 * 1024)):
        small = srtc.Context(0)
    for semiring, dtype in (("plus_times", "f64"), ("min_plus", "i32"), ("or_and", "bool")):
        G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, SEED, 41)
        exp = oracle.spgemm(semiring, dtype, O, O)
        for sch in range(srtc.NUM_SCHEDULES):
            say("lds budget", semiring, dtype, "schedule", sch)
            check_csr(small.contract(semiring, "ik", G, "kj", G, "ij", schedule=sch), exp, semiring, dtype)
    with _Env(SRTC_LDS_BUDGET="20000"):
        tiny = srtc.Context(0)
    G, O = pair_inputs(ctx, "plus_times", "f64", src, dst, n, SEED, 41)
    with pytest.raises(srtc.SrtcError) as e:
        tiny.contract("plus_times", "ik", G, "kj", G, "ij")
    assert e.value.status == -9


def test_force_schedule_and_validate_switches(ctx):
    n = 2000
    src, dst = synth.er_edges(n, 40.0, SEED, tag=50)
    G, O = pair_inputs(ctx, "min_plus", "i32", src, dst, n, SEED, 51)
    exp = oracle.spgemm("min_plus", "i32", O, O)
    with _Env(SRTC_FORCE_SCHEDULE="4"):
        forced = srtc.Context(0)
    # schedule 4 sends every row to the dense windows: only that numeric
    # kernel runs
    srtc.lib().srtc_profile_enable(forced._h, 1)
    check_csr(forced.contract("min_plus", "ik", G, "kj", G, "ij"), exp, "min_plus", "i32")
    names = []
    i = 0
    buf = ctypes.create_string_buffer(96)
    while srtc.lib().srtc_profile_query(forced._h, i, buf, 96, None, None, None) == 0:
        names.append(buf.value.decode())
        i += 1
    numeric = [x for x in names if x.startswith("spgemm.numeric")]
    assert numeric == ["spgemm.numeric.dense.i32"], names
    for bad in ("9", "x", "-1"):
        with _Env(SRTC_FORCE_SCHEDULE=bad):
            with pytest.raises(srtc.SrtcError):
                srtc.Context(0)
    # SRTC_VALIDATE checks operands without opts.validate
    rp = torch.tensor([0, 2, 1, 3], dtype=torch.int64, device="cuda")
    bad = srtc.CSR(rp, torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda"),
                   torch.ones(3, dtype=torch.int32, device="cuda"), (3, 3))
    with _Env(SRTC_VALIDATE="1"):
        checking = srtc.Context(0)
    with pytest.raises(srtc.SrtcError) as e:
        checking.contract("min_plus", "ik", bad, "kj", bad, "ij")
    assert e.value.status == -5
    big = srtc.CSR(torch.tensor([0, 1], dtype=torch.int64, device="cuda"),
                   torch.tensor([0], dtype=torch.int32, device="cuda"),
                   torch.tensor([ID + 1], dtype=torch.int32, device="cuda"), (1, 1))
    with pytest.raises(srtc.SrtcError) as e:
        checking.contract("min_plus", "ik", big, "kj", big, "ij")
    assert e.value.status == -5


def test_allocator_failure_returns_oom_and_frees_everything():
    # a context whose allocator serves `budget` requests, then returns NULL:
    # every budget up to what the product needs ends in SRTC_ERR_OOM, and all
    # memory handed out is returned through the free callback
    n = 3000
    src, dst = synth.er_edges(n, 20.0, SEED, tag=60)
    w = synth.edge_values("i32", src.size, SEED, 61, lo=1, hi=100)
    base = srtc.Context(0)
    G = gpu_fold(base, "min_plus", "i32", dst, src, w, n, n)
    L = srtc.lib()
    state = {"left": 0, "live": {}, "calls": 0}

    def _a(user, nbytes):
        state["calls"] += 1
        if state["left"] <= 0:
            return None
        state["left"] -= 1
        t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")
        state["live"][t.data_ptr()] = t
        return t.data_ptr()

    def _f(user, ptr):
        state["live"].pop(ptr, None)

    cb = (srtc._ALLOC(_a), srtc._FREE(_f))
    h = ctypes.c_void_p()
    assert L.srtc_ctx_create(0, cb[0], cb[1], None, ctypes.byref(h)) == 0
    try:
        ad = srtc._desc(G)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        need = None
        for budget in range(0, 200):
            state["left"] = budget
            cd = srtc._Tensor()
            cd.order, cd.format, cd.dtype = 2, srtc.CSR_FMT, srtc.I32
            cd.dims[0], cd.dims[1] = n, n
            opts = srtc._Opts(0, 1, 0, 0)
            st = L.srtc_contract(h, srtc.MIN_PLUS, None, 0, b"ik", ctypes.byref(ad), b"kj", ctypes.byref(ad), b"ij",
                                 ctypes.byref(cd), ctypes.byref(opts), stream)
            if st == 0:
                need = budget
                for p in (cd.rowptr, cd.colidx, cd.vals):
                    state["live"].pop(p, None)
                break
            assert st == -7, (budget, st)
            torch.cuda.synchronize()
            assert not state["live"], f"budget {budget}: {len(state['live'])} buffers leaked"
        assert need is not None and need > 3
        say("allocations needed:", need)
    finally:
        L.srtc_ctx_destroy(h)


@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_column_blocked_products(ctx, semiring, dtype):
    """B cut into column blocks (forced with SRTC_COL_BLOCKS on inputs the
    library would multiply whole): heavy rows are multiplied block by block
    and written at per-block offsets, light rows against all of B; results
    equal the oracle's for every schedule, with accumulate, and with exact
    cancellations that drop identity results."""
    n = 1 << 14
    src, dst = synth.rmat_edges(14, 16, 0.57, 0.19, 0.19, SEED, tag=70)
    G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, SEED, 71)
    exp = oracle.spgemm(semiring, dtype, O, O)
    for blocks in ("3", "7", "0"):
        with _Env(SRTC_COL_BLOCKS=blocks):
            bctx = srtc.Context(0)
        for sch in range(srtc.NUM_SCHEDULES):
            say("column blocks", blocks, semiring, dtype, "schedule", sch)
            check_csr(bctx.contract(semiring, "ik", G, "kj", G, "ij", schedule=sch), exp, semiring, dtype)
    with _Env(SRTC_COL_BLOCKS="4"):
        bctx = srtc.Context(0)
    C0 = pair_inputs(ctx, semiring, dtype, dst, src, n, SEED, 72)
    exp2 = oracle.spgemm(semiring, dtype, O, O, C_old=C0[1])
    check_csr(bctx.contract(semiring, "ik", G, "kj", G, "ij", C=C0[0], accumulate=True, schedule=5), exp2, semiring,
              dtype)
    if semiring == "plus_times":
        # +-1 values: many sums cancel to exactly 0 and are dropped
        v = np.where(synth.edge_values("f64", src.size, SEED, 73) < 0.5, -1.0, 1.0).astype(oracle.NP_DTYPES[dtype])
        Gc = gpu_fold(ctx, semiring, dtype, dst, src, v, n, n)
        Oc = oracle.fold(semiring, dtype, dst, src, v, n, n)
        expc = oracle.spgemm(semiring, dtype, Oc, Oc)
        for sch in (0, 3, 5):
            check_csr(bctx.contract(semiring, "ik", Gc, "kj", Gc, "ij", schedule=sch), expc, semiring, dtype)
