"""Hub tiles: (+,x) sparse products with the block of the densest rows,
inner indices and columns formed on the matrix cores (GPU only).

The result must be the oracle's product: the same pattern, values within the
(+,x) bounds (1e-12 fp64; fp32 within 1e-5 of the fp64 oracle, which also
covers the tile's fp32 partial sums of at most 128 non-negative terms)."""

import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import check_csr, gpu_fold, pair_inputs, say, values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return srtc.Context(0)


def _profile(ctx):
    rows, i = {}, 0
    name = ctypes.create_string_buffer(96)
    while True:
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        if srtc.lib().srtc_profile_query(ctx._h, i, name, 96, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)):
            return rows
        rows[name.value.decode()] = n.value
        i += 1


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hub_tiles_square_every_size_and_schedule(ctx, dtype):
    # R-MAT 12, edge factor 16: hubs of a few hundred entries; tile sizes from
    # one index to past the matrix (everything dense)
    src, dst = synth.rmat_edges(12, 16, 0.57, 0.19, 0.19, seed=41)
    n = 1 << 12
    G, O = pair_inputs(ctx, "plus_times", dtype, src, dst, n, 41)
    exp = oracle.spgemm("plus_times", dtype, O, O)
    for hub in (1, 64, 700, 16384):
        for sch in range(srtc.NUM_SCHEDULES):
            say("hub tile", dtype, hub, "schedule", sch)
            C = ctx.contract("plus_times", "ik", G, "kj", G, "ij", schedule=sch, hub_tile=hub)
            check_csr(C, exp, "plus_times", dtype)


def test_hub_tiles_rectangular_and_profiled(ctx):
    # A: 3000 x 4096 (rows of one R-MAT graph), B: 4096 x 6000 (another graph
    # with its columns spread), so the three hub sets differ in size and place
    n = 1 << 12
    sa, da = synth.rmat_edges(12, 16, 0.57, 0.19, 0.19, seed=42)
    keep = da < 3000
    va = values("plus_times", "f64", int(keep.sum()), 42)
    sb, db = synth.rmat_edges(12, 12, 0.57, 0.19, 0.19, seed=43)
    cb = (sb.astype(np.int64) * 6000) // n + (sb % 2)   # columns in [0, 6000)
    pairs = np.unique(db.astype(np.int64) * 6000 + cb)
    rb, cb = pairs // 6000, pairs % 6000
    vb = values("plus_times", "f64", rb.size, 43)
    A = gpu_fold(ctx, "plus_times", "f64", da[keep], sa[keep], va, 3000, n)
    B = gpu_fold(ctx, "plus_times", "f64", rb, cb, vb, n, 6000)
    OA = oracle.fold("plus_times", "f64", da[keep], sa[keep], va, 3000, n)
    OB = oracle.fold("plus_times", "f64", rb, cb, vb, n, 6000)
    exp = oracle.spgemm("plus_times", "f64", OA, OB)
    srtc.lib().srtc_profile_enable(ctx._h, 1)
    try:
        for hub in (256, 5000):
            say("rectangular hub tile", hub)
            C = ctx.contract("plus_times", "ik", A, "kj", B, "ij", hub_tile=hub)
            check_csr(C, exp, "plus_times", "f64")
        prof = _profile(ctx)
    finally:
        srtc.lib().srtc_profile_enable(ctx._h, 0)
    assert prof.get("spgemm.hub_gemm_mfma.f64", 0) == 2, prof


def test_hub_tiles_only_where_they_apply(ctx):
    src, dst = synth.rmat_edges(11, 16, 0.57, 0.19, 0.19, seed=44)
    n = 1 << 11
    # (min,+): the tile does not apply; the product is the sparse one
    G, O = pair_inputs(ctx, "min_plus", "i32", src, dst, n, 44)
    check_csr(ctx.contract("min_plus", "ik", G, "kj", G, "ij", hub_tile=128),
              oracle.spgemm("min_plus", "i32", O, O), "min_plus", "i32")
    # (+,x) with an old C to merge: the sparse path merges it; with an empty
    # old C the tile applies
    G, O = pair_inputs(ctx, "plus_times", "f64", src, dst, n, 45)
    P = ctx.contract("plus_times", "ik", G, "kj", G, "ij")
    C = ctx.contract("plus_times", "ik", G, "kj", G, "ij", C=P, accumulate=True, hub_tile=128)
    exp = oracle.spgemm("plus_times", "f64", O, O)
    two = oracle.CSR(exp.rowptr, exp.col, 2.0 * exp.val, exp.nrows, exp.ncols)
    check_csr(C, two, "plus_times", "f64")
    E = srtc.csr_from_host(np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float64), (n, n))
    C = ctx.contract("plus_times", "ik", G, "kj", G, "ij", C=E, accumulate=True, hub_tile=128)
    check_csr(C, exp, "plus_times", "f64")
    # out-of-range sizes and environment values are rejected
    for bad in (-1, 16385):
        with pytest.raises(srtc.SrtcError) as e:
            ctx.contract("plus_times", "ik", G, "kj", G, "ij", hub_tile=bad)
        assert e.value.status == -1
    old = os.environ.get("SRTC_HUB_TILE")
    try:
        os.environ["SRTC_HUB_TILE"] = "many"
        with pytest.raises(srtc.SrtcError):
            srtc.Context(0)
        os.environ["SRTC_HUB_TILE"] = "96"
        c2 = srtc.Context(0)
        check_csr(c2.contract("plus_times", "ik", G, "kj", G, "ij"), exp, "plus_times", "f64")
    finally:
        if old is None:
            os.environ.pop("SRTC_HUB_TILE", None)
        else:
            os.environ["SRTC_HUB_TILE"] = old
