"""Helpers shared by the GPU parity tests: synthetic inputs from the seeded
generators, folded independently by the HIP library and by the oracle, and
comparison of CSR results to the stated tolerances."""

import sys

import numpy as np
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth

PAIRS = [("plus_times", "f64"), ("plus_times", "f32"), ("min_plus", "i32"),
         ("min_plus", "f32"), ("or_and", "bool"), ("max_times", "f32"),
         ("max_times", "f64")]
EXACT = {("min_plus", "i32"), ("min_plus", "f32"), ("or_and", "bool"), ("max_times", "f32"),
         ("max_times", "f64")}
# (+,x) tolerances: fp64 results within 1e-12 relative of the Dot2 oracle;
# fp32 results (exact products, fp64 accumulation, one final rounding)
# within 1e-5 relative of the fp64 oracle on the same fp32 inputs.
RTOL = {("plus_times", "f64"): 1e-12, ("plus_times", "f32"): 1e-5}

TORCH = {"f64": torch.float64, "f32": torch.float32, "i32": torch.int32, "bool": torch.uint8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def values(semiring, dtype, m, seed, tag=0):
    if dtype == "bool":
        return np.ones(m, dtype=np.uint8)
    if dtype == "i32":
        return synth.edge_values("i32", m, seed, tag, lo=1, hi=100)
    v = synth.edge_values(dtype, m, seed, tag)
    if semiring == "max_times":
        # keep (max,x) products away from the identity 0
        v = v + np.asarray(0.125, dtype=v.dtype)
    return v


def gpu_fold(ctx, semiring, dtype, rows, cols, vals, m, n):
    keys = np.asarray(rows, dtype=np.int64) * n + np.asarray(cols, dtype=np.int64)
    coo = srtc.COO(torch.as_tensor(keys, device="cuda"),
                   torch.as_tensor(np.ascontiguousarray(vals, dtype=oracle.NP_DTYPES[dtype]), device="cuda"), (m, n))
    return ctx.fold(semiring, coo, "ij", "i", "j")


def pair_inputs(ctx, semiring, dtype, src, dst, n, seed, tag=0):
    """(GPU CSR, oracle CSR) of the same edge list (A[dst][src] = w)."""
    v = values(semiring, dtype, src.size, seed, tag)
    G = gpu_fold(ctx, semiring, dtype, dst, src, v, n, n)
    O = oracle.fold(semiring, dtype, dst, src, v, n, n)
    return G, O


def check_csr(got, exp, semiring, dtype, rows=None):
    """Compare a GPU CSR (all rows, or the listed rows) with an oracle CSR
    over the same rows: identical structure; values bit-exact for exact
    semirings, within RTOL for (+,x)."""
    rp, col, val = got.to_host()
    if rows is not None:
        rows = np.asarray(rows, dtype=np.int64)
        cnt = rp[rows + 1] - rp[rows]
        idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows]) if rows.size else np.zeros(0, np.int64)
        rp = np.concatenate([[0], np.cumsum(cnt)])
        col, val = col[idx], val[idx]
    assert np.array_equal(rp, exp.rowptr), "row pointers differ"
    assert np.array_equal(col, exp.col), "column indices differ"
    if (semiring, dtype) in RTOL:
        ref = exp.val.astype(np.float64)
        err = np.abs(val.astype(np.float64) - ref)
        bound = RTOL[(semiring, dtype)] * np.abs(ref)
        bad = err > bound
        assert not bad.any(), f"{bad.sum()} values outside rtol {RTOL[(semiring, dtype)]}; worst rel " \
                              f"{(err / np.maximum(np.abs(ref), 1e-300)).max():.3e}"
    else:
        assert np.array_equal(val, exp.val.astype(val.dtype)), "values differ"
