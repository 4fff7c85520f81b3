"""General-order contractions with the shapes of the paper's MP3 equations
(Section 4.3): sparse order-4 integral tensors V times dense amplitudes T,
letters in any order, outputs folded back into an interleaved index order,
a letter in all three tensors (batch / Hadamard), full contraction to a
scalar, and dense x dense (+,x) on the matrix cores.  Compared with the
oracle's dense contraction (GPU only)."""

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import say

pytestmark = pytest.mark.gpu
TORCH = {"f64": torch.float64, "f32": torch.float32, "i32": torch.int32}
RTOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    return srtc.Context(0)


def sparse_tensor(semiring, dtype, dims, dens, seed, tag=0):
    """(GPU COO, dense copy with the identity where absent)."""
    keys = synth.bernoulli_keys(tuple(dims), dens, seed=seed, tag=tag)
    if dtype == "i32":
        vals = synth.edge_values("i32", keys.size, seed, tag, lo=0, hi=50)
    else:
        vals = synth.edge_values(dtype, keys.size, seed, tag)
    fill = oracle.default_add_id(semiring, dtype)
    D = np.full(int(np.prod(dims)), fill, dtype=oracle.NP_DTYPES[dtype])
    D[keys] = vals
    coo = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(vals, device="cuda"), tuple(dims))
    return coo, D.reshape(dims)


def dense_tensor(semiring, dtype, dims, seed, tag=0, absent=0.0):
    n = int(np.prod(dims))
    if dtype == "i32":
        v = synth.edge_values("i32", n, seed, 50 + tag, lo=0, hi=50)
    else:
        v = synth.edge_values(dtype, n, seed, 50 + tag)
    if absent:
        gone = synth.uniform_f64(synth.stream_key(seed, 70 + tag), n) < absent
        v = np.where(gone, np.asarray(oracle.default_add_id(semiring, dtype), dtype=v.dtype), v)
    v = v.reshape(dims)
    return torch.as_tensor(np.ascontiguousarray(v), device="cuda"), v


def check(got, exp, dtype):
    got = got.cpu().numpy() if isinstance(got, torch.Tensor) else got
    assert got.shape == exp.shape
    if dtype in RTOL:
        err = np.abs(got.astype(np.float64) - exp)
        assert np.all(err <= RTOL[dtype] * np.abs(exp)), float((err / np.maximum(np.abs(exp), 1e-300)).max())
    else:
        assert np.array_equal(got, exp)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m,n", [(6, 10), (8, 24)])
def test_mp3_sixth_order_contractions(ctx, dtype, m, n):
    """Z["abij"] (+)= Vabcd["abef"] T["efij"], Vijkl["mnij"] T["abmn"] and
    Vaibj["amei"] T["ebmj"]: the second and third need their output folded
    back (rows ij or ai, columns ab or bj) and the third a permuted T."""
    say("mp3", dtype, m, n)
    sr = "plus_times"
    dens = 0.05 if n > 10 else 0.2
    Vabcd, Vabcd_d = sparse_tensor(sr, dtype, (n, n, n, n), dens, 31, 1)
    Vijkl, Vijkl_d = sparse_tensor(sr, dtype, (m, m, m, m), 0.3, 31, 2)
    Vaibj, Vaibj_d = sparse_tensor(sr, dtype, (n, m, n, m), dens, 31, 3)   # letters a m e i
    T, T_d = dense_tensor(sr, dtype, (n, n, m, m), 31, 4)                  # letters a b i j
    Z0, Z0_d = dense_tensor(sr, dtype, (n, n, m, m), 31, 5)
    # 1. no fold-back
    Z = torch.empty_like(T)
    ctx.contract(sr, "abef", Vabcd, "efij", T, "abij", C=Z)
    check(Z, oracle.contract(sr, dtype, "abef", Vabcd_d, "efij", T_d, "abij"), dtype)
    # 2. rows i j (from V), columns a b: folded back, accumulating into Z0
    Z = Z0.clone()
    ctx.contract(sr, "mnij", Vijkl, "abmn", T, "abij", C=Z, accumulate=True)
    check(Z, Z0_d + oracle.contract(sr, dtype, "mnij", Vijkl_d, "abmn", T_d, "abij"), dtype)
    # 3. interleaved rows a i / columns b j, inner letters m e (T permuted)
    Z = torch.empty_like(T)
    ctx.contract(sr, "amei", Vaibj, "ebmj", T, "abij", C=Z)
    check(Z, oracle.contract(sr, dtype, "amei", Vaibj_d, "ebmj", T_d, "abij"), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mp3_lower_order_terms(ctx, dtype):
    """Fab["af"] T["fbij"] and Fij["ni"] T["abnj"] (dense x dense on MFMA, the
    second folded back), the Hadamard form T = V (.) D (a letter in all three
    tensors) and the energy T["abij"] V["abij"] (no letter in C)."""
    m, n = 7, 20
    say("mp3 lower order", dtype)
    sr = "plus_times"
    Fab, Fab_d = dense_tensor(sr, dtype, (n, n), 41, 1)
    Fij, Fij_d = dense_tensor(sr, dtype, (m, m), 41, 2)
    T, T_d = dense_tensor(sr, dtype, (n, n, m, m), 41, 3)
    D, D_d = dense_tensor(sr, dtype, (n, n, m, m), 41, 4)
    V, V_d = sparse_tensor(sr, dtype, (n, n, m, m), 0.1, 41, 5)
    Z = torch.empty_like(T)
    ctx.contract(sr, "af", Fab, "fbij", T, "abij", C=Z)
    check(Z, oracle.contract(sr, dtype, "af", Fab_d, "fbij", T_d, "abij"), dtype)
    Z0 = Z.clone()
    ctx.contract(sr, "ni", Fij, "abnj", T, "abij", C=Z, accumulate=True)
    check(Z, Z0.cpu().numpy().astype(np.float64) + oracle.contract(sr, dtype, "ni", Fij_d, "abnj", T_d, "abij"),
          dtype)
    H = torch.empty_like(T)
    ctx.contract(sr, "abij", V, "abij", D, "abij", C=H)
    check(H, oracle.contract(sr, dtype, "abij", V_d, "abij", D_d, "abij"), dtype)
    E = torch.zeros((), dtype=TORCH[dtype], device="cuda")
    ctx.contract(sr, "abij", V, "abij", T, "", C=E)
    check(E, oracle.contract(sr, dtype, "abij", V_d, "abij", T_d, ""), dtype)


def test_dense_batched_and_folded_back(ctx):
    """A letter in all three dense tensors is a strided batch of MFMA GEMMs;
    any letter order of the operands and the output."""
    say("dense batched")
    for dtype in ("f64", "f32"):
        A, A_d = dense_tensor("plus_times", dtype, (37, 70, 19), 51, 1)   # letters k z i
        B, B_d = dense_tensor("plus_times", dtype, (70, 37, 45), 51, 2)   # letters z k j
        C = torch.empty((45, 70, 19), dtype=TORCH[dtype], device="cuda")  # letters j z i
        ctx.contract("plus_times", "kzi", A, "zkj", B, "jzi", C=C)
        check(C, oracle.contract("plus_times", dtype, "kzi", A_d, "zkj", B_d, "jzi"), dtype)


@pytest.mark.parametrize("semiring,dtype", [("min_plus", "i32"), ("max_times", "f64")])
def test_fold_back_other_semirings(ctx, semiring, dtype):
    """The folded-back accumulation combines by the semiring's (+)."""
    say("fold-back", semiring, dtype)
    m, n = 5, 13
    V, V_d = sparse_tensor(semiring, dtype, (n, m, n, m), 0.2, 61, 1)    # letters a m e i
    T, T_d = dense_tensor(semiring, dtype, (n, n, m, m), 61, 2, absent=0.3)   # letters e b m j
    Z0, Z0_d = dense_tensor(semiring, dtype, (n, n, m, m), 61, 3, absent=0.5)  # letters a b i j
    Z = Z0.clone()
    ctx.contract(semiring, "amei", V, "ebmj", T, "abij", C=Z, accumulate=True)
    P = oracle.contract(semiring, dtype, "amei", V_d, "ebmj", T_d, "abij")
    exp = np.minimum(Z0_d, P) if semiring == "min_plus" else np.maximum(Z0_d, P)
    check(Z, exp, dtype)


@pytest.mark.parametrize("semiring,dtype", [("plus_times", "f64"), ("min_plus", "i32")])
def test_sparse_output_folded_back(ctx, semiring, dtype):
    """Sparse x sparse with C's letters interleaved (rows a i, columns b j):
    the CSR comes back in C's order with C's first two letters as rows."""
    say("sparse fold-back", semiring, dtype)
    a, k, i, b, j = 9, 14, 6, 11, 5
    A, A_d = sparse_tensor(semiring, dtype, (a, k, i), 0.15, 71, 1)   # letters a k i
    B, B_d = sparse_tensor(semiring, dtype, (k, b, j), 0.15, 71, 2)   # letters k b j
    C = ctx.contract(semiring, "aki", A, "kbj", B, "abij")
    assert tuple(C.dims) == (a, b, i, j) and C.split == 2
    rp, col, val = C.to_host()
    fill = oracle.default_add_id(semiring, dtype)
    got = np.full((a * b, i * j), fill, dtype=oracle.NP_DTYPES[dtype])
    rows = np.repeat(np.arange(a * b), np.diff(rp))
    got[rows, col] = val
    assert all(np.all(np.diff(col[rp[r]:rp[r + 1]]) > 0) for r in range(a * b))
    exp = oracle.contract(semiring, dtype, "aki", A_d, "kbj", B_d, "abij").reshape(a * b, i * j)
    if semiring == "plus_times":
        # absent positions: no product reached them
        assert np.array_equal(got != 0, exp != 0)
        check(got, exp, dtype)
    else:
        assert np.array_equal(got, exp)
    # accumulate: the previous C (same layout) joins by (+)
    C2 = ctx.contract(semiring, "aki", A, "kbj", B, "abij", C=C, accumulate=True)
    rp2, col2, val2 = C2.to_host()
    got2 = np.full((a * b, i * j), fill, dtype=oracle.NP_DTYPES[dtype])
    got2[np.repeat(np.arange(a * b), np.diff(rp2)), col2] = val2
    if semiring == "plus_times":
        check(got2, 2 * exp, dtype)
    else:
        assert np.array_equal(got2, exp)


@pytest.mark.parametrize("semiring,dtype", [("plus_times", "f64"), ("plus_times", "f32"), ("min_plus", "i32")])
def test_dense_elementwise_product(ctx, semiring, dtype):
    """Every letter in all three dense tensors: the elementwise product
    (the MP3 update T += Z (.) D), operands in other letter orders."""
    say("dense hadamard", semiring, dtype)
    Zt, Z_d = dense_tensor(semiring, dtype, (9, 11, 3, 5), 81, 1, absent=0.2 if semiring == "min_plus" else 0.0)
    Dt, D_d = dense_tensor(semiring, dtype, (5, 3, 9, 11), 81, 2, absent=0.2 if semiring == "min_plus" else 0.0)
    C0, C0_d = dense_tensor(semiring, dtype, (9, 11, 3, 5), 81, 3, absent=0.3 if semiring == "min_plus" else 0.0)
    C = C0.clone()
    ctx.contract(semiring, "abij", Zt, "jiab", Dt, "abij", C=C, accumulate=True)
    P = oracle.contract(semiring, dtype, "abij", Z_d, "jiab", D_d, "abij")
    exp = np.minimum(C0_d, P) if semiring == "min_plus" else C0_d.astype(np.float64) + P
    check(C, exp, dtype)
