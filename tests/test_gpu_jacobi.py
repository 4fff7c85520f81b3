"""Jacobi iteration and elementwise transforms against the oracle (GPU
only).  Iterates are compared at the stopping step: the same number of
updates, the solution within the value type's tolerance."""

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import say

pytestmark = pytest.mark.gpu
TORCH = {"f64": torch.float64, "f32": torch.float32}
RTOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    return srtc.Context(0)


def stencil_system(g, dtype, seed):
    src, dst = synth.stencil27_edges(g)
    n = g ** 3
    vals = np.where(src == dst, 27.0, -1.0).astype(oracle.NP_DTYPES[dtype])
    b = synth.uniform_f64(synth.stream_key(seed, 1), n).astype(oracle.NP_DTYPES[dtype])
    return src, dst, vals, b, n


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("g,tol", [(5, 1e-9), (23, 1e-8)])
def test_jacobi_stencil(ctx, dtype, g, tol):
    say("jacobi", dtype, g)
    if dtype == "f32":
        tol = 1e-4
    src, dst, vals, b, n = stencil_system(g, dtype, 7)
    keys = dst.astype(np.int64) * n + src
    A = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(vals, device="cuda"), (n, n))
    bd = torch.as_tensor(b, device="cuda")
    x0 = synth.uniform_f64(synth.stream_key(7, 2), n).astype(oracle.NP_DTYPES[dtype])
    x = torch.as_tensor(x0.copy(), device="cuda")
    it, r = ctx.jacobi(A, bd, x, tol=tol, steps_per_check=6)
    O = oracle.fold("plus_times", dtype, dst, src, vals, n, n)
    xo, lo, ro, ok = oracle.jacobi(O, b, x0, tol, dtype=dtype)
    assert ok and it == lo
    got = x.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - xo) <= RTOL[dtype] * np.abs(xo) + (1e-12 if dtype == "f64" else 1e-6))
    assert r <= tol and abs(r - ro) <= 1e-6 * max(ro, 1e-30) + (1e-13 if dtype == "f64" else 1e-7)


def test_jacobi_cap_errors_and_csr(ctx):
    say("jacobi cap and errors")
    src, dst, vals, b, n = stencil_system(7, "f64", 9)
    keys = dst.astype(np.int64) * n + src
    A = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(vals, device="cuda"), (n, n))
    bd = torch.as_tensor(b, device="cuda")
    O = oracle.fold("plus_times", "f64", dst, src, vals, n, n)
    # a cap below the needed updates: NOT_CONVERGED with x^cap (odd and even)
    for cap in (3, 4, 9):
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        with pytest.raises(srtc.NotConverged):
            ctx.jacobi(A, bd, x, tol=1e-14, max_iters=cap, steps_per_check=4)
        xo, lo, _, ok = oracle.jacobi(O, b, np.zeros(n), 1e-14, max_iters=cap)
        assert not ok and lo == cap
        assert np.allclose(x.cpu().numpy(), xo, rtol=1e-12, atol=1e-15)
    # the folded CSR gives the same iterates as the COO
    Acsr = ctx.fold("plus_times", A, "ij", "i", "j")
    x1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    x2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert ctx.jacobi(A, bd, x1, tol=1e-9) == ctx.jacobi(Acsr, bd, x2, tol=1e-9)
    assert torch.equal(x1, x2)
    # a zero diagonal entry is refused before any step
    Z = srtc.COO(torch.as_tensor(np.array([1], np.int64), device="cuda"),
                 torch.ones(1, dtype=torch.float64, device="cuda"), (2, 2))
    with pytest.raises(srtc.SrtcError) as e:
        ctx.jacobi(Z, torch.ones(2, dtype=torch.float64, device="cuda"), torch.zeros(2, dtype=torch.float64,
                                                                                    device="cuda"))
    assert e.value.status == -1


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_transforms(ctx, dtype):
    say("transforms", dtype)
    rng = np.random.default_rng(21)
    npt = oracle.NP_DTYPES[dtype]
    C0 = (rng.random((5, 7, 3, 4)) + 1).astype(npt)
    Ei = rng.random(3).astype(npt)
    Ea = rng.random(5).astype(npt)
    M = rng.random((7, 4)).astype(npt)
    cases = [
        ("recip", 1.0, "", None, "", None),
        ("scale", -0.5, "", None, "", None),
        ("add", 1.0, "i", Ei, "", None),          # D["abij"] += Ei["i"]
        ("add", -1.0, "a", Ea, "", None),         # D["abij"] -= Ea["a"]
        ("fma", 2.0, "jb", M.T.copy(), "ai", rng.random((5, 3)).astype(npt)),
        ("div_sum", 0.0, "i", Ei, "a", Ea),       # C = C / (A["i"] + B["a"])
    ]
    for op, alpha, ia, A, ib, B in cases:
        C = torch.as_tensor(C0.copy(), device="cuda")
        ctx.transform(op, C, torch.as_tensor(A, device="cuda") if A is not None else None, ia,
                      torch.as_tensor(B, device="cuda") if B is not None else None, ib, "abij", alpha)
        exp = oracle.transform(op, alpha, ia, A, ib, B, "abij", C0)
        got = C.cpu().numpy()
        # both sides evaluate in the value type with at most three roundings
        # (fused or not) on operands that do not cancel (C >= 1, the other
        # terms in [0, 2)), so each is within 3u of the exact value
        u = np.finfo(npt).eps / 2
        assert np.all(np.abs(got.astype(np.float64) - exp) <= 6 * u * np.abs(exp.astype(np.float64))), op
    # a sparse C: its stored values only
    keys = synth.bernoulli_keys((50, 60), 0.1, seed=3)
    v = (synth.uniform_f64(synth.stream_key(3, 9), keys.size) + 0.5).astype(npt)
    S = srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(v, device="cuda"), (50, 60))
    ctx.transform("recip", S, ic="ij", alpha=3.0)
    assert np.allclose(S.val.cpu().numpy(), (npt(3.0) / v), rtol=RTOL[dtype], atol=0)
    with pytest.raises(srtc.SrtcError):
        ctx.transform("add", S, torch.as_tensor(v[:50], device="cuda"), "i", ic="ij")
