"""Full-size parity of the benchmarked workload (GPU only).

R-MAT scale 18, edge factor 16, A.A over (+,x) in fp64 and fp32, in every
SpGEMM schedule, compared on sampled rows (the heaviest rows and a seeded
random sample) with the oracle computing just those rows; plus the order-3
tensor contraction of the same workload in full."""

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
    heavy = np.argsort(w)[-12:]
    rnd = synth.permutation(synth.stream_key(synth.SEED_CFG1, 99), n)[:300]
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
