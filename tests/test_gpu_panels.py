"""Row-panel streaming of a sparse product (GPU only).

C = A (x) B is formed panel by panel (runs of rows within a product budget)
and handed to a consumer; the panels laid end to end must equal the oracle's
product for every semiring, a budget smaller than one row's products makes
that row a panel alone, and a consumer may stop the product."""

import numpy as np
import pytest
import torch

import oracle
import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import PAIRS, check_csr, pair_inputs, say

pytestmark = pytest.mark.gpu

SEED = 0x5EED2100


@pytest.fixture(scope="module")
def ctx():
    return srtc.Context(0)


def stitch(panels, ncols):
    """One CSR from consecutive panels (row0, CSR)."""
    rps, cols, vals, m = [np.zeros(1, np.int64)], [], [], 0
    base = 0
    for row0, P in panels:
        assert row0 == m
        rp, c, v = P.to_host()
        rps.append(rp[1:] + base)
        cols.append(c)
        vals.append(v)
        base += rp[-1]
        m += P.shape[0]
    return srtc.CSR(torch.as_tensor(np.concatenate(rps)), torch.as_tensor(np.concatenate(cols)),
                    torch.as_tensor(np.concatenate(vals)), (m, ncols))


@pytest.mark.parametrize("semiring,dtype", PAIRS)
def test_panels_equal_the_product(ctx, semiring, dtype):
    scale = 12
    n = 1 << scale
    src, dst = synth.rmat_edges(scale, 8, 0.57, 0.19, 0.19, SEED, tag=1)
    G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, SEED, 2)
    exp = oracle.spgemm(semiring, dtype, O, O)
    nb = np.diff(O.rowptr)
    w = np.zeros(n, np.int64)
    np.add.at(w, np.repeat(np.arange(n), nb), nb[O.col])
    budget = int(w.sum() // 9)
    for sch in (-1, 0, 5):
        panels = []
        count = ctx.contract_panels(semiring, "ik", G, "kj", G, "ij", lambda r0, P: panels.append((r0, P)),
                                    panel_products=budget, schedule=sch)
        say("panels", semiring, dtype, "schedule", sch, "count", count)
        assert count == len(panels) >= 9
        for r0, P in panels:
            r1 = r0 + P.shape[0]
            assert P.shape[0] == 1 or w[r0:r1].sum() <= budget
            # the next row would have exceeded the budget
            assert r1 == n or w[r0:r1 + 1].sum() > budget
        check_csr(stitch(panels, n), exp, semiring, dtype)


@pytest.mark.parametrize("semiring,dtype", [("plus_times", "f64"), ("plus_times", "f32"), ("min_plus", "i32")])
def test_panels_reuse_b_tables(ctx, semiring, dtype):
    """R-MAT 15 (32,768 columns: two to eight dense windows per row, so the
    window tables exist) in about a dozen panels: B's window tables and value
    records are built for the first panel and reused by the others; every
    panel's rows equal the oracle's."""
    scale = 15
    n = 1 << scale
    src, dst = synth.rmat_edges(scale, 8, 0.57, 0.19, 0.19, SEED, tag=3)
    G, O = pair_inputs(ctx, semiring, dtype, src, dst, n, SEED, 4)
    exp = oracle.spgemm(semiring, dtype, O, O)
    nb = np.diff(O.rowptr)
    budget = int(nb[O.col].sum() // 12)
    for sch in (3, 0, 6):
        panels = []
        count = ctx.contract_panels(semiring, "ik", G, "kj", G, "ij", lambda r0, P: panels.append((r0, P)),
                                    panel_products=budget, schedule=sch)
        say("panels reusing B's tables", semiring, dtype, "schedule", sch, "count", count)
        assert count == len(panels) >= 12
        check_csr(stitch(panels, n), exp, semiring, dtype)


def test_panels_single_rows_and_stop(ctx):
    n = 2000
    src, dst = synth.er_edges(n, 8.0, SEED, tag=3)
    G, O = pair_inputs(ctx, "min_plus", "i32", src, dst, n, SEED, 4)
    exp = oracle.spgemm("min_plus", "i32", O, O)
    panels = []
    ctx.contract_panels("min_plus", "ik", G, "kj", G, "ij", lambda r0, P: panels.append((r0, P)), panel_products=1)
    assert len(panels) == n and all(P.shape[0] == 1 for _, P in panels)
    check_csr(stitch(panels, n), exp, "min_plus", "i32")
    seen = []
    with pytest.raises(srtc.SrtcError) as e:
        ctx.contract_panels("min_plus", "ik", G, "kj", G, "ij",
                            lambda r0, P: seen.append(r0) or (False if len(seen) == 3 else None), panel_products=5000)
    assert e.value.status == -1 and len(seen) == 3
    # COO operands and a transposed B fold first
    keys = torch.as_tensor(src.astype(np.int64) * n + dst, device="cuda")  # B stored as (j, k)
    w = synth.edge_values("i32", src.size, SEED, 4, lo=1, hi=100)
    Bt = srtc.COO(keys, torch.as_tensor(w, device="cuda"), (n, n))
    panels = []
    ctx.contract_panels("min_plus", "ik", G, "jk", Bt, "ij", lambda r0, P: panels.append((r0, P)),
                        panel_products=40000)
    check_csr(stitch(panels, n), exp, "min_plus", "i32")
