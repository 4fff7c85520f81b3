"""Learned schedule selection on timings the method generates (GPU only).

The training set is the first 40 matrices of the selector recipe (ER,
R-MAT, 27-point stencil, power-law rows) as (+,x) fp32 and (min,+) int32
A.A, every schedule timed by the exhaustive tuner.  After training on the
GPU, the selector's picks must cost no more in total than the best single
fixed schedule on those timings (what the network gains over running
without it), and its choice must survive save/load.  Which schedule wins is
timing-dependent and not pinned."""

import numpy as np
import pytest
import torch

import paper_1512_00066_amd as srtc
from gen import synth
from gpu_common import say
from paper_1512_00066_amd import selector as S

pytestmark = pytest.mark.gpu


def test_selector_trained_on_generated_timings(tmp_path):
    ctx = srtc.Context(0)
    X, T = [], []
    for i in range(40):
        fam, n, src, dst, _ = synth.selector_matrix(i, synth.SEED_CFG4)
        say("selector matrix", i, fam, n)
        keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
        for sr, dt in (("plus_times", "f32"), ("min_plus", "i32")):
            v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=i, lo=1, hi=100)
            A = ctx.fold(sr, srtc.COO(keys, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
            f, t = S.collect(ctx, sr, A, A, reps=2)
            assert f.shape == (srtc.NUM_FEATURES,) and np.all(np.isfinite(f))
            assert t.shape == (srtc.NUM_SCHEDULES,) and np.all(t > 0)
            X.append(f)
            T.append(t)
    X, T = np.array(X, np.float32), np.array(T, np.float64)
    fixed = S.best_fixed(T)
    loss = S.train(ctx, X, T, epochs=600, batch=32, lr=2e-3, seed=3)
    ev = S.evaluate(ctx, X, T, fixed)
    say("selector loss", loss, "fixed", fixed, {k: ev[k] for k in ("mean_regret", "fixed_regret", "total_gain", "hits")})
    assert np.isfinite(loss)
    assert ev["total_gain"] >= 0.99
    path = str(tmp_path / "selector.bin")
    ctx.selector_save(path)
    c2 = srtc.Context(0)
    c2.selector_load(path)
    assert [c2.select(x) for x in X] == ev["picks"]
