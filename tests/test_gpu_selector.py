"""Learned schedule selection on timings the method generates (GPU only).

Training sets are matrices of the selector recipe (ER, R-MAT, 27-point
stencil, power-law rows) as (+,x) fp32 and (min,+) int32 A.A, plus row
panels of R-MAT graphs, every schedule timed by the exhaustive tuner.  On
matrices it never saw, the trained network must stay within 10% of the
exhaustive tuner's time on average and cost no more in total than the best
single fixed schedule (what the network gains over running without it);
its choices survive save/load; its optimizer step and its features match
the oracle.  Which schedule wins is timing-dependent and not pinned."""

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
    path = str(tmp_path / "selector.bin")
    ctx.selector_save(path)
    c2 = srtc.Context(0)
    c2.selector_load(path)
    assert [c2.select(x) for x in X] == ev["picks"]


def _mats(ctx, idx, pairs=(("plus_times", "f32"), ("min_plus", "i32"))):
    for i in idx:
        fam, n, src, dst, _ = synth.selector_matrix(i, synth.SEED_CFG4)
        keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
        for sr, dt in pairs:
            v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=i, lo=1, hi=100)
            A = ctx.fold(sr, srtc.COO(keys, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
            host = ((dst, src, v, n, n), (dst, src, v, n, n))
            yield f"{fam}{i}/{sr}", sr, dt, A, A, host


def _panels(ctx, scale, js, pairs=(("plus_times", "f32"), ("min_plus", "i32"))):
    n = 1 << scale
    src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, synth.SEED_CFG4, tag=300 + scale)
    keys_b = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
    for sr, dt in pairs:
        v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=300 + scale, lo=1, hi=100)
        B = ctx.fold(sr, srtc.COO(keys_b, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
        for j in js:
            rows = synth.selector_panel_rows(n, 1000 * scale + j, synth.SEED_CFG4)
            pos = np.full(n, -1, dtype=np.int64)
            pos[rows] = np.arange(rows.size)
            sel = pos[dst] >= 0
            Ap = ctx.fold(sr, srtc.COO(torch.as_tensor(pos[dst[sel]] * n + src[sel], device="cuda"),
                                       torch.as_tensor(v[sel], device="cuda"), (rows.size, n)), "ij", "i", "j")
            host = ((pos[dst[sel]], src[sel], v[sel], rows.size, n), (dst, src, v, n, n))
            yield f"panel{scale}.{j}/{sr}", sr, dt, Ap, B, host


def test_selector_held_out_regret_and_gain():
    """Trained on generated matrices and R-MAT 17/18 row panels, evaluated on
    matrices of the same recipe it never saw and on row panels of a larger
    R-MAT graph (scale 19): mean regret against the exhaustive tuner at most
    0.10 and total time no worse than the best fixed schedule's."""
    ctx = srtc.Context(0)
    X, T = [], []
    train = list(_mats(ctx, range(0, 96))) + list(_panels(ctx, 17, range(8))) + list(_panels(ctx, 18, range(8)))
    for name, sr, dt, A, B, _ in train:
        f, t = S.collect(ctx, sr, A, B, reps=3)
        X.append(f)
        T.append(t)
    say("training samples", len(X))
    X, T = np.array(X, np.float32), np.array(T, np.float64)
    fixed = S.best_fixed(T)
    loss = S.train(ctx, X, T, epochs=500, batch=32, lr=2e-3, seed=11)
    Xh, Th, names = [], [], []
    held = list(_mats(ctx, range(4000, 4032))) + list(_panels(ctx, 19, range(100, 103)))
    for name, sr, dt, A, B, _ in held:
        # ground truth for the regret: median of 10 timings after a warm-up
        f, t = S.collect(ctx, sr, A, B, reps=10)
        Xh.append(f)
        Th.append(t)
        names.append(name)
    ev = S.evaluate(ctx, np.array(Xh, np.float32), np.array(Th, np.float64), fixed)
    worst = int(np.argmax(ev["regret"]))
    say("held-out: loss", loss, "fixed", fixed, "mean regret", ev["mean_regret"], "total gain", ev["total_gain"],
        "fixed regret", ev["fixed_regret"], "worst", names[worst], ev["regret"][worst])
    assert ev["mean_regret"] <= 0.10
    assert ev["total_gain"] >= 1.0


def test_adam_step_matches_oracle():
    """Five Adam updates by the library's kernel against the fp64 formulas."""
    from oracle import mlp as omlp
    ctx = srtc.Context(0)
    npar = srtc.mlp_num_params()
    rng = np.random.default_rng(17)
    p = rng.normal(scale=0.3, size=npar).astype(np.float32)
    m1 = np.zeros(npar, np.float32)
    m2 = np.zeros(npar, np.float32)
    P, M1, M2 = (torch.as_tensor(x.copy(), device="cuda") for x in (p, m1, m2))
    rp, rm, rv = p.astype(np.float64), m1.astype(np.float64), m2.astype(np.float64)
    # the kernel's hyperparameters are fp32 values: the oracle takes the same
    # numbers (0.999 itself is not representable in fp32)
    lr, b1, b2, eps = (float(np.float32(x)) for x in (3e-3, 0.9, 0.999, 1e-8))
    u = 2.0 ** -24
    mag = np.zeros(npar)  # the first-moment recurrence on magnitudes
    for t in range(1, 6):
        g = rng.normal(scale=10.0 ** rng.uniform(-3, 1), size=npar).astype(np.float32)
        g[::7] = 0.0
        ctx.mlp_adam_step(P, torch.as_tensor(g, device="cuda"), M1, M2, t, lr, b1, b2, eps)
        rp, rm, rv = omlp.adam_step(rp, g.astype(np.float64), rm, rv, t, lr, b1, b2, eps)
        mag = b1 * mag + (1 - b1) * np.abs(g.astype(np.float64))
        gp, gm, gv = (x.cpu().numpy().astype(np.float64) for x in (P, M1, M2))
        # fp32 arithmetic, a few roundings per step: the first moment can
        # cancel, so its error is bounded by the recurrence on magnitudes;
        # the second moment has no cancellation; a parameter moves by at most
        # about lr per step
        assert np.all(np.abs(gm - rm) <= 3 * u * t * mag), t
        assert np.all(np.abs(gv - rv) <= 3 * u * t * np.abs(rv)), t
        assert np.all(np.abs(gp - rp) <= 4 * u * np.abs(rp) + 1e-5 * lr * t), t


def test_features_match_oracle():
    """The 32 features of the library against the oracle's definitions:
    histogram fractions and one-hots exactly, logarithms and the CV within
    fp32 rounding."""
    import oracle
    ctx = srtc.Context(0)
    cases = [c for c in _mats(ctx, [0, 1, 2, 3, 9, 14], pairs=(("plus_times", "f32"), ("min_plus", "i32")))]
    cases += list(_panels(ctx, 17, [3], pairs=(("plus_times", "f32"),)))
    for name, sr, dt, A, B, host in cases:
        got = ctx.features(sr, A, B)
        # the oracle folds the same generated edge lists itself
        (ar, ac, av, am, an), (br, bc, bv, bm, bn) = host
        OA = oracle.fold(sr, dt, ar, ac, av, am, an)
        OB = oracle.fold(sr, dt, br, bc, bv, bm, bn)
        exp = oracle.features(sr, OA, OB)
        say("features", name)
        exact = list(range(0, 20)) + [28, 29, 30, 31]
        assert np.array_equal(got[exact], exp[exact]), (name, got[exact], exp[exact])
        rest = [q for q in range(32) if q not in exact]
        np.testing.assert_allclose(got[rest], exp[rest], rtol=1e-6, atol=1e-6, err_msg=name)
