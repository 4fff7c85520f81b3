#!/usr/bin/env python3
"""Benchmark of the semiring contraction hot path on one MI355X.

Default workload (--workload rmat21; one "step" = every hot-path stage over
one batch of synthetic input already resident in HBM):
  * R-MAT scale 21 (2,097,152 vertices), edge factor 16,
    (a,b,c,d) = (0.57,0.19,0.19,0.05), relabelled
  * C = A.A in full, in (+,x) fp64 and fp32 (values U[0,1)) and (min,+)
    int32 (weights U[1,100]): per product the fold of the COO edge list to
    CSR, the features and the learned selector's schedule choice, then the
    symbolic, numeric and compaction passes of every row panel (C has
    2.65e10 entries, more than one GPU holds in fp64, so it is streamed in
    panels of at most --panel-products products and each panel is
    released once handed over)
  * the selector is trained in the same run, before the timed steps, on
    timings of generated matrices and R-MAT 17-19 row panels; after the
    timed steps every schedule is timed on the full fp32 and int32 products
    (a matrix the selector never saw), giving its regret against the
    exhaustive tuner and its gain over the best fixed schedule
    (config.selector.held_out_rmat21; --no-regret skips it)
  * beside it, the batched form of 512 uneven ER instances against the same
    work as per-instance calls (config.batched_vs_plain, its own timing;
    --no-batch-comparison skips it)
Metric: semiring ops per second (one op = one (x) and one (+); SpGEMM ops =
products A_ik*B_kj), aggregated over the step.  Other workloads:
--workload rmat18 | rmat20_sssp | batch512 | selector | masked18 | apsp2048 |
mp3 | jacobi | gemm.

Prints one JSON line (see the module help for the fields).
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "semiring SpGEMM/SpMM ops/s + HBM GB/s fraction; batched/learned vs plain"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources the SpGEMM kernels are compiled from (the
    dominant kernel of the default workload); traffic measured with HBM
    counters is reported only while it matches."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1512_00066_amd", "csrc")
    for f in ("common.hpp", "internal.hpp", "spgemm.hip"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_table(ctx):
    import ctypes
    import paper_1512_00066_amd as srtc
    rows = []
    i = 0
    name = ctypes.create_string_buffer(96)
    while True:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        st = srtc.lib().srtc_profile_query(ctx._h, i, name, 96, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by))
        if st != 0:
            break
        rows.append((name.value.decode(), n.value, ms.value, by.value))
        i += 1
    return rows


def rmat18_inputs(synth):
    scale, ef = 18, 16
    n = 1 << scale
    src, dst = synth.rmat_edges(scale, ef, 0.57, 0.19, 0.19, synth.SEED_CFG1)
    v64 = synth.edge_values("f64", src.size, synth.SEED_CFG1, 0)
    v32 = synth.edge_values("f32", src.size, synth.SEED_CFG1, 1)
    dims = (512, 512, 512)
    tkeys = synth.bernoulli_keys(dims, 1e-3, seed=synth.SEED_CFG1, tag=1)
    tv = synth.uniform_f32(synth.stream_key(synth.SEED_CFG1, 11), tkeys.size)
    M = synth.uniform_f32(synth.stream_key(synth.SEED_CFG1, 12), 512 * 64).reshape(512, 64)
    return dict(n=n, src=src, dst=dst, v64=v64, v32=v32, dims=dims, tkeys=tkeys, tv=tv, M=M)


def cpu_baseline_rmat18(inp, products_by_row, seconds):
    """The oracle on a bounded random sample of rows of the same workload
    (fp64 and fp32 A.A) plus the full tensor contraction; ops/s."""
    import oracle
    from gen import synth
    n = inp["n"]
    A64 = oracle.fold("plus_times", "f64", inp["dst"], inp["src"], inp["v64"], n, n)
    A32 = oracle.fold("plus_times", "f32", inp["dst"], inp["src"], inp["v32"], n, n)
    perm = synth.permutation(synth.stream_key(synth.SEED_CFG1, 77), n)
    w = products_by_row
    # calibrate on a small prefix, then size the sample to the time budget
    cum = np.cumsum(w[perm])
    k0 = int(np.searchsorted(cum, 2e7)) + 1
    t0 = time.perf_counter()
    oracle.spgemm("plus_times", "f64", A64, A64, rows=perm[:k0])
    rate = max(cum[k0 - 1] / max(time.perf_counter() - t0, 1e-3), 1.0)
    budget = rate * seconds / 2.2
    k = int(np.searchsorted(cum, budget)) + 1
    rows = perm[:k]
    ops = 0.0
    t = 0.0
    for A, dt in ((A64, "f64"), (A32, "f32")):
        t1 = time.perf_counter()
        oracle.spgemm("plus_times", dt, A, A, rows=rows)
        t += time.perf_counter() - t1
        ops += float(w[rows].sum())
    F = oracle.fold_tensor("plus_times", "f32", inp["tkeys"], inp["tv"], inp["dims"], "ijk", "ij", "k")
    t1 = time.perf_counter()
    oracle.spmm("plus_times", "f32", F, inp["M"])
    t += time.perf_counter() - t1
    ops += float(F.nnz) * 64
    return {"value": ops / t, "unit": "semiring-ops/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{k} of {n} rows (random) of both A.A products ({int(w[rows].sum())} products each) "
                      f"+ the full tensor contraction; {t:.1f} s"}


def oracle_timing(fn, reps):
    """Median seconds of `reps` runs of fn after one warm-up (the paper's
    protocol, Section 6)."""
    fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def roofline_of(prof, dominant=None):
    """Roofline record of the dominant kernel (the largest total time, or
    the named one): algorithmic bytes per launch over the average launch
    time (HIP events on the launch stream), HBM bytes from the committed
    counter record when it was taken on the current kernel sources."""
    if dominant is None:
        nm, cnt, tms, by = max(prof, key=lambda r: r[2])
    else:
        nm, cnt, tms, by = next(r for r in prof if r[0] == dominant)
    achieved = (by / cnt) / (tms / cnt / 1e3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        try:
            rec = json.load(open(tf))
            k = rec.get("kernels", {}).get(nm)
            if (k and rec.get("source_hash") == kernel_source_hash()
                    and rec.get("workload", "rmat18") == WORKLOAD_TAG[0]):
                traffic = k.get("hbm_bytes_per_launch")
        except Exception:
            traffic = None
    rec = {"bound": "hbm", "kernel": nm, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "avg_launch_ms": round(tms / cnt, 4),
           "algorithmic_bytes_per_launch": round(by / cnt), "launches": cnt}
    if traffic:
        # the measured form: counted HBM bytes over the same launch time
        rec["traffic_frac"] = round(traffic / (tms / cnt / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return rec


WORKLOAD_TAG = [""]


def train_selector(ctx, args):
    """A selector trained on timings of the training recipe (generated
    matrices as (+,x) fp32 and (min,+) int32 A.A, and row panels of R-MAT
    17-19 graphs), or loaded from --selector-file."""
    import torch
    import paper_1512_00066_amd as srtc
    from paper_1512_00066_amd import selector as S
    from gen import synth
    if args.selector_file:
        ctx.selector_load(args.selector_file)
        return {"loaded": args.selector_file}
    pairs = (("plus_times", "f32"), ("min_plus", "i32"))
    X, T = [], []
    t0 = time.perf_counter()
    for i in range(args.bench_selector_matrices):
        fam, n, src, dst, _ = synth.selector_matrix(i, synth.SEED_CFG4)
        keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
        for sr, dt in pairs:
            v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=i, lo=1, hi=100)
            A = ctx.fold(sr, srtc.COO(keys, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
            f, t = S.collect(ctx, sr, A, A, reps=3)
            X.append(f)
            T.append(t)
    for scale in (17, 18, 19):
        n = 1 << scale
        src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, synth.SEED_CFG4, tag=300 + scale)
        keys_b = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
        for sr, dt in pairs:
            v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=300 + scale, lo=1, hi=100)
            B = ctx.fold(sr, srtc.COO(keys_b, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
            for j in range(args.bench_selector_panels):
                rows = synth.selector_panel_rows(n, 1000 * scale + j, synth.SEED_CFG4)
                pos = np.full(n, -1, dtype=np.int64)
                pos[rows] = np.arange(rows.size)
                sel = pos[dst] >= 0
                Ap = ctx.fold(sr, srtc.COO(torch.as_tensor(pos[dst[sel]] * n + src[sel], device="cuda"),
                                           torch.as_tensor(v[sel], device="cuda"), (rows.size, n)), "ij", "i", "j")
                f, t = S.collect(ctx, sr, Ap, B, reps=3)
                X.append(f)
                T.append(t)
    X, T = np.array(X, np.float32), np.array(T, np.float64)
    t1 = time.perf_counter()
    loss = S.train(ctx, X, T, epochs=400, batch=64, lr=1e-3, seed=0)
    fixed = S.best_fixed(T)
    ev = S.evaluate(ctx, X, T, fixed)
    log(f"selector: {len(X)} samples collected in {t1 - t0:.1f} s, trained to loss {loss:.4f}; "
        f"in-sample regret {ev['mean_regret']:.3f}, gain over fixed schedule {fixed} {ev['total_gain']:.3f}")
    return {"samples": int(len(X)), "collect_s": round(t1 - t0, 1), "train_loss": loss, "fixed_schedule": fixed,
            "in_sample_mean_regret": ev["mean_regret"], "in_sample_gain": ev["total_gain"]}


def run_rmat21(args):
    """R-MAT scale 21 (2,097,152 vertices), edge factor 16, (a,b,c,d) =
    (0.57,0.19,0.19,0.05), relabelled: the full square C = A.A, whose
    output (2.4e10 entries) exceeds what one GPU holds in fp64, streamed in
    row panels through the library.  A step, for each of (+,x) fp64 (values
    U[0,1)), (+,x) fp32 and (min,+) int32 (weights U[1,100]): fold of the
    COO edge list to CSR, features and schedule selection by the learned
    selector, then every row panel's symbolic, numeric and compaction
    passes; each panel is handed to a consumer that releases it."""
    import torch
    import oracle
    import paper_1512_00066_amd as srtc
    from gen import synth

    WORKLOAD_TAG[0] = "rmat21"
    ctx = srtc.Context(0)
    scale = 21
    n = 1 << scale
    log("generating R-MAT 21 ...")
    src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, synth.SEED_CFG4, tag=21)
    kinds = (("plus_times", "f64"), ("plus_times", "f32"), ("min_plus", "i32"))
    vals = {dt: synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=21, lo=1, hi=100) for _, dt in kinds}
    keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
    coo = {dt: srtc.COO(keys, torch.as_tensor(vals[dt], device="cuda"), (n, n)) for _, dt in kinds}
    A = ctx.fold("plus_times", coo["f64"], "ij", "i", "j")
    rn = torch.diff(A.rowptr)
    wrow = torch.zeros(n, dtype=torch.int64, device="cuda")
    wrow.index_add_(0, torch.repeat_interleave(torch.arange(n, device="cuda"), rn), rn[A.col.long()])
    products = int(wrow.sum().item())
    wrow = wrow.cpu().numpy()
    del A, rn
    ops_step = len(kinds) * products
    log(f"nnz(A) entries generated {src.size}, products per A.A {products}, ops/step {ops_step:.4e}")
    sel_info = {"forced_schedule": args.schedule} if args.schedule >= 0 else train_selector(ctx, args)
    if args.schedule < 0:
        # the schedule the timed step will pick for each product (the same
        # features and network; reported, not used)
        picks = {}
        for sr, dt in kinds:
            Af = ctx.fold(sr, coo[dt], "ij", "i", "j")
            picks[dt] = ctx.select(ctx.features(sr, Af, Af))
            del Af
        sel_info["picks"] = picks
        log(f"selected schedules: {picks}")
    if args.dtypes:
        kinds = tuple(k for k in kinds if k[1] in args.dtypes.split(","))
        ops_step = len(kinds) * products
    budget = int(args.panel_products)
    nnz_out = {}

    def step():
        for sr, dt in kinds:
            Af = ctx.fold(sr, coo[dt], "ij", "i", "j")
            tot = [0]

            def consume(r0, P):
                tot[0] += P.nnz

            ctx.contract_panels(sr, "ik", Af, "kj", Af, "ij", consume, panel_products=budget, schedule=args.schedule)
            nnz_out[dt] = tot[0]
            del Af

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    srtc.lib().srtc_profile_enable(ctx._h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = profile_table(ctx)
    srtc.lib().srtc_profile_enable(ctx._h, 0)
    ms = (t1 - t0) * 1e3 / args.steps
    log(f"nnz(C) {nnz_out}; {ms:.1f} ms/step")
    log("kernel profile (name, launches, total ms, GB/s algorithmic):")
    for nm, cnt, tms, by in sorted(prof, key=lambda r: -r[2]):
        log(f"  {nm:34s} {cnt:5d} {tms:10.3f} {by / max(tms, 1e-9) / 1e6:10.1f}")
    out = {"metric": METRIC, "value": ops_step * args.steps / (t1 - t0), "unit": "semiring-ops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32+i32", "data": "synthetic",
           "config": {"workload": "rmat21_AxA_full_panels_f64_f32_i32", "rmat_scale": scale, "edge_factor": 16,
                      "abcd": [0.57, 0.19, 0.19, 0.05], "products_per_AxA": products, "nnz_C": nnz_out,
                      "panel_products": budget, "selector": sel_info},
           "roofline": roofline_of(prof)}
    if args.schedule < 0 and not args.no_regret:
        sel_info["held_out_rmat21"] = held_out_regret(ctx, coo, sel_info, budget)
    if not args.no_batch_comparison:
        del coo
        out["config"]["batched_vs_plain"] = batch_comparison(args)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline_sampled(n, src, dst, vals, kinds, wrow, args.cpu_seconds, synth.SEED_CFG4)
    return out


def batch_comparison(args):
    """The batched form against per-instance calls (the 512 uneven ER
    instances of --workload batch512: a (min,+) A.A and an 8-source
    Bellman-Ford fixpoint each, per-instance schedules from the exhaustive
    tuner), 2 timed steps after a warm-up, reported beside the default line
    (its own timing; not part of the line's value)."""
    import copy
    a2 = copy.copy(args)
    a2.steps, a2.warmup, a2.no_cpu_baseline, a2.schedule = 2, 1, True, -1
    o = run_batch512(a2)
    c = o["config"]
    return {"workload": c["workload"], "instances": c["instances"], "products": c["products"],
            "batched_ms_per_step": round(o["ms_per_step"], 2),
            "per_instance_ms_per_step": round(c["per_instance_ms_per_step"], 2),
            "speedup": round(c["batched_speedup"], 3), "batched_semiring_ops_per_s": o["value"],
            "batch_tuned_schedule": c["batch_tuned"]["schedule"],
            "batch_tuned_ms_per_step": round(c["batch_tuned"]["ms_per_step"], 2),
            "batch_tuned_speedup": round(c["batch_tuned"]["speedup_vs_per_instance"], 3),
            "dominant_kernel": o["roofline"]["kernel"], "dominant_frac": o["roofline"]["frac"]}


def held_out_regret(ctx, coo, sel_info, budget):
    """The selector on the matrix it never saw: the full R-MAT 21 square in
    (+,x) fp32 and (min,+) int32, every schedule timed by streaming the whole
    product in panels (one warm-up, then the median of 3; a schedule whose
    warm-up takes over 3x the best one so far keeps its warm-up time, which
    cannot change the best).  Regret = T_pick / T_best - 1; gain = T_fixed /
    T_pick with the best fixed schedule of the training set.  Untimed."""
    import torch
    import paper_1512_00066_amd as srtc
    res = {}
    for sr, dt in (("plus_times", "f32"), ("min_plus", "i32")):
        Af = ctx.fold(sr, coo[dt], "ij", "i", "j")

        def once(sch):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.contract_panels(sr, "ik", Af, "kj", Af, "ij", lambda r0, P: None, panel_products=budget,
                                schedule=sch)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3

        times = []
        for sch in range(srtc.NUM_SCHEDULES):
            w = once(sch)
            best = min(times) if times else w
            times.append(w if w > 3 * best else float(np.median([once(sch) for _ in range(3)])))
            log(f"held-out R-MAT 21 {dt} schedule {sch}: {times[-1]:.1f} ms")
        pick = sel_info["picks"][dt]
        fixed = sel_info.get("fixed_schedule", pick)
        res[dt] = {"times_ms": [round(x, 1) for x in times], "pick": pick, "best": int(np.argmin(times)),
                   "regret": round(times[pick] / min(times) - 1.0, 4),
                   "gain_over_fixed": round(times[fixed] / times[pick], 4)}
        log(f"held-out R-MAT 21 {dt}: pick {pick} best {res[dt]['best']} regret {res[dt]['regret']} "
            f"gain over fixed schedule {fixed} {res[dt]['gain_over_fixed']}")
        del Af
    return res


def cpu_baseline_sampled(n, src, dst, vals, kinds, w, seconds, seed):
    """The oracle on a bounded random sample of rows of the same products:
    median of 3 timed runs after a warm-up on all host threads, and on one
    thread for the first product, as semiring-ops/s."""
    import oracle
    from gen import synth
    Os = {dt: oracle.fold(sr, dt, dst, src, vals[dt], n, n) for sr, dt in kinds}
    perm = synth.permutation(synth.stream_key(seed, 77), n)
    cum = np.cumsum(w[perm])
    sr0, dt0 = kinds[0]
    k0 = int(np.searchsorted(cum, 2e7)) + 1
    t0 = time.perf_counter()
    oracle.spgemm(sr0, dt0, Os[dt0], Os[dt0], rows=np.sort(perm[:k0]))
    rate = max(cum[k0 - 1] / max(time.perf_counter() - t0, 1e-3), 1.0)
    # 4 runs per product (warm-up + 3) plus the one-thread runs: ~seconds total
    k = int(np.searchsorted(cum, rate * seconds / (5.0 * len(kinds)))) + 1
    rows = np.sort(perm[:k])
    ops = float(w[rows].sum())
    t_all = 0.0
    for sr, dt in kinds:
        t_all += oracle_timing(lambda: oracle.spgemm(sr, dt, Os[dt], Os[dt], rows=rows), 3)
    threads = oracle.num_threads()
    k1 = max(1, k // max(threads, 1))
    rows1 = np.sort(perm[:k1])
    oracle.set_threads(1)
    try:
        t1 = oracle_timing(lambda: oracle.spgemm(sr0, dt0, Os[dt0], Os[dt0], rows=rows1), 3)
    finally:
        oracle.set_threads(threads)
    return {"value": ops * len(kinds) / t_all, "unit": "semiring-ops/s", "cores": threads, "kind": "oracle",
            "value_one_thread": float(w[rows1].sum()) / t1,
            "sample": f"{k} random rows of each of the {len(kinds)} products ({int(ops)} products each), median "
                      f"of 3 runs after a warm-up; one thread: {k1} rows of the {dt0} product; the fold is not "
                      f"timed"}


def run_rmat18(args):
    import torch
    import paper_1512_00066_amd as srtc
    from gen import synth

    ctx = srtc.Context(0)
    log("generating R-MAT 18 and the order-3 tensor ...")
    inp = rmat18_inputs(synth)
    n = inp["n"]
    dev = "cuda"
    keysA = torch.as_tensor(inp["dst"].astype(np.int64) * n + inp["src"], device=dev)
    v64 = torch.as_tensor(inp["v64"], device=dev)
    v32 = torch.as_tensor(inp["v32"], device=dev)
    T = srtc.COO(torch.as_tensor(inp["tkeys"], device=dev), torch.as_tensor(inp["tv"], device=dev), inp["dims"])
    Md = torch.as_tensor(inp["M"], device=dev)
    Cd = torch.empty((512, 512, 64), dtype=torch.float32, device=dev)
    coo64 = srtc.COO(keysA, v64, (n, n))
    coo32 = srtc.COO(keysA, v32, (n, n))

    # exact operation count: products of A.A from the folded pattern
    A64 = ctx.fold("plus_times", coo64, "ij", "i", "j")
    rp = A64.rowptr.cpu().numpy()
    col = A64.col.cpu().numpy()
    rn = np.diff(rp)
    wrow = np.zeros(n, dtype=np.int64)
    np.add.at(wrow, np.repeat(np.arange(n), rn), rn[col])
    products = int(wrow.sum())
    t_nnz = int(inp["tkeys"].size)
    ops_step = 2 * products + 64 * t_nnz
    log(f"nnz(A)={A64.nnz} products={products} nnz(T)={t_nnz} ops/step={ops_step:.4e}")

    sched = {}
    if args.schedules:
        a, b = (int(x) for x in args.schedules.split(","))
        sched = {"f64": a, "f32": b}
    elif args.schedule >= 0:
        sched = {"f64": args.schedule, "f32": args.schedule}
    elif not args.no_autotune:
        A32 = ctx.fold("plus_times", coo32, "ij", "i", "j")
        for dt, A in (("f64", A64), ("f32", A32)):
            best, times = ctx.autotune("plus_times", A, A, reps=10)
            sched[dt] = best
            log(f"autotune {dt}: best={best} times_ms={np.round(times, 2).tolist()}")
        del A32
    del A64

    def step():
        outs = []
        for coo in (coo64, coo32):
            A = ctx.fold("plus_times", coo, "ij", "i", "j")
            C = ctx.contract("plus_times", "ik", A, "kj", A, "ij", schedule=-1 if not sched else
                             sched["f64" if coo is coo64 else "f32"], hub_tile=args.hub_tile)
            outs.append(C.nnz)
            del A, C
        ctx.contract("plus_times", "ijk", T, "kl", Md, "ijl", C=Cd)
        return outs

    for _ in range(args.warmup):
        nnz = step()
    torch.cuda.synchronize()
    srtc.lib().srtc_profile_enable(ctx._h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nnz = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = profile_table(ctx)
    srtc.lib().srtc_profile_enable(ctx._h, 0)
    ms = (t1 - t0) * 1e3 / args.steps
    value = ops_step * args.steps / (t1 - t0)
    log(f"nnz(C) f64/f32 = {nnz}; {ms:.2f} ms/step")
    log("kernel profile (name, launches, total ms, GB/s algorithmic):")
    for nm, cnt, tms, by in sorted(prof, key=lambda r: -r[2]):
        log(f"  {nm:32s} {cnt:5d} {tms:10.3f} {by / max(tms, 1e-9) / 1e6:10.1f}")
    WORKLOAD_TAG[0] = "rmat18"
    roof = roofline_of(prof)
    out = {"metric": METRIC, "value": value, "unit": "semiring-ops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "rmat18_AxA_f64_f32+tensor512_fold_contraction", "rmat_scale": 18,
                      "edge_factor": 16, "abcd": [0.57, 0.19, 0.19, 0.05], "tensor_dims": [512, 512, 512],
                      "tensor_density": 1e-3, "dense_M": [512, 64], "products_per_AxA": products,
                      "schedules": sched, "hub_tile": args.hub_tile},
           "roofline": roof}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline_rmat18(inp, wrow, args.cpu_seconds)
    return out


def run_rmat20_sssp(args):
    """Multi-source SSSP and BFS: R-MAT 20 (edge factor 16, int32 weights in
    [1,255]), 64 seeded sources; a step = fold + Bellman-Ford fixpoint as a
    (min,+) SpMM with graph-captured steps + bit-packed BFS."""
    import torch
    import oracle
    import paper_1512_00066_amd as srtc
    from gen import synth

    ctx = srtc.Context(0)
    scale, nsrc = 20, 64
    n = 1 << scale
    log("generating R-MAT 20 ...")
    src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, synth.SEED_CFG2)
    w = synth.edge_values("i32", src.size, synth.SEED_CFG2, lo=1, hi=255)
    sources = synth.pick_sources(n, src, nsrc, synth.SEED_CFG2)
    coo = srtc.COO(torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda"), torch.as_tensor(w, device="cuda"),
                   (n, n))
    P0 = np.full((n, nsrc), oracle.INT_INF, np.int32)
    P0[sources, np.arange(nsrc)] = 0
    P0d = torch.as_tensor(P0, device="cuda")
    X = torch.empty_like(P0d)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    rec = {}

    def step():
        A = ctx.fold("min_plus", coo, "ij", "i", "j")
        X.copy_(P0d)
        ev[0].record()
        it = ctx.fixpoint("min_plus", A, X, steps_per_check=4, changed_rows_only=args.changed_rows)
        ev[1].record()
        lev, depth = ctx.bfs_levels(A, sources)
        ev[2].record()
        rec.update(nnz=A.nnz, it=it, depth=depth)
        return A

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_bf = t_bfs = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        torch.cuda.synchronize()
        t_bf += ev[0].elapsed_time(ev[1])
        t_bfs += ev[1].elapsed_time(ev[2])
    t1 = time.perf_counter()
    nnz, it, depth = rec["nnz"], rec["it"], rec["depth"]
    ops_step = it * nnz * nsrc + (depth + 1) * nnz * nsrc
    ms = (t1 - t0) * 1e3 / args.steps
    # one fixpoint step reads A (col + val + rowptr), reads P and writes P
    step_bytes = 8.0 * nnz + 8.0 * (n + 1) + 2.0 * 4 * n * nsrc
    step_ms = t_bf / args.steps / it
    achieved = step_bytes / (step_ms / 1e3) / 1e9
    log(f"nnz(A)={nnz} BF steps={it} BFS depth={depth}; BF {t_bf / args.steps:.2f} ms, BFS {t_bfs / args.steps:.2f} ms, "
        f"step {ms:.2f} ms")
    out = {"metric": METRIC, "value": ops_step * args.steps / (t1 - t0), "unit": "semiring-ops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
           "config": {"workload": "rmat20_64src_bellman_ford_fixpoint+bfs", "rmat_scale": 20, "edge_factor": 16,
                      "weights": [1, 255], "sources": nsrc, "nnz_A": nnz, "bf_steps": it, "bfs_depth": depth,
                      "steps_per_graph": 4, "bf_ms": t_bf / args.steps, "bfs_ms": t_bfs / args.steps,
                      "changed_rows_only": bool(args.changed_rows),
                      "ops_note": "nnz(A) x sources per Bellman-Ford step and per BFS level; with changed-rows-only "
                                  "steps the iterates are the same and ops are counted as for full steps"},
           "roofline": {"bound": "hbm", "kernel": "spmm.fixpoint_step (graph-captured; fixpoint time / steps)",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "avg_launch_ms": round(step_ms, 4), "algorithmic_bytes_per_launch": round(step_bytes)}}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
        t2 = time.perf_counter()
        _, it_o, _ = oracle.bellman_ford("min_plus", "i32", O, P0)
        lev = oracle.bfs_levels(O, sources)
        t3 = time.perf_counter()
        ops_o = it_o * O.nnz * nsrc + (int(lev.max()) + 1) * O.nnz * nsrc
        out["cpu_baseline"] = {"value": ops_o / (t3 - t2), "unit": "semiring-ops/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"the whole workload: Bellman-Ford from all {nsrc} sources "
                               f"({it_o} steps) + BFS; {t3 - t2:.1f} s"}
    return out


def run_batch512(args):
    """512 uneven ER instances (n log-uniform in [1e3,1e5], degree uniform in
    [4,32], int32 weights [1,100]): each gets a (min,+) A.A and an 8-source
    Bellman-Ford fixpoint.  The step runs all instances batched (one set of
    persistent launches per phase); the same work as per-instance calls is
    timed in the same run for comparison, and so is the batched step with
    one schedule for the whole batch from the batch tuner."""
    import torch
    import oracle
    import paper_1512_00066_amd as srtc
    from gen import synth

    ctx = srtc.Context(0)
    ninst, nsrc = 512, 8
    ns, ds = synth.er_batch_params(ninst, synth.SEED_CFG3)
    log("generating 512 ER instances ...")
    As, X0s, host = [], [], []
    products = 0
    for b in range(ninst):
        n = int(ns[b])
        src, dst = synth.er_edges(n, float(ds[b]), synth.SEED_CFG3, tag=b)
        w = synth.edge_values("i32", src.size, synth.SEED_CFG3, tag=b, lo=1, hi=100)
        coo = srtc.COO(torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda"),
                       torch.as_tensor(w, device="cuda"), (n, n))
        A = ctx.fold("min_plus", coo, "ij", "i", "j")
        rn = torch.diff(A.rowptr)
        products += int(rn[A.col.long()].sum().item())
        sources = synth.pick_sources(n, src, nsrc, synth.SEED_CFG3, tag=b)
        X0 = torch.full((n, nsrc), oracle.INT_INF, dtype=torch.int32, device="cuda")
        X0[torch.as_tensor(sources, device="cuda"), torch.arange(sources.size, device="cuda")] = 0
        As.append(A)
        X0s.append(X0)
        host.append((src, dst, w, sources))
    nnz = [A.nnz for A in As]
    log(f"sum n={int(ns.sum())} sum nnz={sum(nnz)} products={products}")
    # SpGEMM schedules: one forced for every instance, or each instance's
    # own from the exhaustive tuner (median of 3 timed runs after a warm-up)
    if args.schedule >= 0:
        scheds = [args.schedule] * ninst
    else:
        t0 = time.perf_counter()
        scheds = [int(ctx.autotune("min_plus", A, A, reps=3)[0]) for A in As]
        log(f"per-instance autotune: {time.perf_counter() - t0:.1f} s; schedules used "
            f"{dict(zip(*np.unique(scheds, return_counts=True)))}")

    def batched():
        Cs = ctx.batch_contract("min_plus", As, As, schedules=scheds)
        Xs = [x.clone() for x in X0s]
        its = ctx.batch_fixpoint("min_plus", As, Xs, steps_per_check=4)
        del Cs, Xs
        return its

    def single():
        its = []
        for A, x0, sch in zip(As, X0s, scheds):
            C = ctx.contract("min_plus", "ik", A, "kj", A, "ij", schedule=sch)
            X = x0.clone()
            its.append(ctx.fixpoint("min_plus", A, X, steps_per_check=4))
            del C, X
        return its

    def timed(fn, k, profile=False):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        if profile:
            srtc.lib().srtc_profile_enable(ctx._h, 1)
        t0 = time.perf_counter()
        for _ in range(k):
            its = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k, its

    t_b, its_b = timed(batched, args.steps, profile=True)
    prof = profile_table(ctx)
    srtc.lib().srtc_profile_enable(ctx._h, 0)
    t_s, its_s = timed(single, max(1, args.steps // 2))
    assert list(its_b) == list(its_s), "batched and per-instance fixpoints took different step counts"
    # the same batched step with one schedule for the whole batch, chosen by
    # the batch tuner (every schedule timed on the batch as a whole)
    batch_tuned = None
    if args.schedule < 0:
        t0 = time.perf_counter()
        bbest, btimes = ctx.batch_autotune("min_plus", As, As, reps=3)
        tune_s = time.perf_counter() - t0

        def batched_one():
            Cs = ctx.batch_contract("min_plus", As, As)  # the batch tuner's cached pick
            Xs = [x.clone() for x in X0s]
            its = ctx.batch_fixpoint("min_plus", As, Xs, steps_per_check=4)
            del Cs, Xs
            return its

        t_1, its_1 = timed(batched_one, args.steps)
        assert list(its_1) == list(its_b), "the batch-tuned step took different fixpoint step counts"
        batch_tuned = {"schedule": int(bbest), "tune_s": round(tune_s, 1),
                       "spgemm_ms_per_schedule": [round(float(x), 2) for x in btimes],
                       "ms_per_step": t_1 * 1e3, "speedup_vs_per_instance": t_s / t_1}
        log(f"batch-tuned schedule {bbest}: {t_1 * 1e3:.2f} ms per step, {t_s / t_1:.2f}x the per-instance calls")
    ops_step = products + sum(it * z * nsrc for it, z in zip(its_b, nnz))
    log(f"batched {t_b * 1e3:.2f} ms, per-instance {t_s * 1e3:.2f} ms, speedup {t_s / t_b:.2f}x")
    log("kernel profile (batched steps):")
    for nm, cnt, tms, by in sorted(prof, key=lambda r: -r[2])[:12]:
        log(f"  {nm:32s} {cnt:5d} {tms:10.3f} {by / max(tms, 1e-9) / 1e6:10.1f}")
    nm, cnt, tms, by = max(prof, key=lambda r: r[2])
    achieved = (by / cnt) / (tms / cnt / 1e3) / 1e9
    out = {"metric": METRIC, "value": ops_step / t_b, "unit": "semiring-ops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t_b * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "i32", "data": "synthetic",
           "config": {"workload": "batch512_er_minplus_AxA+8src_bellman_ford", "instances": ninst,
                      "sum_n": int(ns.sum()), "sum_nnz": int(sum(nnz)), "products": products,
                      "bf_steps_max": int(max(its_b)), "per_instance_ms_per_step": t_s * 1e3,
                      "batched_speedup": t_s / t_b, "per_instance_value": ops_step / t_s,
                      "schedules": {int(k): int(v) for k, v in zip(*np.unique(scheds, return_counts=True))},
                      "batch_tuned": batch_tuned},
           "roofline": {"bound": "hbm", "kernel": nm, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "avg_launch_ms": round(tms / cnt, 4), "algorithmic_bytes_per_launch": round(by / cnt)}}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        ops_o, t_o, k = 0.0, 0.0, 0
        for b in range(ninst):
            src, dst, w, sources = host[b]
            n = int(ns[b])
            t2 = time.perf_counter()
            O = oracle.fold("min_plus", "i32", dst, src, w, n, n)
            t3 = time.perf_counter()
            C = oracle.spgemm("min_plus", "i32", O, O)
            P0 = np.full((n, nsrc), oracle.INT_INF, np.int32)
            P0[sources, np.arange(sources.size)] = 0
            _, it_o, _ = oracle.bellman_ford("min_plus", "i32", O, P0)
            t4 = time.perf_counter()
            rn = np.diff(O.rowptr)
            ops_o += float(rn[O.col].sum()) + it_o * O.nnz * nsrc
            t_o += t4 - t3
            k += 1
            if t_o > args.cpu_seconds:
                break
        out["cpu_baseline"] = {"value": ops_o / t_o, "unit": "semiring-ops/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"the first {k} of {ninst} instances (A.A + "
                               f"{nsrc}-source Bellman-Ford each); {t_o:.1f} s"}
    return out


def run_selector(args):
    """Learned schedule selection.  Training set: ``--selector-matrices``
    generated matrices (ER, R-MAT, 27-point stencil, power-law rows), each as
    (+,x) fp32 and (min,+) int32 A.A, plus ``--selector-panels`` row panels
    (2^10-2^14 random rows) of R-MAT graphs of scales 17-20 times the whole
    graph, every schedule timed by the exhaustive tuner; the MLP is trained
    on the GPU.  Held out: a row panel of R-MAT
    scale 21 (edge factor 16, default a,b,c,d; rows 0..2^18-1 of the
    relabelled graph, i.e. a random eighth) times the whole matrix, in both
    semirings.  The step timed is the held-out panel product with the
    selected schedule, both semirings."""
    import torch
    import oracle
    import paper_1512_00066_amd as srtc
    from paper_1512_00066_amd import selector as S
    from gen import synth

    ctx = srtc.Context(0)
    pairs = (("plus_times", "f32"), ("min_plus", "i32"))
    X, T, fams = [], [], []
    t0 = time.perf_counter()
    for i in range(args.selector_matrices):
        fam, n, src, dst, _ = synth.selector_matrix(i, synth.SEED_CFG4)
        keys = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
        for sr, dt in pairs:
            v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=i, lo=1, hi=100)
            A = ctx.fold(sr, srtc.COO(keys, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
            f, t = S.collect(ctx, sr, A, A, reps=2)
            X.append(f)
            T.append(t)
            fams.append(fam + "/" + sr)
            del A
        if i % 200 == 0:
            log(f"  training matrix {i}: {time.perf_counter() - t0:.1f} s")
    # wide matrices: row panels of R-MAT graphs of scales 17-20 times the
    # whole graph (up to 2^20 columns; the held-out panel below is of a
    # larger graph and a larger panel)
    for scale in args.selector_panel_scales:
        n = 1 << scale
        src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, synth.SEED_CFG4, tag=300 + scale)
        keys_b = torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda")
        for sr, dt in pairs:
            v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=300 + scale, lo=1, hi=100)
            B = ctx.fold(sr, srtc.COO(keys_b, torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
            for j in range(args.selector_panels):
                rows = synth.selector_panel_rows(n, 1000 * scale + j, synth.SEED_CFG4)
                pos = np.full(n, -1, dtype=np.int64)
                pos[rows] = np.arange(rows.size)
                sel = pos[dst] >= 0
                Ap = ctx.fold(sr, srtc.COO(torch.as_tensor(pos[dst[sel]] * n + src[sel], device="cuda"),
                                           torch.as_tensor(v[sel], device="cuda"), (rows.size, n)), "ij", "i", "j")
                f, t = S.collect(ctx, sr, Ap, B, reps=2)
                X.append(f)
                T.append(t)
                fams.append(f"panel{scale}/" + sr)
                del Ap
            del B
        log(f"  panels of R-MAT {scale}: {time.perf_counter() - t0:.1f} s")
    X, T = np.array(X, dtype=np.float32), np.array(T, dtype=np.float64)
    t_collect = time.perf_counter() - t0
    fixed = S.best_fixed(T)
    t1 = time.perf_counter()
    loss = S.train(ctx, X, T, epochs=args.selector_epochs, batch=128, lr=1e-3, seed=0)
    t_train = time.perf_counter() - t1
    ins = S.evaluate(ctx, X, T, fixed)
    log(f"collected {len(X)} samples in {t_collect:.1f} s; trained in {t_train:.1f} s, loss {loss:.4f}; "
        f"fixed schedule {fixed}; in-sample mean regret {ins['mean_regret']:.3f} "
        f"(fixed {ins['fixed_regret']:.3f}), gain {ins['total_gain']:.3f}")

    log("generating R-MAT 21 ...")
    scale = 21
    n = 1 << scale
    prow = 1 << 18
    src, dst = synth.rmat_edges(scale, 16, 0.57, 0.19, 0.19, synth.SEED_CFG4, tag=21)
    sel = dst < prow
    held = {}
    for sr, dt in pairs:
        v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=21, lo=1, hi=100)
        B = ctx.fold(sr, srtc.COO(torch.as_tensor(dst.astype(np.int64) * n + src, device="cuda"),
                                  torch.as_tensor(v, device="cuda"), (n, n)), "ij", "i", "j")
        Ap = ctx.fold(sr, srtc.COO(torch.as_tensor(dst[sel].astype(np.int64) * n + src[sel], device="cuda"),
                                   torch.as_tensor(v[sel], device="cuda"), (prow, n)), "ij", "i", "j")
        # the ground truth of the held-out regret: median of 10 after a warm-up
        f, t = S.collect(ctx, sr, Ap, B, reps=10)
        ev = S.evaluate(ctx, f[None, :], t[None, :], fixed)
        rp = Ap.rowptr
        nb = torch.diff(B.rowptr)
        products = int(nb[Ap.col.long()].sum().item())
        held[sr] = {"times_ms": [round(float(x), 3) for x in t], "pick": ev["picks"][0], "best": int(np.argmin(t)),
                    "regret": ev["regret"][0], "gain_over_fixed": ev["gain"][0], "products": products, "A": Ap, "B": B}
        log(f"held-out {sr}: times {np.round(t, 1).tolist()} pick {ev['picks'][0]} best {int(np.argmin(t))} "
            f"regret {ev['regret'][0]:.3f} gain over fixed {ev['gain'][0]:.3f}")

    def step():
        for sr, _ in pairs:
            h = held[sr]
            C = ctx.contract(sr, "ik", h["A"], "kj", h["B"], "ij", schedule=h["pick"])
            del C

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    srtc.lib().srtc_profile_enable(ctx._h, 1)
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = profile_table(ctx)
    srtc.lib().srtc_profile_enable(ctx._h, 0)
    ms = (t3 - t2) * 1e3 / args.steps
    ops_step = sum(held[sr]["products"] for sr, _ in pairs)
    nm, cnt, tms, by = max(prof, key=lambda r: r[2])
    achieved = (by / cnt) / (tms / cnt / 1e3) / 1e9
    out = {"metric": METRIC, "value": ops_step / (ms / 1e3), "unit": "semiring-ops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+i32", "data": "synthetic",
           "config": {"workload": "rmat21_panel_AxA_learned_schedule", "rmat_scale": 21, "edge_factor": 16,
                      "panel_rows": prow, "training_samples": int(len(X)), "training_matrices": args.selector_matrices,
                      "training_panels": args.selector_panels * len(args.selector_panel_scales),
                      "fixed_schedule": fixed, "train_loss": loss, "collect_s": t_collect, "train_s": t_train,
                      "in_sample": {k: ins[k] for k in ("mean_regret", "max_regret", "fixed_regret", "total_gain",
                                                         "hits")},
                      "held_out": {sr: {k: v for k, v in h.items() if k not in ("A", "B")} for sr, h in held.items()}},
           "roofline": {"bound": "hbm", "kernel": nm, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "avg_launch_ms": round(tms / cnt, 4), "algorithmic_bytes_per_launch": round(by / cnt)}}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        sr, dt = pairs[0]
        v = synth.edge_values(dt, src.size, synth.SEED_CFG4, tag=21)
        Bo = oracle.fold(sr, dt, dst, src, v, n, n)
        nb = np.diff(Bo.rowptr)
        w = np.zeros(n, dtype=np.int64)
        np.add.at(w, np.repeat(np.arange(n), nb), nb[Bo.col])
        perm = synth.permutation(synth.stream_key(synth.SEED_CFG4, 77), prow)
        k, t_o, ops_o = 256, 0.0, 0.0
        while t_o < args.cpu_seconds / 2 and k <= prow:
            rows = perm[:k]
            t4 = time.perf_counter()
            oracle.spgemm(sr, dt, Bo, Bo, rows=rows)
            t_o = time.perf_counter() - t4
            ops_o = float(w[rows].sum())
            k *= 2
        out["cpu_baseline"] = {"value": ops_o / t_o, "unit": "semiring-ops/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{k // 2} random panel rows of the (+,x) fp32 product "
                               f"({int(ops_o)} products); {t_o:.1f} s"}
    return out


def run_masked18(args):
    """Masked contraction on R-MAT 18 (edge factor 16, fp64 values): C = A (.)
    (A.A) over A's own pattern (the shape of triangle counting); every
    product is formed and tested against the mask row.  A step = fold + the
    masked contraction."""
    import torch
    import oracle
    import paper_1512_00066_amd as srtc
    from gen import synth

    ctx = srtc.Context(0)
    inp = rmat18_inputs(synth)
    n = inp["n"]
    coo = srtc.COO(torch.as_tensor(inp["dst"].astype(np.int64) * n + inp["src"], device="cuda"),
                   torch.as_tensor(inp["v64"], device="cuda"), (n, n))
    A0 = ctx.fold("plus_times", coo, "ij", "i", "j")
    rn = torch.diff(A0.rowptr)
    products = int(rn[A0.col.long()].sum().item())

    def step():
        A = ctx.fold("plus_times", coo, "ij", "i", "j")
        C = ctx.contract_masked("plus_times", "ik", A, "kj", A, "ij", A)
        return C.nnz

    for _ in range(args.warmup):
        nz = step()
    torch.cuda.synchronize()
    srtc.lib().srtc_profile_enable(ctx._h, 1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nz = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = profile_table(ctx)
    srtc.lib().srtc_profile_enable(ctx._h, 0)
    ms = (t1 - t0) * 1e3 / args.steps
    nm, cnt, tms, by = max(prof, key=lambda r: r[2])
    achieved = (by / cnt) / (tms / cnt / 1e3) / 1e9
    log(f"masked: products {products}, nnz(C) {nz}, {ms:.2f} ms/step")
    out = {"metric": METRIC, "value": products / (ms / 1e3), "unit": "semiring-ops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "rmat18_masked_A_dot_AxA_f64", "rmat_scale": 18, "edge_factor": 16,
                      "products": products, "nnz_C": nz, "mask_nnz": A0.nnz},
           "roofline": {"bound": "hbm", "kernel": nm, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "avg_launch_ms": round(tms / cnt, 4), "algorithmic_bytes_per_launch": round(by / cnt)}}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        O = oracle.fold("plus_times", "f64", inp["dst"], inp["src"], inp["v64"], n, n)
        rno = np.diff(O.rowptr)
        w = np.zeros(n, dtype=np.int64)
        np.add.at(w, np.repeat(np.arange(n), rno), rno[O.col])
        perm = synth.permutation(synth.stream_key(synth.SEED_CFG1, 78), n)
        k, t_o, ops_o = 1024, 0.0, 0.0
        while t_o < args.cpu_seconds / 2 and k <= n:
            rows = np.sort(perm[:k])
            Asub = oracle.CSR(np.concatenate([[0], np.cumsum(rno[rows])]),
                              np.concatenate([O.col[O.rowptr[r]:O.rowptr[r + 1]] for r in rows]),
                              np.concatenate([O.val[O.rowptr[r]:O.rowptr[r + 1]] for r in rows]), k, n)
            t2 = time.perf_counter()
            oracle.spgemm_masked("plus_times", "f64", Asub, O, Asub)
            t_o = time.perf_counter() - t2
            ops_o = float(w[rows].sum())
            k *= 2
        out["cpu_baseline"] = {"value": ops_o / t_o, "unit": "semiring-ops/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{k // 2} random rows ({int(ops_o)} products); {t_o:.1f} s"}
    return out


def run_apsp2048(args):
    """All-pairs shortest paths by Tiskin's path doubling on the paper's APSP
    workload: a complete directed graph on n = 2,048 vertices with integer
    weights uniform in [1, n^2].  A step = fold of the edge list + every
    round (sparsify the exactly-l-hop paths, P <- P (+) P_l (x) P over packed
    (weight, hops) paths) + distance/hop extraction.  Ops = path sums formed,
    sum over rounds of nnz(P_l) * n."""
    import torch
    import oracle
    import paper_1512_00066_amd as srtc
    from gen import synth

    ctx = srtc.Context(0)
    n = args.apsp_n
    src, dst, w = synth.dense_graph(n, synth.SEED_CFG0)
    coo = srtc.COO(torch.as_tensor(dst * n + src, device="cuda"), torch.as_tensor(w, device="cuda"), (n, n))
    rn = []

    def step():
        return ctx.apsp_tiskin(coo, round_nnz=rn)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    srtc.lib().srtc_profile_enable(ctx._h, 1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, H, rounds = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = profile_table(ctx)
    srtc.lib().srtc_profile_enable(ctx._h, 0)
    ms = (t1 - t0) * 1e3 / args.steps
    ops = float(sum(rn)) * n
    dense_rounds = int(np.ceil(np.log2(n)))
    for r in prof:
        log(f"  {r[0]:28s} launches {r[1] // args.steps:3d}/step  {r[2] / args.steps:8.3f} ms/step")
    nm, cnt, tms, _ = max(prof, key=lambda r: r[2])
    # ALU bound of the dominant kernel, from the instructions one path sum
    # takes per lane at 64 lanes x 256 CUs x 2.4 GHz: 32-bit tiles an add
    # and half a three-way min (1.5), 64-bit tiles a 64-bit add, a 64-bit
    # compare and two selects (4); the CSR x dense product about 6 with its
    # identity tests.  Dense rounds form all n^3 sums of a round (identity
    # operands included); the CSR product forms nnz(P_l) * n.
    per_sum = {"apsp.dense_round.u32": 1.5, "apsp.dense_round.u64": 4.0}.get(nm, 6.0)
    alu_peak = 256 * 64 * 2.4e9 / per_sum / 1e12
    if nm.startswith("apsp.dense_round"):
        sums_per_launch = float(n) ** 3
    else:
        sparse_rounds = [x for x in rn if x < 0.25 * n * n]
        sums_per_launch = float(sum(sparse_rounds)) * n / max(1, len(sparse_rounds))
    achieved = sums_per_launch / (tms / cnt / 1e3) / 1e12
    log(f"apsp n={n}: rounds {rounds}, nnz(P_l) {rn}, max hops {int(H.max())}, {ms:.2f} ms/step; "
        f"dominant {nm}: {tms / cnt:.3f} ms/launch")
    out = {"metric": METRIC, "value": ops / (ms / 1e3), "unit": "semiring-ops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64 (i32 weight, u32 hops)", "data": "synthetic",
           "config": {"workload": f"apsp_tiskin_dense{n}", "n": n, "weights": [1, n * n], "rounds": rounds,
                      "round_nnz": rn, "path_sums": ops, "dense_doubling_path_sums": float(dense_rounds) * n ** 3,
                      "work_ratio_vs_dense_doubling": round(ops / (float(dense_rounds) * n ** 3), 4),
                      "kernels_ms_per_step": {r[0]: round(r[2] / args.steps, 4) for r in prof}},
           "roofline": {"bound": "alu", "kernel": nm, "achieved": round(achieved, 3), "peak": round(alu_peak, 3),
                        "unit": "T path-sums/s", "frac": round(achieved / alu_peak, 4), "traffic": None,
                        "avg_launch_ms": round(tms / cnt, 4), "path_sums_per_launch": sums_per_launch}}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        m, t_o, ops_o = 256, 0.0, 0.0
        while t_o < args.cpu_seconds / 4 and m <= n:
            s2, d2, w2 = synth.dense_graph(m, synth.SEED_CFG0)
            O = oracle.fold("min_plus", "i32", d2, s2, w2, m, m)
            t2 = time.perf_counter()
            _, _, _, pl = oracle.apsp_tiskin(O)
            t_o = time.perf_counter() - t2
            ops_o = float(sum(pl)) * m
            m *= 2
        m //= 2
        reps = 1
        while t_o < args.cpu_seconds / 2:   # the whole solve is short: repeat it
            t2 = time.perf_counter()
            oracle.apsp_tiskin(O)
            t_o += time.perf_counter() - t2
            ops_o += float(sum(pl)) * m
            reps += 1
        out["cpu_baseline"] = {"value": ops_o / t_o, "unit": "semiring-ops/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"the same recipe at n = {m}, {reps} solves "
                               f"({int(ops_o)} path sums); {t_o:.1f} s"}
    return out


def run_mp3(args):
    """The MP3 energy of Section 4.3 on a synthetic system (Section 6's MP3
    experiment): m occupied and n virtual orbitals, the five integral
    tensors 1% sparse (fp64, Bernoulli pattern), Fock blocks and amplitudes
    dense.  A step = every contraction of the MP3 listing: T = V (.) D, Z =
    Fab.T - Fij.T + Vabcd.T/2 + Vijkl.T/2 - Vaibj.T (three of them with their
    outputs folded back, the last with T permuted), T += Z (.) D, and the
    energy T.V.  The listing's scalar factors are folded into the synthetic
    inputs; the copy Z = Vijab and the denominator D (broadcast sums and a
    reciprocal) are inputs.  Ops = multiply-adds: nonzeros x dense extent
    for sparse terms, M N K for dense ones, one per entry for elementwise."""
    import torch
    import oracle
    import paper_1512_00066_amd as srtc
    from gen import synth

    ctx = srtc.Context(0)
    m, n = args.mp3_m, args.mp3_n
    seed = synth.SEED_CFG1
    dens = 0.01

    def sparse(dims, tag, scale=1.0):
        keys = synth.bernoulli_keys(dims, dens, seed=seed, tag=tag)
        vals = synth.edge_values("f64", keys.size, seed, tag) * scale
        return srtc.COO(torch.as_tensor(keys, device="cuda"), torch.as_tensor(vals, device="cuda"), dims), keys, vals

    def dense(dims, tag, lo=0.0, hi=1.0):
        v = lo + (hi - lo) * synth.uniform_f64(synth.stream_key(seed, 200 + tag), int(np.prod(dims)))
        return torch.as_tensor(v.reshape(dims), device="cuda")

    log(f"generating MP3 tensors m={m} n={n} ...")
    Vabij, _, _ = sparse((n, n, m, m), 1)
    Vabcd, kabcd, vabcd = sparse((n, n, n, n), 2, 0.5)
    Vijkl, _, _ = sparse((m, m, m, m), 3, 0.5)
    Vaibj, _, _ = sparse((n, m, n, m), 4, -1.0)          # letters a m e i
    Fab = dense((n, n), 5, -0.1, 0.1)
    Fij = dense((m, m), 6, -0.1, 0.1)                    # -Fij folded in
    ea = synth.uniform_f64(synth.stream_key(seed, 7), n) + 1.0    # virtual energies in [1, 2)
    ei = synth.uniform_f64(synth.stream_key(seed, 8), m) - 2.0    # occupied energies in [-2, -1)
    den = -ea[:, None, None, None] - ea[None, :, None, None] + ei[None, None, :, None] + ei[None, None, None, :]
    D = torch.as_tensor(1.0 / den, device="cuda")
    T = torch.empty((n, n, m, m), dtype=torch.float64, device="cuda")
    Z = torch.empty_like(T)
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    terms = []

    def step():
        ctx.contract("plus_times", "abij", Vabij, "abij", D, "abij", C=T)
        ctx.contract("plus_times", "af", Fab, "fbij", T, "abij", C=Z)
        ctx.contract("plus_times", "ni", Fij, "abnj", T, "abij", C=Z, accumulate=True)
        ctx.contract("plus_times", "abef", Vabcd, "efij", T, "abij", C=Z, accumulate=True)
        ctx.contract("plus_times", "mnij", Vijkl, "abmn", T, "abij", C=Z, accumulate=True)
        ctx.contract("plus_times", "amei", Vaibj, "ebmj", T, "abij", C=Z, accumulate=True)
        ctx.contract("plus_times", "abij", Z, "abij", D, "abij", C=T, accumulate=True)
        ctx.contract("plus_times", "abij", Vabij, "abij", T, "", C=E)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    srtc.lib().srtc_profile_enable(ctx._h, 1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = profile_table(ctx)
    srtc.lib().srtc_profile_enable(ctx._h, 0)
    ms = (t1 - t0) * 1e3 / args.steps
    nnz = {k: int(t.keys.numel()) for k, t in (("Vabij", Vabij), ("Vabcd", Vabcd), ("Vijkl", Vijkl),
                                               ("Vaibj", Vaibj))}
    dense_t = n * n * m * m
    ops = (nnz["Vabij"] + n * n * (n * m * m) + m * m * (n * n * m) + nnz["Vabcd"] * m * m + nnz["Vijkl"] * n * n
           + nnz["Vaibj"] * n * m + dense_t + nnz["Vabij"])
    for r in prof:
        log(f"  {r[0]:28s} launches {r[1] // args.steps:3d}/step  {r[2] / args.steps:8.3f} ms/step")
    nm, cnt, tms, by = max(prof, key=lambda r: r[2])
    if nm.startswith("dense.gemm_mfma"):
        flops = 2.0 * (n * n * (n * m * m) + m * m * (n * n * m)) * args.steps
        achieved, peak, unit, bound = flops / (tms / 1e3) / 1e12, 78.6, "TFLOP/s", "mfma"
    else:
        achieved, peak, unit, bound = (by / cnt) / (tms / cnt / 1e3) / 1e9, HBM_PEAK_GBS, "GB/s", "hbm"
    log(f"mp3 m={m} n={n}: nnz {nnz}, E = {float(E.item()):.6e}, {ms:.2f} ms/step")
    out = {"metric": METRIC, "value": ops / (ms / 1e3), "unit": "semiring-ops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"mp3_m{m}_n{n}_1pct", "m": m, "n": n, "density": dens, "nnz": nnz,
                      "ops_per_step": ops, "energy": float(E.item()),
                      "kernels_ms_per_step": {r[0]: round(r[2] / args.steps, 4) for r in prof}},
           "roofline": {"bound": bound, "kernel": nm, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                        "frac": round(achieved / peak, 4), "traffic": None, "avg_launch_ms": round(tms / cnt, 4)}}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        # the largest term, Vabcd["abef"] T["efij"], on random (a, b) rows
        O = oracle.fold_tensor("plus_times", "f64", kabcd, vabcd, (n, n, n, n), "abef", "ab", "ef")
        Tm = T.cpu().numpy().reshape(n * n, m * m)
        rno = np.diff(O.rowptr)
        perm = synth.permutation(synth.stream_key(seed, 79), n * n)
        k, t_o, ops_o = 256, 0.0, 0.0
        while t_o < args.cpu_seconds / 2 and k <= n * n:
            rows = np.sort(perm[:k])
            sub = oracle.CSR(np.concatenate([[0], np.cumsum(rno[rows])]),
                             np.concatenate([O.col[O.rowptr[r]:O.rowptr[r + 1]] for r in rows]),
                             np.concatenate([O.val[O.rowptr[r]:O.rowptr[r + 1]] for r in rows]), k, n * n)
            t2 = time.perf_counter()
            oracle.spmm("plus_times", "f64", sub, Tm)
            t_o = time.perf_counter() - t2
            ops_o = float(sub.nnz) * m * m
            k *= 2
        reps = 1
        while t_o < args.cpu_seconds / 2:   # every row already: repeat
            t2 = time.perf_counter()
            oracle.spmm("plus_times", "f64", sub, Tm)
            t_o += time.perf_counter() - t2
            ops_o += float(sub.nnz) * m * m
            reps += 1
        out["cpu_baseline"] = {"value": ops_o / t_o, "unit": "semiring-ops/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"Vabcd.T on {sub.nrows} random (a,b) rows, {reps} "
                               f"runs ({int(ops_o)} multiply-adds); {t_o:.1f} s"}
    return out


def run_jacobi(args):
    """Jacobi iteration (Section 4.1) on the 27-point stencil of a g^3 grid
    (g = 128: 2.1M unknowns, 55.9M nonzeros, fp64; diagonal 27, neighbours
    -1, so strictly diagonally dominant) with b uniform in [0, 1): a step =
    fold of the COO matrix + the whole solve from x = 0 to |b - A x| <= 1e-8.
    Ops = nonzeros per update (one multiply-add each)."""
    import torch
    import oracle
    import paper_1512_00066_amd as srtc
    from gen import synth

    ctx = srtc.Context(0)
    g = args.jacobi_g
    n = g ** 3
    log(f"generating the 27-point stencil g={g} ...")
    src, dst = synth.stencil27_edges(g)
    vals = np.where(src == dst, 27.0, -1.0)
    b = synth.uniform_f64(synth.stream_key(synth.SEED_CFG4, 31), n)
    coo = srtc.COO(torch.as_tensor(dst * n + src, device="cuda"), torch.as_tensor(vals, device="cuda"), (n, n))
    bd = torch.as_tensor(b, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    tol = 1e-8

    def step():
        x.zero_()
        return ctx.jacobi(coo, bd, x, tol=tol, steps_per_check=32)

    for _ in range(args.warmup):
        it, r = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        it, r = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    # time per update from two capped solves (the difference cancels the
    # fold and set-up)
    A = ctx.fold("plus_times", coo, "ij", "i", "j")

    def capped(cap):
        x.zero_()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        try:
            ctx.jacobi(A, bd, x, tol=0.0, max_iters=cap, steps_per_check=32)
        except srtc.NotConverged:
            pass
        torch.cuda.synchronize()
        return time.perf_counter() - ta

    capped(64)
    t_lo, t_hi = min(capped(64) for _ in range(3)), min(capped(576) for _ in range(3))
    step_ms = (t_hi - t_lo) * 1e3 / 512
    nnz = A.nnz
    step_bytes = 12.0 * nnz + 8.0 * (n + 1) + 32.0 * n
    achieved = step_bytes / (step_ms / 1e3) / 1e9
    log(f"jacobi g={g}: n={n} nnz={nnz}, {it} updates to |r| = {r:.3e}, {ms:.2f} ms/solve, {step_ms * 1e3:.1f} us/update")
    out = {"metric": METRIC, "value": float(it) * nnz / (ms / 1e3), "unit": "semiring-ops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"jacobi_stencil27_g{g}", "n": n, "nnz": nnz, "tol": tol, "updates": it,
                      "residual": r, "us_per_update": step_ms * 1e3},
           "roofline": {"bound": "hbm", "kernel": "jacobi_step (graph-captured; from the time of 512 extra updates)",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "avg_launch_ms": round(step_ms, 4), "algorithmic_bytes_per_launch": round(step_bytes)}}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        O = oracle.fold("plus_times", "f64", dst, src, vals, n, n)
        k, t_o = 2, 0.0
        while t_o < args.cpu_seconds / 2:
            t2 = time.perf_counter()
            oracle.jacobi(O, b, np.zeros(n), 0.0, max_iters=k)
            t_o = time.perf_counter() - t2
            k *= 2
        out["cpu_baseline"] = {"value": float(k // 2) * O.nnz / t_o, "unit": "semiring-ops/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"{k // 2} updates of the full system; {t_o:.1f} s"}
    return out


def run_gemm(args):
    """The dense (+,x) tile path on its own: C["ij"] = A["ik"] B["kj"] with
    dense fp64 operands of M = N = K = 8,192 (values uniform in [0,1)) on
    the matrix cores, plus the same in fp32 (fp64 flushes).  A step = both
    products.  Ops = multiply-adds (M N K per product)."""
    import torch
    import paper_1512_00066_amd as srtc
    from gen import synth

    ctx = srtc.Context(0)
    n = args.gemm_n
    res = {}
    for dt, tt in (("f64", torch.float64), ("f32", torch.float32)):
        A = torch.as_tensor(synth.uniform_f64(synth.stream_key(5, 1), n * n).reshape(n, n), device="cuda").to(tt)
        B = torch.as_tensor(synth.uniform_f64(synth.stream_key(5, 2), n * n).reshape(n, n), device="cuda").to(tt)
        C = torch.empty((n, n), dtype=tt, device="cuda")
        res[dt] = (A, B, C)

    def step():
        for dt in ("f64", "f32"):
            A, B, C = res[dt]
            ctx.contract("plus_times", "ik", A, "kj", B, "ij", C=C)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    srtc.lib().srtc_profile_enable(ctx._h, 1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = profile_table(ctx)
    srtc.lib().srtc_profile_enable(ctx._h, 0)
    ms = (t1 - t0) * 1e3 / args.steps
    flops = 2.0 * n ** 3
    rate = {}
    for nm, cnt, tms, _ in prof:
        if nm.startswith("dense.gemm_mfma"):
            rate[nm] = (tms / cnt, flops / (tms / cnt / 1e3) / 1e12)
    f64_ms, f64_tf = rate["dense.gemm_mfma.f64"]
    f32_ms, f32_tf = rate["dense.gemm_mfma.f32"]
    log(f"gemm n={n}: {ms:.2f} ms/step; fp64 {f64_ms:.3f} ms = {f64_tf:.1f} TFLOP/s, "
        f"fp32 {f32_ms:.3f} ms = {f32_tf:.1f} TFLOP/s")
    out = {"metric": METRIC, "value": 2 * n ** 3 / (ms / 1e3), "unit": "semiring-ops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": f"dense_gemm_{n}_f64_f32", "n": n,
                      "f32": {"ms_per_launch": round(f32_ms, 4), "tflops": round(f32_tf, 2), "peak": 157.3,
                              "frac": round(f32_tf / 157.3, 4)}},
           "roofline": {"bound": "mfma", "kernel": "dense.gemm_mfma.f64", "achieved": round(f64_tf, 2),
                        "peak": 78.6, "unit": "TFLOP/s", "frac": round(f64_tf / 78.6, 4), "traffic": None,
                        "avg_launch_ms": round(f64_ms, 4)}}
    if not args.no_cpu_baseline:
        import oracle
        log("timing the oracle on the host ...")
        k, t_o, ops_o = 1024, 0.0, 0.0
        while t_o < args.cpu_seconds / 2 and k <= n:
            a = synth.uniform_f64(synth.stream_key(5, 3), k * k).reshape(k, k)
            t2 = time.perf_counter()
            oracle.dense_plus_times(a, a)
            t_o = time.perf_counter() - t2
            ops_o = float(k) ** 3
            k *= 2
        reps = 1
        while t_o < args.cpu_seconds / 2:   # the full size is short: repeat it
            t2 = time.perf_counter()
            oracle.dense_plus_times(a, a)
            t_o += time.perf_counter() - t2
            ops_o += float(k // 2) ** 3
            reps += 1
        out["cpu_baseline"] = {"value": ops_o / t_o, "unit": "semiring-ops/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{reps} fp64 products of size {k // 2}^3; {t_o:.1f} s"}
    return out


def copy_calibration(args):
    """A plain device copy of known size (1 GiB read, 1 GiB written per
    launch), run under the same HBM counters as the kernels, to scale
    FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # the achievable HBM rate of a plain copy (bytes read + written per second)
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": args.steps,
                      "ms_per_copy": round(ms, 4), "copy_GBps": round(2 * nbytes / (ms / 1e3) / 1e9, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat21", choices=["rmat21", "rmat18", "rmat20_sssp", "batch512", "selector",
                                                               "masked18", "apsp2048", "mp3", "jacobi", "gemm"])
    ap.add_argument("--panel-products", type=float, default=8e9,
                    help="rmat21: products per row panel of the streamed product")
    ap.add_argument("--selector-file", default="", help="rmat21: load the selector instead of training it")
    ap.add_argument("--dtypes", default="", help="rmat21: only these of f64,f32,i32 (profiling runs)")
    ap.add_argument("--bench-selector-matrices", type=int, default=160,
                    help="rmat21: generated training matrices for the selector")
    ap.add_argument("--bench-selector-panels", type=int, default=6,
                    help="rmat21: row panels per R-MAT scale 17-19 in the selector's training set")
    ap.add_argument("--schedule", type=int, default=-1, help="force one SpGEMM schedule")
    ap.add_argument("--schedules", default="", help="SpGEMM schedules for fp64,fp32 (e.g. 0,5)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--hub-tile", type=int, default=0, help="rmat18: hub block formed on the matrix cores")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch-comparison", action="store_true",
                    help="rmat21: skip the batched-vs-per-instance comparison of the 512 ER instances")
    ap.add_argument("--no-regret", action="store_true",
                    help="rmat21: skip timing every schedule on the full product (the selector's held-out regret)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--selector-matrices", type=int, default=2000)
    ap.add_argument("--selector-epochs", type=int, default=400)
    ap.add_argument("--selector-panels", type=int, default=40, help="selector: wide row panels per R-MAT scale")
    ap.add_argument("--selector-panel-scales", type=int, nargs="*", default=[17, 18, 19, 20])
    ap.add_argument("--apsp-n", type=int, default=2048, help="apsp2048: vertices of the dense graph")
    ap.add_argument("--mp3-m", type=int, default=32, help="mp3: occupied orbitals")
    ap.add_argument("--jacobi-g", type=int, default=128, help="jacobi: grid side of the 27-point stencil")
    ap.add_argument("--gemm-n", type=int, default=8192, help="gemm: M = N = K of the dense products")
    ap.add_argument("--mp3-n", type=int, default=128, help="mp3: virtual orbitals")
    ap.add_argument("--changed-rows", action="store_true",
                    help="rmat20_sssp: fixpoint steps gather only from rows changed in the previous step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args)
        return
    out = {"rmat21": run_rmat21, "rmat18": run_rmat18, "rmat20_sssp": run_rmat20_sssp, "batch512": run_batch512,
           "selector": run_selector, "masked18": run_masked18, "apsp2048": run_apsp2048,
           "mp3": run_mp3, "jacobi": run_jacobi, "gemm": run_gemm}[args.workload](args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
