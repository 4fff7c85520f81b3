#!/usr/bin/env python3
"""Benchmark of the semiring contraction hot path on one MI355X.

Default workload (one "step" = every hot-path stage this workload uses,
over one batch of synthetic input already resident in HBM):
  * R-MAT scale 18 (262,144 vertices), edge factor 16,
    (a,b,c,d) = (0.57,0.19,0.19,0.05), relabelled; values U[0,1)
    - fold of the COO edge list to CSR (fp64), schedule selection,
      C = A.A over (+,x) fp64: symbolic, numeric, compaction
    - the same in fp32 (exact products, fp64 accumulation)
  * order-3 tensor T[512,512,512] (Bernoulli 1e-3, fp32) contracted with a
    dense M[512,64]: C["ijl"] = T["ijk"] * M["kl"] (fold + SpMM)
Metric: semiring ops per second (one op = one (x) and one (+); SpGEMM ops =
products A_ik*B_kj, SpMM ops = nnz(T) * 64), aggregated over the step.

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
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1512_00066_amd", "csrc")
    for f in sorted(os.listdir(d)):
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
            best, times = ctx.autotune("plus_times", A, A, reps=2)
            sched[dt] = best
            log(f"autotune {dt}: best={best} times_ms={np.round(times, 2).tolist()}")
        del A32
    del A64

    def step():
        outs = []
        for coo in (coo64, coo32):
            A = ctx.fold("plus_times", coo, "ij", "i", "j")
            C = ctx.contract("plus_times", "ik", A, "kj", A, "ij", schedule=-1 if not sched else
                             sched["f64" if coo is coo64 else "f32"])
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
    dom = max(prof, key=lambda r: r[2])
    nm, cnt, tms, by = dom
    achieved = (by / cnt) / (tms / cnt / 1e3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        try:
            rec = json.load(open(tf))
            if rec.get("kernel") == nm and rec.get("source_hash") == kernel_source_hash():
                traffic = rec.get("hbm_bytes_per_launch")
        except Exception:
            traffic = None
    roof = {"bound": "hbm", "kernel": nm, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "avg_launch_ms": round(tms / cnt, 4), "algorithmic_bytes_per_launch": round(by / cnt)}
    out = {"metric": METRIC, "value": value, "unit": "semiring-ops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "rmat18_AxA_f64_f32+tensor512_fold_contraction", "rmat_scale": 18,
                      "edge_factor": 16, "abcd": [0.57, 0.19, 0.19, 0.05], "tensor_dims": [512, 512, 512],
                      "tensor_density": 1e-3, "dense_M": [512, 64], "products_per_AxA": products,
                      "schedules": sched},
           "roofline": roof}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline_rmat18(inp, wrow, args.cpu_seconds)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat18", choices=["rmat18"])
    ap.add_argument("--schedule", type=int, default=-1, help="force one SpGEMM schedule")
    ap.add_argument("--schedules", default="", help="SpGEMM schedules for fp64,fp32 (e.g. 0,5)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)
    out = run_rmat18(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
