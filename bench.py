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

Also reported (unless --only-plain): the batched stage sequence (8 uneven
block products summed into one C; per-block eager launches + sparse sum vs
the fused product captured as one graph), uniform and R-MAT variants, and
the backward pass at fixed sparsity; with --mcl, 10 Markov-clustering
iterations in one graph.
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
    runs, t_total = 0, 0.0
    total_products = int(oracle.rowub(Af, Bf).sum())
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


def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def _time_batched(args, pairs, m, bytes_in):
    """Per-block eager launches (symbolic with read-back + numeric per block,
    then the sparse sum) against the fused product captured as one graph."""
    import torch
    from paper_2603_21444_amd import binding
    from paper_2603_21444_amd.graph import StageGraph

    def eager():
        parts = [binding.spgemm(a, b) for a, b in pairs]
        return binding.merge(parts)

    for _ in range(max(1, args.warmup)):
        Ce = eager()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Ce = eager()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    nnz = Ce.nnz
    del Ce
    torch.cuda.empty_cache()
    g = StageGraph(pairs)
    for _ in range(max(1, args.warmup)):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    Cg = g.result()
    assert Cg.nnz == nnz, (Cg.nnz, nnz)
    plan = binding.Plan()
    plan.symbolic([a for a, _ in pairs], [b for _, b in pairs])
    _, products = plan.info()
    del g, Cg
    torch.cuda.empty_cache()
    alg = bytes_in + 4 * (m + 1) + 8 * nnz
    return {
        "products": int(products), "nnz_C": int(nnz),
        "graph_ms": round(graph_ms, 3), "eager_per_block_ms": round(eager_ms, 3),
        "graph_gflops": round(2 * products / graph_ms / 1e6, 2),
        "eager_gflops": round(2 * products / eager_ms / 1e6, 2),
        "graph_speedup": round(eager_ms / graph_ms, 3),
        "graph_alg_GBs": round(alg / graph_ms / 1e6, 1),
    }


def bench_batched(args):
    """8 uneven block products summed into one C (uniform variant)."""
    from paper_2603_21444_amd import binding, synth
    m, n, K = 1 << 18, 1 << 20, 8
    rng = synth.rng_for(SEED + 3, 11)
    kdims = rng.integers(1 << 18, (1 << 20) + 1, size=K)
    pairs = []
    for k in range(K):
        Ak = synth.varnnz_csr(m, int(kdims[k]), 4, 32, SEED + 3, np.float32, "normal", stream=2 * k)
        Bk = synth.varnnz_csr(int(kdims[k]), n, 4, 32, SEED + 3, np.float32, "normal", stream=2 * k + 1)
        pairs.append((binding.to_device(Ak), binding.to_device(Bk)))
    log("[bench] batched blocks generated")
    bytes_in = sum(csr_bytes(a.shape[0], a.nnz, 4) + csr_bytes(b.shape[0], b.nnz, 4) for a, b in pairs)
    r = _time_batched(args, pairs, m, bytes_in)
    r["workload"] = ("C = sum_k A_k B_k, 8 blocks, m = 2^18, n = 2^20, inner K_k ~ U[2^18, 2^20], "
                     "4..32 nnz/row, FP32 N(0,1)")
    return r


def bench_batched_rmat(args):
    """Power-law variant: A = R-MAT scale 20, edge factor 16, split into 8
    uneven inner blocks; B 2^20 x 2^20 with 4..32 uniform columns per row."""
    from paper_2603_21444_amd import binding, synth
    n = 1 << 20
    seed = SEED + 6
    A = synth.rmat_csr(20, 16, seed=seed, dtype=np.float32, values="normal", stream=0)
    Bm = synth.varnnz_csr(n, n, 4, 32, seed, np.float32, "normal", stream=1)
    bounds = synth.column_blocks(n, 8, n // 16, n // 4, seed)
    pairs = [(binding.to_device(a), binding.to_device(b)) for a, b in synth.split_inner(A, Bm, bounds)]
    log("[bench] R-MAT blocks generated")
    bytes_in = sum(csr_bytes(a.shape[0], a.nnz, 4) + csr_bytes(b.shape[0], b.nnz, 4) for a, b in pairs)
    r = _time_batched(args, pairs, n, bytes_in)
    r["workload"] = ("C = sum_k A_k B_k, A = R-MAT(0.57,0.19,0.19,0.05) scale 20 edge factor 16 split "
                     "into 8 uneven inner blocks, B 2^20 x 2^20 with 4..32 nnz/row, FP32 N(0,1)")
    return r


def bench_backward(args):
    """Backward at fixed sparsity: A, B 2^18 x 2^18, 16 nnz/row, FP32 N(0,1),
    loss <W, C> with W N(0,1) on S(C)."""
    import torch
    from paper_2603_21444_amd import binding, synth
    n, d = 1 << 18, 16
    A = synth.uniform_csr(n, n, d, SEED + 5, np.float32, "normal", stream=0)
    B = synth.uniform_csr(n, n, d, SEED + 5, np.float32, "normal", stream=1)
    dA_, dB_ = binding.to_device(A), binding.to_device(B)
    plan = binding.Plan()
    rp, nnz = plan.symbolic([dA_], [dB_])
    col, vals = plan.numeric([dA_], [dB_], rp, nnz)
    W = torch.from_numpy(synth.draw_values(synth.rng_for(SEED + 5, 9), nnz, "normal", np.float32)).cuda()
    dC = binding.DeviceCSR((n, n), rp, col, W)
    for _ in range(max(1, args.warmup)):
        plan.backward(dA_, dB_, dC)
    torch.cuda.synchronize()
    ev = _events(2)
    s = torch.cuda.current_stream()
    ev[0].record(s)
    for _ in range(args.steps):
        plan.backward(dA_, dB_, dC)
    ev[1].record(s)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / args.steps
    _, products = plan.info()
    alg = csr_bytes(n, A.nnz, 4) + csr_bytes(n, B.nnz, 4) + 4 * (n + 1) + 8 * nnz + 4 * (A.nnz + B.nnz)
    return {
        "workload": "dA = (W B^T) on S(A), dB = (A^T W) on S(B); A, B 2^18 x 2^18, 16 nnz/row, FP32",
        "products": int(products), "ms": round(ms, 4),
        "gflops": round(4 * products / ms / 1e6, 2),
        "alg_GBs": round(alg / ms / 1e6, 1), "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4),
    }


def bench_mcl(args):
    """10 Markov-clustering iterations on n = 2^19 (24 + 1 per column), FP32,
    recorded as one graph."""
    import torch
    from paper_2603_21444_amd import binding, synth
    from paper_2603_21444_amd.graph import MCLGraph
    n = 1 << 19
    X = synth.mcl_matrix(n, 24, SEED + 4, np.float32)
    g = MCLGraph(binding.to_device(X), iters=10)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    Y = g.result()
    return {"workload": "MCL, n = 2^19, 24 + 1 nnz per column, r = 2, prune < 1e-4, top-1000, "
                        "10 iterations in one graph",
            "ms_10_iterations": round(ms, 2), "final_nnz": Y.nnz}


def traffic_from_profile(kernel_src_hash):
    """HBM bytes per launch of the numeric kernel from the committed counter
    summary, if it was taken from the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "numeric_uniform2p20_fp32_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != kernel_src_hash:
        return None
    return int(fields["traffic_bytes"])


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_21444_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()


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
    ap.add_argument("--only-plain", action="store_true", help="skip the batched and backward workloads")
    ap.add_argument("--mcl", action="store_true", help="also time 10 MCL iterations (n = 2^19)")
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
            "kernel": "numeric pass (row-binned LDS kernels: bucket placement, hash, sort fallback; all bins of one step)",
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile(kernel_source_hash()),
            "algorithmic_bytes": num_bytes,
            "numeric_ms": round(r["num_ms"], 4),
        },
    }
    if not args.only_plain:
        log("[bench] batched stage sequence")
        out["batched_graph"] = bench_batched(args)
        torch.cuda.empty_cache()
        log("[bench] batched stage sequence, R-MAT")
        out["batched_graph_rmat"] = bench_batched_rmat(args)
        torch.cuda.empty_cache()
        log("[bench] backward")
        out["backward"] = bench_backward(args)
        torch.cuda.empty_cache()
    if args.mcl:
        log("[bench] MCL")
        out["mcl"] = bench_mcl(args)
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
