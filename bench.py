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
  cpu_baseline  the FP64 oracle on the host cores, same inputs (all
             threads on the whole product; one thread on a row sample)

Further legs, each with its own workload, all on by default (--legs picks
some):
  batched      8 uneven block products summed into one C: per-block eager
               launches + sparse sum, the fused product eagerly, and the
               fused product captured as one graph (autotuned)
  rmat         the same with a power-law (R-MAT scale 20) left operand
  backward     dA, dB at fixed sparsity
  mcl          10 Markov-clustering iterations (n = 2^19) in one graph, and
               the same iterations eagerly with per-iteration timing
  mcl_paper    the same in the paper's step order (prune 0.002, squaring)
  restriction  C = A R with an aggregation operator R (2^20 x 2^17)
  permute      random symmetric permutation of a banded matrix, and A^2 of
               the banded matrix against A^2 of the permuted one
"""
from __future__ import annotations

import argparse
import ctypes as C
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
LEGS = ["batched", "rmat", "backward", "mcl", "mcl_paper", "restriction", "permute"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def csr_bytes(nrows, nnz, vbytes):
    return 4 * (nrows + 1) + (4 + vbytes) * nnz


def make_inputs(n, d, seed):
    from paper_2603_21444_amd import synth
    A = synth.uniform_csr(n, n, d, seed, np.float32, "u01", stream=0)
    B = synth.uniform_csr(n, n, d, seed, np.float32, "u01", stream=1)
    return A, B


def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def _roof(alg_bytes, ms):
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    return round(gbs, 1), round(gbs / HBM_PEAK_GBS, 4)


def time_product(args, dA, dB, plan=None):
    """Symbolic + numeric per step (wall clock, eager read-back of nnz) and
    the numeric pass alone (HIP events on the stream it runs on)."""
    import torch
    from paper_2603_21444_amd import binding
    plan = plan or binding.Plan()
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
    _, products = plan.info()
    return dict(ms_step=ms_step, num_ms=num_ms, nnz=nnz, products=products)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, B, budget_s):
    """The oracle as it stands: all threads on the whole product (mean of up
    to 6 runs within the budget), one thread on the first 2^16 rows."""
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
    threads = oracle.num_threads()
    rows1 = min(1 << 16, A.shape[0])
    As = oracle_sample(Af, rows1)
    p1 = int(oracle.rowub(As, Bf).sum())
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.spgemm(As, Bf)
        sec1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    return dict(value=round(2.0 * total_products / sec / 1e9, 3), unit="GFLOP/s",
                cores=threads, kind="oracle",
                sample=f"full C = A B (2^20 rows, {total_products} products), {threads} threads, "
                       f"mean of {runs} run(s), {sec:.2f} s each; one thread: first {rows1} rows "
                       f"({p1} products) in {sec1:.2f} s",
                single_thread_value=round(2.0 * p1 / sec1 / 1e9, 4),
                cpu_model=cpu_model(), host_cpus=os.cpu_count())


def oracle_sample(M, rows):
    from paper_2603_21444_amd.synth import HostCSR
    e = int(M.indptr[rows])
    return HostCSR((rows, M.shape[1]), M.indptr[:rows + 1], M.indices[:e], M.data[:e])


def _wall(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps, out


def _time_batched(args, pairs, m, bytes_in):
    """Three forms of the same sum of block products on the same GPU:
      per-block eager: per block an eager product (symbolic with nnz read-
        back, numeric) on its own reused plan and workspace, then the sparse
        sum of the partials on a reused plan;
      fused eager: the fused product's capture-safe calls issued eagerly;
      graph: the same calls captured once and replayed.
    The graph uses the autotuner's tuning for this input."""
    import torch
    from paper_2603_21444_amd import autotune, binding
    from paper_2603_21444_amd.graph import StageGraph

    As = [a for a, _ in pairs]
    Bs = [b for _, b in pairs]
    if args.graph_only:
        # the graph alone (for kernel profiles): tuning from the autotuner's
        # cache when an earlier run of the same workload filled it
        tuning = autotune.tune(As, Bs, use_cache=True)
        g = StageGraph(pairs, tuning=tuning)
        for _ in range(max(1, args.warmup)):
            g.replay()
        graph_ms, _ = _wall(g.replay, args.steps)
        Cg = g.result()
        return {"graph_ms": round(graph_ms, 3), "nnz_C": int(Cg.nnz),
                "tuning": autotune.describe(tuning)}
    plans = [binding.Plan() for _ in pairs]
    mplan = binding.Plan()

    def per_block():
        parts = [binding.spgemm(a, b, plan=p) for (a, b), p in zip(pairs, plans)]
        return binding.merge(parts, plan=mplan)

    for _ in range(max(1, args.warmup)):
        Ce = per_block()
    nnz = Ce.nnz
    del Ce
    per_block_ms, Ce = _wall(per_block, args.steps)
    del Ce
    del plans, mplan
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    tuning = autotune.tune(As, Bs, use_cache=args.tuning_cache)
    tune_s = time.perf_counter() - t0
    g = StageGraph(pairs, tuning=tuning)
    stream = torch.cuda.current_stream()
    for _ in range(max(1, args.warmup)):
        g.record(stream)
    fused_ms, _ = _wall(lambda: g.record(stream), args.steps)
    for _ in range(max(1, args.warmup)):
        g.replay()
    graph_ms, _ = _wall(g.replay, args.steps)
    Cg = g.result()
    assert Cg.nnz == nnz, (Cg.nnz, nnz)
    _, products = g.plan.info()
    if products < 0:
        plan = binding.Plan()
        plan.symbolic(As, Bs)
        _, products = plan.info()
    del g, Cg
    torch.cuda.empty_cache()
    alg = bytes_in + 4 * (m + 1) + 8 * nnz
    gbs, frac = _roof(alg, graph_ms)
    return {
        "products": int(products), "nnz_C": int(nnz),
        "graph_ms": round(graph_ms, 3), "eager_fused_ms": round(fused_ms, 3),
        "eager_per_block_ms": round(per_block_ms, 3),
        "graph_gflops": round(2 * products / graph_ms / 1e6, 2),
        "eager_fused_gflops": round(2 * products / fused_ms / 1e6, 2),
        "eager_gflops": round(2 * products / per_block_ms / 1e6, 2),
        "graph_speedup": round(per_block_ms / graph_ms, 3),
        "fusion_speedup": round(per_block_ms / fused_ms, 3),
        "capture_speedup": round(fused_ms / graph_ms, 3),
        "graph_alg_GBs": gbs, "graph_hbm_frac": frac, "algorithmic_bytes": int(alg),
        "tuning": autotune.describe(tuning), "tune_s": round(tune_s, 2),
    }


def bench_batched(args):
    """8 uneven block products summed into one C (uniform variant)."""
    from paper_2603_21444_amd import binding, synth
    m = 1 << 18
    pairs = [(binding.to_device(a), binding.to_device(b))
             for a, b in synth.batched_uniform_blocks(SEED + 3)]
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
    _, _, hpairs = synth.batched_rmat_blocks(SEED + 6)
    pairs = [(binding.to_device(a), binding.to_device(b)) for a, b in hpairs]
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
    need = C.c_size_t(0)
    binding.lib().spgemm_backward_deterministic_workspace_size(B.nnz, C.byref(need))
    det_ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")

    def timed(det):
        for _ in range(max(1, args.warmup)):
            plan.backward(dA_, dB_, dC, deterministic=det, det_workspace=det_ws)
        torch.cuda.synchronize()
        ev = _events(2)
        s = torch.cuda.current_stream()
        ev[0].record(s)
        for _ in range(args.steps):
            plan.backward(dA_, dB_, dC, deterministic=det, det_workspace=det_ws)
        ev[1].record(s)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / args.steps

    ms = timed(False)
    det_ms = timed(True)
    _, products = plan.info()
    alg = csr_bytes(n, A.nnz, 4) + csr_bytes(n, B.nnz, 4) + 4 * (n + 1) + 8 * nnz + 4 * (A.nnz + B.nnz)
    gbs, frac = _roof(alg, ms)
    return {
        "workload": "dA = (W B^T) on S(A), dB = (A^T W) on S(B); A, B 2^18 x 2^18, 16 nnz/row, FP32",
        "products": int(products), "ms": round(ms, 4),
        "deterministic_dB_ms": round(det_ms, 4),
        "gflops": round(4 * products / ms / 1e6, 2),
        "alg_GBs": gbs, "hbm_frac": frac, "algorithmic_bytes": int(alg),
    }


def bench_mcl(args, order="workload"):
    """10 Markov-clustering iterations on n = 2^19 (24 + 1 per column), FP32:
    eagerly, one at a time with HIP events around each (products from the
    plan), then recorded as one graph and replayed."""
    import torch
    from paper_2603_21444_amd import binding, synth
    from paper_2603_21444_amd.graph import MCLGraph
    n = 1 << 19
    if order == "workload":
        r, prune, topk = 2, 1e-4, 1000
    else:
        r, prune, topk = 2, 0.002, 500
    X = synth.mcl_matrix(n, 24, SEED + 4, np.float32)
    dX = binding.to_device(X)
    plan = binding.Plan()
    s = torch.cuda.current_stream()
    Y = binding.mcl_iteration(dX, r, prune, topk, plan=plan, order=order)  # warm-up
    del Y
    torch.cuda.synchronize()
    per_it = []
    Y = dX
    for t in range(10):
        nnz_in = Y.nnz
        e0, e1 = _events(2)
        e0.record(s)
        Y = binding.mcl_iteration(Y, r, prune, topk, plan=plan, order=order)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        _, products = plan.info()
        alg = csr_bytes(n, nnz_in, 4) + csr_bytes(n, Y.nnz, 4)
        per_it.append({"ms": round(ms, 2), "products": int(products), "nnz_out": int(Y.nnz),
                       "gflops": round(2 * products / ms / 1e6, 1),
                       "alg_GBs": round(alg / ms / 1e6, 1)})
    eager_ms = sum(p["ms"] for p in per_it)
    total_products = sum(p["products"] for p in per_it)
    del Y
    torch.cuda.empty_cache()
    g = MCLGraph(dX, iters=10, r=r, prune=prune, topk=topk, order=order)
    g.replay()
    torch.cuda.synchronize()
    reps = 1
    graph_ms, _ = _wall(g.replay, reps)
    Yg = g.result()
    out = {"workload": (f"MCL ({'inflate r=2, renormalise, prune < 1e-4, top-1000' if order == 'workload' else 'paper order: normalise, prune < 0.002, square'}), "
                        "n = 2^19, 24 + 1 nnz per column, FP32, 10 iterations in one graph"),
           "ms_10_iterations_graph": round(graph_ms, 2), "ms_10_iterations_eager": round(eager_ms, 2),
           "products_10_iterations": int(total_products),
           "graph_gflops": round(2 * total_products / graph_ms / 1e6, 1),
           "final_nnz": Yg.nnz, "per_iteration_eager": per_it}
    del g, Yg
    torch.cuda.empty_cache()
    return out


def bench_restriction(args, A):
    """C = A R: A the plain workload's left operand (2^20 x 2^20, 16 per
    row), R an aggregation operator 2^20 x 2^17 (one entry per row, FP32 in
    (0,1]): 16 products per row, the low-flop regime."""
    from paper_2603_21444_amd import binding, synth
    n, nc = A.shape[0], A.shape[0] >> 3
    R = synth.aggregation_csr(n, nc, SEED + 7, np.float32, "u01")
    dA, dR = binding.to_device(A), binding.to_device(R)
    r = time_product(args, dA, dR)
    alg = csr_bytes(n, A.nnz, 4) + csr_bytes(n, R.nnz, 4) + 4 * (n + 1) + 8 * r["nnz"]
    gbs, frac = _roof(alg, r["num_ms"])
    return {"workload": "C = A R, A 2^20 x 2^20 uniform 16/row FP32 (0,1], R 2^20 x 2^17 aggregation "
                        "(one entry per row, aggregates of 8 points, FP32 (0,1])",
            "products": int(r["products"]), "nnz_C": int(r["nnz"]),
            "ms_step": round(r["ms_step"], 4), "numeric_ms": round(r["num_ms"], 4),
            "gflops": round(2 * r["products"] / r["ms_step"] / 1e6, 2),
            "numeric_alg_GBs": gbs, "numeric_hbm_frac": frac, "algorithmic_bytes": int(alg)}


def bench_permute(args):
    """Random symmetric permutation of a banded 2^20 x 2^20 matrix (16 per
    row on three diagonal bands), timed on the device, and C = A A on the
    banded matrix against C = A A on the permuted one."""
    import torch
    from paper_2603_21444_amd import binding, synth
    n = 1 << 20
    A = synth.banded_csr(n, 16, [0, n // 8, -n // 8], 256, SEED + 8, np.float32)
    p = torch.from_numpy(synth.random_permutation(n, SEED + 8)).cuda()
    dA = binding.to_device(A)
    plan = binding.Plan()
    out = (torch.empty(n + 1, dtype=torch.int32, device="cuda"),
           torch.empty(A.nnz, dtype=torch.int32, device="cuda"),
           torch.empty(A.nnz, dtype=torch.float32, device="cuda"))
    for _ in range(max(1, args.warmup)):
        PA = binding.permute(dA, p, p, plan=plan, out=out)
    perm_ms, PA = _wall(lambda: binding.permute(dA, p, p, plan=plan, out=out), args.steps)
    assert plan.status() == binding.SPG_OK
    perm_alg = 2 * csr_bytes(n, A.nnz, 4) + 4 * n
    band = time_product(args, dA, dA)
    perm = time_product(args, PA, PA)
    gbs, frac = _roof(perm_alg, perm_ms)
    return {"workload": "banded A 2^20 x 2^20, 16 per row on bands at offsets 0, +-2^17 "
                        "(half-width 256), FP32; B = P A P^T with a random P",
            "permute_ms": round(perm_ms, 4), "permute_alg_GBs": gbs, "permute_hbm_frac": frac,
            "banded_AA_ms": round(band["ms_step"], 4), "permuted_AA_ms": round(perm["ms_step"], 4),
            "banded_AA_gflops": round(2 * band["products"] / band["ms_step"] / 1e6, 2),
            "permuted_AA_gflops": round(2 * perm["products"] / perm["ms_step"] / 1e6, 2),
            "products": int(band["products"]), "nnz_AA": int(band["nnz"])}


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


# Sources the plain product's numeric pass is built and launched from (its
# kernels, their headers, the binning that routes its rows, the launchers);
# the backward, MCL, permutation, split-row and one-thread-per-row sources
# take no part in it.
NUMERIC_SOURCES = ("api.hip", "binning.hip", "row_kernels.hip", "wave_kernels.hip",
                   "rowops.hpp", "common.hpp", "internal.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_21444_amd", "csrc")
    for name in NUMERIC_SOURCES:
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
    ap.add_argument("--legs", default=",".join(LEGS),
                    help=f"comma-separated further legs ({','.join(LEGS)}), or 'none'")
    ap.add_argument("--only-plain", action="store_true", help="same as --legs none")
    ap.add_argument("--skip-plain", action="store_true",
                    help="run only the chosen legs (the headline fields are then absent)")
    ap.add_argument("--graph-only", action="store_true",
                    help="batched legs: time only the graph replays (kernel profiles)")
    ap.add_argument("--tuning-cache", action="store_true",
                    help="batched legs: store the autotuner's choice in its cache (for --graph-only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by rows of A and C; see the design notes)", file=sys.stderr)
        sys.exit(2)
    legs = [] if (args.only_plain or args.legs == "none") else [x for x in args.legs.split(",") if x]
    for leg in legs:
        if leg not in LEGS:
            ap.error(f"unknown leg {leg!r}")
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = 1 << args.log2n
    d = args.nnz_per_row
    log(f"[bench] generating A, B: {n} x {n}, {d} per row")
    A, B = make_inputs(n, d, SEED + 1)
    out = {"metric": METRIC}
    if not args.skip_plain:
        log("[bench] plain product")
        from paper_2603_21444_amd import binding
        r = time_product(args, binding.to_device(A), binding.to_device(B))
        torch.cuda.empty_cache()
        products = r["products"]
        gflops = 2.0 * products / (r["ms_step"] * 1e-3) / 1e9
        num_bytes = csr_bytes(n, A.nnz, 4) + csr_bytes(n, B.nnz, 4) + 4 * (n + 1) + 8 * r["nnz"]
        achieved = num_bytes / (r["num_ms"] * 1e-3) / 1e9
        out.update({
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
        })
    runners = {
        "batched": lambda: bench_batched(args),
        "rmat": lambda: bench_batched_rmat(args),
        "backward": lambda: bench_backward(args),
        "mcl": lambda: bench_mcl(args, "workload"),
        "mcl_paper": lambda: bench_mcl(args, "paper"),
        "restriction": lambda: bench_restriction(args, A),
        "permute": lambda: bench_permute(args),
    }
    names = {"batched": "batched_graph", "rmat": "batched_graph_rmat", "mcl": "mcl",
             "mcl_paper": "mcl_paper_order", "backward": "backward", "restriction": "restriction",
             "permute": "permute"}
    for leg in legs:
        log(f"[bench] {leg}")
        out[names[leg]] = runners[leg]()
        torch.cuda.empty_cache()
    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
    if args.cpu_budget > 0 and not args.skip_plain:
        log("[bench] oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(A, B, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
