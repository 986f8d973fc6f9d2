"""Autotuner for the row kernels' launch parameters and the bin thresholds.

For each bin that carries a noticeable share of the work it times the
symbolic + numeric passes (HIP events, eager, outside any graph capture)
over a few candidate (lanes per row, lanes per A entry) pairs, then over the
symbolic pass's own lanes per A entry, then over the bin's upper threshold
(a fraction of the products its LDS tables are sized for: the rows above
the threshold move to the next bin, whose tables are twice as large, so the
threshold is also the table load factor of those rows), and keeps the
fastest; the other bins keep their current setting.  Rows beyond every LDS
bin (heavy rows) get their lanes per A entry tuned the same way, in both
passes.  This is the architecture-specific tuning of LDS (shared memory)
use and team sizes the paper's local kernels rely on (§4.4).  Results are cached in a JSON file
keyed by dtype, shape, number of block products and the rounded per-bin row
histogram, so a capture reuses them without timing.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import binding

BIN_EDGES = [0] + [8 << b for b in range(1, 12)]
# candidate (lanes, sub) per bin size class
CANDIDATES = {
    1: [(8, 4), (8, 8), (16, 8), (1, 1)],
    2: [(8, 8), (16, 8), (16, 16)],
    3: [(16, 8), (16, 16), (32, 16)],
    4: [(32, 8), (32, 16), (64, 16)],
    5: [(64, 16), (64, 8), (32, 16), (64, 32)],
    6: [(64, 16), (64, 32), (128, 16)],
    7: [(64, 16), (128, 16), (256, 16)],
    8: [(128, 16), (256, 16), (256, 32)],
    9: [(512, 32), (512, 16), (256, 16)],
    10: [(512, 16), (1024, 16)],
    11: [(1024, 16)],
}
# candidate lanes per A entry of the symbolic count
SYM_SUB_CANDIDATES = (4, 8, 16, 32)
# rows beyond every LDS bin (split over many blocks, or one block each):
# their bin index and its candidate lanes per A entry, in both passes
HEAVY_BIN = 12
HEAVY_SUB_CANDIDATES = (16, 32, 64)
# candidate upper thresholds of a bin, as fractions of its table capacity
EDGE_FRACTIONS = (1.0, 0.75, 0.5)
# the last LDS bin of the product passes keeps its full edge
LAST_TUNED_EDGE_BIN = 10


def edge_for(b: int, frac: float) -> int:
    """Threshold of bin b at the given fraction of its capacity (0 = full)."""
    return 0 if frac >= 1.0 else max(1, int(BIN_EDGES[b] * frac))


def default_cache_path() -> str:
    base = os.environ.get("SPG_TUNING_CACHE", os.path.expanduser("~/.cache/paper_2603_21444_amd"))
    return os.path.join(base, "tuning.json")


def _key(As, Bs, dtype, counts) -> str:
    hist = [0 if c == 0 else int(round(math.log2(c))) for c in counts]
    return json.dumps([str(dtype), As[0].shape[0], Bs[0].shape[1], len(As), hist])


def _time(As, Bs, tuning, reps: int) -> float:
    plan = binding.Plan(tuning=tuning)
    rp, nnz = plan.symbolic(As, Bs)
    plan.numeric(As, Bs, rp, nnz)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        rp, nnz = plan.symbolic(As, Bs)
        plan.numeric(As, Bs, rp, nnz)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(As, Bs, reps: int = 3, cache_path: str | None = None, share: float = 0.05,
         use_cache: bool = True) -> binding.SpgTuning:
    """Tuning for the product sum_k A_k B_k (DeviceCSR lists)."""
    plan = binding.Plan()
    plan.symbolic(As, Bs)
    sym, num = plan.bins()
    counts = [max(a, b) for a, b in zip(sym, num)]
    dtype = As[0].vals.dtype if As[0].vals is not None else torch.float32
    key = _key(As, Bs, dtype, counts)
    path = cache_path or default_cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
        if key in cache:
            return _from_json(cache[key])
    t = binding.default_tuning()
    work = [counts[b] * BIN_EDGES[b] if 1 <= b <= 11 else 0 for b in range(len(counts))]
    total = sum(work) or 1
    for b in sorted(range(1, 12), key=lambda b: -work[b]):
        if work[b] < share * total:
            continue
        best, best_ms = None, float("inf")
        for lanes, sub in CANDIDATES[b]:
            t.lanes[b], t.sub[b] = lanes, sub
            ms = _time(As, Bs, t, reps)
            if ms < best_ms:
                best, best_ms = (lanes, sub), ms
        t.lanes[b], t.sub[b] = best
        best_s = t.sym_sub[b]
        for s in SYM_SUB_CANDIDATES:
            if s == best_s:
                continue
            t.sym_sub[b] = s
            ms = _time(As, Bs, t, reps)
            if ms < best_ms:
                best_s, best_ms = s, ms
        t.sym_sub[b] = best_s
        if b <= LAST_TUNED_EDGE_BIN:
            best_e = t.bin_edge[b]
            for f in EDGE_FRACTIONS:
                e = edge_for(b, f)
                if e == best_e:
                    continue
                t.bin_edge[b] = e
                ms = _time(As, Bs, t, reps)
                if ms < best_ms:
                    best_e, best_ms = e, ms
            t.bin_edge[b] = best_e
    # heavy rows (more products than the last LDS bin of a pass holds, at
    # least 4096 each): lanes per A entry of the numeric, then the symbolic pass
    if HEAVY_BIN < len(counts) and counts[HEAVY_BIN] * 4096 >= share * total:
        best_ms = _time(As, Bs, t, reps)
        for field in ("sub", "sym_sub"):
            arr = getattr(t, field)
            best = arr[HEAVY_BIN]
            for s in HEAVY_SUB_CANDIDATES:
                if s == best:
                    continue
                arr[HEAVY_BIN] = s
                ms = _time(As, Bs, t, reps)
                if ms < best_ms:
                    best, best_ms = s, ms
            arr[HEAVY_BIN] = best
    if use_cache:
        cache[key] = _to_json(t)
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return t


def _to_json(t: binding.SpgTuning) -> dict:
    return {"lanes": list(t.lanes), "sub": list(t.sub), "sym_sub": list(t.sym_sub),
            "bin_edge": list(t.bin_edge), "heavy_slots": t.heavy_slots,
            "max_window": t.max_window}


def _from_json(d: dict) -> binding.SpgTuning:
    t = binding.default_tuning()
    for b, v in enumerate(d["lanes"]):
        t.lanes[b] = v
    for b, v in enumerate(d["sub"]):
        t.sub[b] = v
    for b, v in enumerate(d.get("sym_sub", [])):
        t.sym_sub[b] = v
    for b, v in enumerate(d.get("bin_edge", [])):
        t.bin_edge[b] = v
    t.heavy_slots = d["heavy_slots"]
    t.max_window = d["max_window"]
    return t


def describe(t: binding.SpgTuning, bins=range(1, HEAVY_BIN + 1)) -> dict:
    """Compact record of a tuning for reports: per bin that differs from the
    default (the LDS bins and the heavy rows' bin), lanes per row, lanes per
    A entry (numeric, symbolic) and the bin's upper threshold (0 = its table
    capacity)."""
    d = binding.default_tuning()
    out = {}
    for b in bins:
        cur = (t.lanes[b], t.sub[b], t.sym_sub[b], t.bin_edge[b])
        if cur != (d.lanes[b], d.sub[b], d.sym_sub[b], d.bin_edge[b]):
            out[str(b)] = list(cur)
    return {"changed_bins": out, "heavy_slots": t.heavy_slots, "max_window": t.max_window}
