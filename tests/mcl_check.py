"""Stepwise parity check of one GPU Markov-clustering iteration against the
FP64 oracle on the same input (the GPU's own previous output).

Pattern decisions whose oracle value lies within relative 1e-4 of the prune
threshold or of the top-k cut may go either way (FP32 path vs FP64 oracle);
every other decision must match.  Kept values agree to relative 1e-4 with the
oracle's, and on rows whose kept set differs (a decision inside the band),
with the oracle's values over the GPU's kept set: renormalised over that set
for the workload order, the element-wise power alone for the paper's order.
"""
from __future__ import annotations

import numpy as np

import oracle
from helpers import row_ids, row_subset


def check_mcl_step(X, got, r, prune, topk, rows=None, order="workload", rtol=1e-4):
    """Compare rows `rows` (default: all) of the GPU output `got` with the
    oracle run on X.  Returns the number of pattern decisions that fell
    inside the band."""
    n = X.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    Xf = X if X.data.dtype == np.float64 else X.with_data(X.data.astype(np.float64))
    cnt, ocol, oval = oracle.mcl_rows(Xf, rows, r, prune, topk, order=order, flat=True)
    g = row_subset(got, rows)
    glen = np.diff(g.indptr)
    # canonical rows
    rid = row_ids(g)
    if g.indices.size:
        same = rid[1:] == rid[:-1]
        assert np.all(g.indices[1:][same] > g.indices[:-1][same]), "output rows not canonical"
    # rows of equal length: compare columns entry by entry
    eq = glen == cnt.astype(np.int64)
    ridr = np.repeat(np.arange(rows.size), cnt)
    gsel, rsel = eq[rid], eq[ridr]
    diffcol = g.indices[gsel] != ocol[rsel]
    bad_rows = np.unique(rid[gsel][diffcol])
    eq[bad_rows] = False
    gsel, rsel = eq[rid], eq[ridr]
    gv = np.asarray(g.data[gsel], dtype=np.float64)
    ov = oval[rsel]
    err = np.abs(gv - ov) > rtol * np.abs(ov)
    assert not err.any(), (f"{int(err.sum())} kept values off by more than {rtol} relative "
                           f"(rows {np.unique(rid[gsel][err])[:8].tolist()})")
    flip_rows = np.nonzero(~eq)[0]
    ocp = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(cnt, out=ocp[1:])
    nflip = 0
    rp = 1 if order == "paper" else r  # the band is on the normalised values before the power
    for c0 in range(0, flip_rows.size, 16):
        chunk = flip_rows[c0:c0 + 16]
        _, allc, allv = oracle.mcl_rows(Xf, rows[chunk], rp, 0.0, 10 ** 9, order=order)
        for t, slot in enumerate(chunk):
            i = int(rows[slot])
            s, e = int(g.indptr[slot]), int(g.indptr[slot + 1])
            gc = g.indices[s:e]
            gvr = np.asarray(g.data[s:e], dtype=np.float64)
            oc = ocol[ocp[slot]:ocp[slot + 1]]
            pre = dict(zip(allc[t].tolist(), allv[t].tolist()))
            ranked = np.sort(allv[t])[::-1]
            kth = ranked[min(topk, ranked.size) - 1] if ranked.size else 0.0
            for j in set(gc.tolist()) ^ set(oc.tolist()):
                v = pre[j]
                near_prune = abs(v - prune) <= 1e-4 * prune
                near_kth = abs(v - kth) <= 1e-4 * kth
                assert near_prune or near_kth, f"row {i} col {j}: value {v} outside the band"
                nflip += 1
            kept = np.array([pre[j] for j in gc.tolist()])
            want = kept / kept.sum() if order == "workload" else kept ** r
            assert np.allclose(gvr, want, rtol=rtol, atol=0), f"row {i}: values over the GPU's kept set"
    return nflip
