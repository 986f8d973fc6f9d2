"""Captured HIP graphs of whole stage sequences (no host synchronisation).

StageGraph  one GPU's rounds of the outer algorithm (§3.3.1, Alg. 1): the
            block products A_k B_k of all rounds summed into one C by the
            fused product (one accumulator per C row across all blocks, so
            the partial products are never written), recorded once and
            replayed.  Buffers are fixed (the analogue of the persistent
            tile buffers of §4.1-4.2); errors surface in the plan's device
            status word.
MCLGraph    `iters` Markov-clustering iterations (§5.7) on ping-pong
            buffers of capacity n * min(topk, n), recorded as one graph.

Capture uses torch.cuda.CUDAGraph on a side stream; every call recorded is
a capture-safe library call (capacity given, no read-back).  An eager run
first sizes the workspace, loads every kernel and fixes C's capacity.
"""
from __future__ import annotations

import torch

from . import binding


class StageGraph:
    def __init__(self, pairs, capacity: int | None = None, tuning=None):
        self.As = [a for a, _ in pairs]
        self.Bs = [b for _, b in pairs]
        self.plan = binding.Plan(tuning=tuning)
        m, n = self.As[0].shape[0], self.Bs[0].shape[1]
        dev = self.As[0].row_ptr.device
        dtype = self.As[0].vals.dtype
        rp, nnz = self.plan.symbolic(self.As, self.Bs)       # eager sizing run
        self.capacity = int(capacity if capacity is not None else max(nnz, 1))
        self.row_ptr = torch.empty(m + 1, dtype=torch.int32, device=dev)
        self.col = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.vals = torch.empty(self.capacity, dtype=dtype, device=dev)
        self.plan.numeric(self.As, self.Bs, rp, nnz)          # loads the numeric kernels
        torch.cuda.synchronize()
        self.shape = (m, n)
        self.graph = torch.cuda.CUDAGraph()
        self.stream = torch.cuda.Stream()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self.record(self.stream)

    def record(self, stream=None):
        """The recorded sequence (also callable eagerly, capture-safe).  It
        starts by clearing the status word, which the capture-safe calls
        keep raised once an error occurs."""
        self.plan.clear_status(stream)
        self.plan.symbolic(self.As, self.Bs, capacity=self.capacity, stream=stream,
                           rp=self.row_ptr)
        self.plan.numeric(self.As, self.Bs, self.row_ptr, self.capacity, col=self.col,
                          vals=self.vals, stream=stream)

    def replay(self):
        self.graph.replay()

    def result(self) -> binding.DeviceCSR:
        """C after a replay (synchronises; raises if the device status is set)."""
        torch.cuda.synchronize()
        st = self.plan.status()
        if st != binding.SPG_OK:
            raise binding.SpgError(st, "StageGraph")
        nnz = int(self.row_ptr[-1].item())
        return binding.DeviceCSR(self.shape, self.row_ptr, self.col[:nnz], self.vals[:nnz])


class MCLGraph:
    """`iters` MCL iterations on ping-pong buffers, recorded as one graph.
    `capacity` (entries per buffer) defaults to n * min(topk, n), which
    always suffices; a smaller one makes an iteration raise SPG_ERR_CAPACITY
    in the status word, and every later iteration of the replay then skips
    its work, so result() reports it."""

    def __init__(self, X: binding.DeviceCSR, iters: int = 10, r: int = 2,
                 prune: float = 1e-4, topk: int = 1000, tuning=None,
                 capacity: int | None = None, order: str = "workload"):
        n = X.shape[0]
        dev = X.row_ptr.device
        self.n, self.iters, self.r, self.prune, self.topk = n, iters, r, prune, topk
        self.order = order
        self.plan = binding.Plan(tuning=tuning)
        cap = n * min(topk, n) if capacity is None else int(capacity)
        self.capacity = cap
        self.bufs = []
        for _ in range(2):
            self.bufs.append((torch.empty(n + 1, dtype=torch.int32, device=dev),
                              torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                              torch.empty(max(cap, 1), dtype=torch.float32, device=dev)))
        self.X0 = X
        # warm-up outside the capture: workspace, kernels
        binding.mcl_iteration(X, r, prune, topk, plan=self.plan, out=self.bufs[1],
                              capacity=cap, capture=True, order=order)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        self.stream = torch.cuda.Stream()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self.record(self.stream)

    def _view(self, k):
        rp, col, vals = self.bufs[k]
        return binding.DeviceCSR((self.n, self.n), rp, col, vals)

    def record(self, stream=None):
        self.plan.clear_status(stream)
        src = self.X0
        for t in range(self.iters):
            dst = self.bufs[t % 2]
            binding.mcl_iteration(src, self.r, self.prune, self.topk, plan=self.plan, out=dst,
                                  stream=stream, capture=True, capacity=self.capacity,
                                  order=self.order)
            src = self._view(t % 2)

    def buffer(self, t: int) -> binding.DeviceCSR:
        """Output of iteration t (0-based) after a replay, valid while no
        later iteration has overwritten its ping-pong buffer (t >= iters - 2).
        Synchronises; raises if the device status is set."""
        if not (self.iters - 2 <= t < self.iters):
            raise ValueError("only the last two iterations' outputs are kept")
        torch.cuda.synchronize()
        st = self.plan.status()
        if st != binding.SPG_OK:
            raise binding.SpgError(st, "MCLGraph")
        rp, col, vals = self.bufs[t % 2]
        nnz = int(rp[-1].item())
        return binding.DeviceCSR((self.n, self.n), rp, col[:nnz], vals[:nnz])

    def replay(self):
        self.graph.replay()

    def result(self) -> binding.DeviceCSR:
        """Output of the last iteration (synchronises; raises if the device
        status is set)."""
        return self.buffer(self.iters - 1)
