"""MI355X (gfx950) local SpGEMM hot path: C = A B in CSR, the sparse sum of
partial products, batched stage graphs, MCL iterations and the backward pass
at fixed sparsity, all in hand-written HIP kernels behind a C ABI.

The compiled library is loaded lazily by `paper_2603_21444_amd.binding`;
importing this package does not touch the GPU.
"""
__all__ = ["synth", "binding"]
