"""ctypes binding of the C ABI in include/spgemm.h.

Argument marshalling only: torch provides device memory and the stream,
every step of the computation runs in the HIP kernels of libspgemm.so.
There is no CPU fallback: without the built library, or without a GPU,
these functions raise.

Low-level names mirror the C ABI (spgemm_symbolic, spgemm_numeric,
spgemm_merge, spgemm_backward, spgemm_mcl_iteration, ...).  On top sit
small helpers that allocate outputs with torch and run a whole pass:
`spgemm`, `batched`, `merge`, `Plan`.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SPG_LIB_PATH", os.path.join(HERE, "libspgemm.so"))

SPG_OK, SPG_ERR_INVALID, SPG_ERR_SHAPE, SPG_ERR_OVERFLOW = 0, 1, 2, 3
SPG_ERR_CAPACITY, SPG_ERR_WORKSPACE, SPG_ERR_HIP, SPG_ERR_UNSUPPORTED, SPG_ERR_ARG = 4, 5, 6, 7, 8
SPG_ERR_SCRATCH = 9
SPG_SCRATCH_BYTES = 128 << 20
SPG_F32, SPG_F64 = 0, 1
SPG_MCL_INFLATE_FIRST, SPG_MCL_PAPER = 0, 1
MCL_ORDERS = {"workload": SPG_MCL_INFLATE_FIRST, "paper": SPG_MCL_PAPER}
SPG_FLAG_VALIDATE = 1
SPG_MAX_PARTS = 16
SPG_NBINS = 16

# every symbol the header declares (checked by the CPU test suite)
EXPORTS = [
    "spgemm_plan_create", "spgemm_plan_destroy", "spgemm_workspace_size",
    "spgemm_plan_status", "spgemm_plan_clear_status", "spgemm_plan_info", "spgemm_status_string",
    "spgemm_symbolic", "spgemm_symbolic_noalloc", "spgemm_numeric", "spgemm_merge", "spgemm_backward",
    "spgemm_backward_deterministic", "spgemm_backward_deterministic_workspace_size",
    "spgemm_mcl_workspace_size", "spgemm_mcl_iteration", "spgemm_mcl_iteration_order",
    "spgemm_permute_workspace_size", "spgemm_permute",
    "spgemm_default_tuning", "spgemm_plan_set_tuning", "spgemm_plan_bins",
]


class SpgCsr(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("vals", C.c_void_p)]


class SpgTuning(C.Structure):
    _fields_ = [("lanes", C.c_int32 * SPG_NBINS), ("sub", C.c_int32 * SPG_NBINS),
                ("sym_sub", C.c_int32 * SPG_NBINS),
                ("heavy_slots", C.c_int32), ("max_window", C.c_int32),
                ("bin_edge", C.c_int32 * SPG_NBINS)]


class SpgError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} (status {code})")


_lib = None


def lib():
    """Load libspgemm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
        PC = C.POINTER(SpgCsr)
        sig = {
            "spgemm_plan_create": (C.c_int, [U32, C.POINTER(P)]),
            "spgemm_plan_destroy": (None, [P]),
            "spgemm_workspace_size": (C.c_int, [I32, I32, I32, C.POINTER(C.c_size_t)]),
            "spgemm_plan_status": (C.c_int, [P, C.POINTER(I32)]),
            "spgemm_plan_clear_status": (C.c_int, [P, P]),
            "spgemm_plan_info": (C.c_int, [P, C.POINTER(I64), C.POINTER(I64)]),
            "spgemm_status_string": (C.c_char_p, [C.c_int]),
            "spgemm_symbolic": (C.c_int, [P, I32, PC, PC, P, C.POINTER(I64), I64, P, C.c_size_t, P]),
            "spgemm_symbolic_noalloc": (C.c_int, [P, I32, PC, PC, P, I64, P]),
            "spgemm_numeric": (C.c_int, [P, I32, PC, PC, C.c_int, P, P, P]),
            "spgemm_merge": (C.c_int, [P, I32, PC, C.c_int, P, C.POINTER(I64), I64, P, P, P,
                                       C.c_size_t, P]),
            "spgemm_backward": (C.c_int, [P, PC, PC, PC, C.c_int, P, P, P]),
            "spgemm_backward_deterministic": (C.c_int, [P, PC, PC, PC, C.c_int, P, P, P, C.c_size_t, P]),
            "spgemm_backward_deterministic_workspace_size": (C.c_int, [C.c_int64, C.POINTER(C.c_size_t)]),
            "spgemm_mcl_workspace_size": (C.c_int, [I32, I32, C.POINTER(C.c_size_t)]),
            "spgemm_mcl_iteration": (C.c_int, [P, PC, I32, C.c_float, I32, P, P, P, I64,
                                               C.POINTER(I64), P, C.c_size_t, P]),
            "spgemm_permute_workspace_size": (C.c_int, [I32, I32, C.POINTER(C.c_size_t)]),
            "spgemm_permute": (C.c_int, [P, PC, P, P, C.c_int, P, P, P, P, C.c_size_t, P]),
            "spgemm_mcl_iteration_order": (C.c_int, [P, PC, I32, I32, C.c_float, I32, P, P, P,
                                                     I64, C.POINTER(I64), P, C.c_size_t, P]),
            "spgemm_default_tuning": (C.c_int, [C.POINTER(SpgTuning)]),
            "spgemm_plan_set_tuning": (C.c_int, [P, C.POINTER(SpgTuning)]),
            "spgemm_plan_bins": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(code: int) -> str:
    try:
        return lib().spgemm_status_string(code).decode()
    except Exception:  # library missing: still give a message
        return f"status {code}"


def _check(code: int, where: str):
    if code != SPG_OK:
        raise SpgError(code, where)


# ---------------------------------------------------------------- torch side
def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def dtype_code(dt) -> int:
    torch = _torch()
    if dt == torch.float32:
        return SPG_F32
    if dt == torch.float64:
        return SPG_F64
    raise ValueError(f"unsupported value dtype {dt}")


@dataclasses.dataclass
class DeviceCSR:
    """CSR on the GPU as torch tensors (int32 row_ptr/col_idx)."""
    shape: tuple
    row_ptr: object
    col_idx: object
    vals: object = None

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def spg(self) -> SpgCsr:
        return SpgCsr(self.shape[0], self.shape[1], self.nnz, self.row_ptr.data_ptr(),
                      self.col_idx.data_ptr() if self.nnz else None,
                      self.vals.data_ptr() if (self.vals is not None and self.nnz) else None)

    def to_host(self):
        from .synth import HostCSR
        return HostCSR(tuple(self.shape), self.row_ptr.cpu().numpy().astype(np.int64),
                       self.col_idx.cpu().numpy().astype(np.int32),
                       None if self.vals is None else self.vals.cpu().numpy())


def to_device(M, device="cuda", dtype=None) -> DeviceCSR:
    """Copy a host CSR (indptr/indices/data attributes) to the GPU."""
    torch = _torch()
    if M.shape[0] > 2**31 - 1 or M.nnz > 2**31 - 1:
        raise ValueError("CSR too large for int32 indices")
    rp = torch.from_numpy(np.ascontiguousarray(M.indptr, dtype=np.int32)).to(device)
    ci = torch.from_numpy(np.ascontiguousarray(M.indices, dtype=np.int32)).to(device)
    v = None
    if M.data is not None:
        d = np.ascontiguousarray(M.data if dtype is None else M.data.astype(dtype))
        v = torch.from_numpy(d).to(device)
    return DeviceCSR(tuple(M.shape), rp, ci, v)


def _arr(csrs):
    arr = (SpgCsr * len(csrs))()
    for k, M in enumerate(csrs):
        arr[k] = M.spg()
    return arr


def workspace_size(m: int, n: int, kmax: int) -> int:
    b = C.c_size_t(0)
    _check(lib().spgemm_workspace_size(m, n, kmax, C.byref(b)), "spgemm_workspace_size")
    return int(b.value)


def default_tuning() -> SpgTuning:
    t = SpgTuning()
    _check(lib().spgemm_default_tuning(C.byref(t)), "spgemm_default_tuning")
    return t


class Plan:
    """Owns an spg_plan and its workspace (a torch uint8 tensor)."""

    def __init__(self, validate: bool = False, tuning: SpgTuning | None = None):
        self.h = C.c_void_p()
        _check(lib().spgemm_plan_create(SPG_FLAG_VALIDATE if validate else 0, C.byref(self.h)),
               "spgemm_plan_create")
        self.ws = None
        if tuning is not None:
            self.set_tuning(tuning)

    def set_tuning(self, t: SpgTuning):
        _check(lib().spgemm_plan_set_tuning(self.h, C.byref(t)), "spgemm_plan_set_tuning")

    def __del__(self):
        try:
            if self.h:
                lib().spgemm_plan_destroy(self.h)
                self.h = C.c_void_p()
        except Exception:
            pass

    def workspace(self, m: int, n: int, kmax: int, device="cuda"):
        torch = _torch()
        need = workspace_size(m, n, kmax)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
        return self.ws

    def status(self) -> int:
        s = C.c_int32(0)
        _check(lib().spgemm_plan_status(self.h, C.byref(s)), "spgemm_plan_status")
        return int(s.value)

    def clear_status(self, stream=None):
        """Queue a clear of the device status word (capture-safe)."""
        _check(lib().spgemm_plan_clear_status(self.h, _stream(stream)), "spgemm_plan_clear_status")

    def bins(self):
        """(symbolic bin counts, numeric bin counts) after an eager symbolic call."""
        s = (C.c_int32 * SPG_NBINS)()
        n = (C.c_int32 * SPG_NBINS)()
        _check(lib().spgemm_plan_bins(self.h, s, n), "spgemm_plan_bins")
        return list(s), list(n)

    def info(self):
        nnz, prod = C.c_int64(0), C.c_int64(0)
        _check(lib().spgemm_plan_info(self.h, C.byref(nnz), C.byref(prod)), "spgemm_plan_info")
        return int(nnz.value), int(prod.value)

    # ---- product C = sum_k A_k B_k
    def symbolic(self, As, Bs, capacity: int | None = None, stream=None, rp=None):
        """Symbolic pass; eager (returns nnz) unless `capacity` is given, in
        which case nothing is read back and the call is graph-capturable."""
        torch = _torch()
        K = len(As)
        m, n = As[0].shape[0], Bs[0].shape[1]
        dev = As[0].row_ptr.device
        kmax = max(A.shape[1] for A in As)
        ws = self.workspace(m, n, kmax, dev)
        if rp is None:
            rp = torch.empty(m + 1, dtype=torch.int32, device=dev)
        nnz = C.c_int64(-1)
        eager = capacity is None
        _check(lib().spgemm_symbolic(self.h, K, _arr(As), _arr(Bs), _ptr(rp),
                                     C.byref(nnz) if eager else None,
                                     -1 if eager else int(capacity), _ptr(ws), ws.numel(),
                                     _stream(stream)), "spgemm_symbolic")
        return rp, (int(nnz.value) if eager else None)

    def symbolic_noalloc(self, As, Bs, rp, capacity: int, stream=None):
        """Symbolic pass in the library's static scratch (no workspace, no
        read-back; errors go to the device status word)."""
        _check(lib().spgemm_symbolic_noalloc(self.h, len(As), _arr(As), _arr(Bs), _ptr(rp),
                                             int(capacity), _stream(stream)),
               "spgemm_symbolic_noalloc")
        return rp

    def numeric(self, As, Bs, rp, nnz: int, dtype=None, col=None, vals=None, stream=None):
        torch = _torch()
        dev = rp.device
        dtype = dtype or As[0].vals.dtype
        if col is None:
            col = torch.empty(max(nnz, 0), dtype=torch.int32, device=dev)
        if vals is None:
            vals = torch.empty(max(nnz, 0), dtype=dtype, device=dev)
        _check(lib().spgemm_numeric(self.h, len(As), _arr(As), _arr(Bs), dtype_code(dtype),
                                    _ptr(col) if col.numel() else None,
                                    _ptr(vals) if vals.numel() else None, _stream(stream)),
               "spgemm_numeric")
        return col, vals

    # ---- sparse sum C = sum_k P_k
    def merge_count(self, Ps, capacity: int | None = None, stream=None):
        torch = _torch()
        m, n = Ps[0].shape
        dev = Ps[0].row_ptr.device
        ws = self.workspace(m, n, m, dev)
        rp = torch.empty(m + 1, dtype=torch.int32, device=dev)
        nnz = C.c_int64(-1)
        eager = capacity is None
        _check(lib().spgemm_merge(self.h, len(Ps), _arr(Ps), SPG_F32, _ptr(rp),
                                  C.byref(nnz) if eager else None,
                                  -1 if eager else int(capacity), None, None, _ptr(ws),
                                  ws.numel(), _stream(stream)), "spgemm_merge(count)")
        return rp, (int(nnz.value) if eager else None)

    def merge_fill(self, Ps, rp, nnz: int, dtype=None, col=None, vals=None, stream=None):
        torch = _torch()
        dev = rp.device
        dtype = dtype or Ps[0].vals.dtype
        if col is None:
            col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        if vals is None:
            vals = torch.empty(max(nnz, 1), dtype=dtype, device=dev)
        ws = self.ws
        _check(lib().spgemm_merge(self.h, len(Ps), _arr(Ps), dtype_code(dtype), _ptr(rp), None,
                                  -1, _ptr(col), _ptr(vals), _ptr(ws), ws.numel(),
                                  _stream(stream)), "spgemm_merge(fill)")
        return col[:nnz], vals[:nnz]

    # ---- backward at fixed sparsity
    def backward(self, A, B, dC, want_dA=True, want_dB=True, stream=None,
                 deterministic=False, det_workspace=None):
        """dA, dB of C = A B at fixed sparsity; deterministic=True gives dB
        the same bits on every run (fixed-point accumulation in a workspace
        of its own: det_workspace, or allocated here)."""
        torch = _torch()
        dtype = A.vals.dtype
        dA = torch.empty(A.nnz, dtype=dtype, device=A.vals.device) if want_dA else None
        dB = torch.empty(B.nnz, dtype=dtype, device=B.vals.device) if want_dB else None
        a, b, c = A.spg(), B.spg(), dC.spg()
        pa = _ptr(dA) if (dA is not None and dA.numel()) else None
        pb = _ptr(dB) if (dB is not None and dB.numel()) else None
        if not deterministic:
            _check(lib().spgemm_backward(self.h, C.byref(a), C.byref(b), C.byref(c),
                                         dtype_code(dtype), pa, pb, _stream(stream)),
                   "spgemm_backward")
            return dA, dB
        need = C.c_size_t(0)
        _check(lib().spgemm_backward_deterministic_workspace_size(B.nnz, C.byref(need)),
               "spgemm_backward_deterministic_workspace_size")
        ws = det_workspace
        if ws is None or ws.numel() < need.value:
            ws = torch.empty(need.value, dtype=torch.uint8, device=A.vals.device)
        _check(lib().spgemm_backward_deterministic(self.h, C.byref(a), C.byref(b), C.byref(c),
                                                   dtype_code(dtype), pa, pb, _ptr(ws),
                                                   ws.numel(), _stream(stream)),
               "spgemm_backward_deterministic")
        return dA, dB


def spgemm(A: DeviceCSR, B: DeviceCSR, plan: Plan | None = None, stream=None) -> DeviceCSR:
    """C = A B on the GPU (symbolic + numeric)."""
    return batched([(A, B)], plan, stream)


def batched(pairs, plan: Plan | None = None, stream=None) -> DeviceCSR:
    """C = sum_k A_k B_k in one fused pass."""
    plan = plan or Plan()
    As = [a for a, _ in pairs]
    Bs = [b for _, b in pairs]
    rp, nnz = plan.symbolic(As, Bs, stream=stream)
    col, vals = plan.numeric(As, Bs, rp, nnz, stream=stream)
    return DeviceCSR((As[0].shape[0], Bs[0].shape[1]), rp, col, vals)


def merge(parts, plan: Plan | None = None, stream=None) -> DeviceCSR:
    """C = sum_k P_k (union pattern, values added)."""
    plan = plan or Plan()
    rp, nnz = plan.merge_count(parts, stream=stream)
    col, vals = plan.merge_fill(parts, rp, nnz, stream=stream)
    return DeviceCSR(tuple(parts[0].shape), rp, col, vals)


def mcl_workspace_size(n: int, topk: int) -> int:
    b = C.c_size_t(0)
    _check(lib().spgemm_mcl_workspace_size(n, topk, C.byref(b)), "spgemm_mcl_workspace_size")
    return int(b.value)


def mcl_iteration(X: DeviceCSR, r: int = 2, prune: float = 1e-4, topk: int = 1000,
                  plan: Plan | None = None, out=None, stream=None,
                  capture: bool = False, capacity: int | None = None,
                  order: str = "workload") -> DeviceCSR:
    """One Markov-clustering iteration on X = M^T (FP32).  `out` may hold
    preallocated (row_ptr, col_idx, vals) of `capacity` entries (default
    n*min(topk, n), which always suffices).  With capture=True nothing is
    read back (graph-capturable); the result then spans the whole capacity
    and its length is row_ptr[n].  order: "workload" (inflate, normalise,
    prune, top-k, renormalise) or "paper" (normalise, prune, top-k, power)."""
    torch = _torch()
    plan = plan or Plan()
    n = X.shape[0]
    dev = X.row_ptr.device
    need = mcl_workspace_size(n, topk)
    if plan.ws is None or plan.ws.numel() < need:
        plan.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    cap = n * min(topk, n) if capacity is None else int(capacity)
    if out is None:
        out = (torch.empty(n + 1, dtype=torch.int32, device=dev),
               torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
               torch.empty(max(cap, 1), dtype=torch.float32, device=dev))
    rp, col, vals = out
    nnz = C.c_int64(-1)
    x = X.spg()
    _check(lib().spgemm_mcl_iteration_order(plan.h, C.byref(x), MCL_ORDERS[order], r,
                                            C.c_float(prune), topk, _ptr(rp), _ptr(col),
                                            _ptr(vals), cap, None if capture else C.byref(nnz),
                                            _ptr(plan.ws), plan.ws.numel(), _stream(stream)),
           "spgemm_mcl_iteration_order")
    if capture:
        return DeviceCSR((n, n), rp, col, vals)
    k = int(nnz.value)
    return DeviceCSR((n, n), rp, col[:k], vals[:k])


def permute_workspace_size(m: int, n: int) -> int:
    b = C.c_size_t(0)
    _check(lib().spgemm_permute_workspace_size(m, n, C.byref(b)), "spgemm_permute_workspace_size")
    return int(b.value)


def permute(A: DeviceCSR, row_perm=None, col_perm=None, plan: Plan | None = None,
            stream=None, out=None) -> DeviceCSR:
    """B[row_perm[i], col_perm[j]] = A[i, j] on the GPU (int32 device
    permutations or None for the identity; rows of B come out in ascending
    column order).  Errors (an array that is not a permutation) go to the
    plan's device status word."""
    torch = _torch()
    plan = plan or Plan()
    m, n = A.shape
    dev = A.row_ptr.device
    need = permute_workspace_size(m, n)
    if plan.ws is None or plan.ws.numel() < need:
        plan.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if out is None:
        out = (torch.empty(m + 1, dtype=torch.int32, device=dev),
               torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev),
               None if A.vals is None else torch.empty(max(A.nnz, 1), dtype=A.vals.dtype, device=dev))
    rp, col, vals = out
    a = A.spg()
    dt = dtype_code(A.vals.dtype) if A.vals is not None else SPG_F32
    _check(lib().spgemm_permute(plan.h, C.byref(a), _ptr(row_perm), _ptr(col_perm), dt, _ptr(rp),
                                _ptr(col), _ptr(vals), _ptr(plan.ws), plan.ws.numel(),
                                _stream(stream)), "spgemm_permute")
    return DeviceCSR((m, n), rp, col[:A.nnz], None if vals is None else vals[:A.nnz])
