"""Python binding of libbgcr.so, the MI355X block GCRO-DR library.

Argument marshalling only: every step of the solve runs in the HIP library.
The functions carry the names of the C ABI in include/bgcr.h; `DeviceCSR` and
`Sequence` are thin conveniences over them.  PyTorch provides device memory
and streams.  Importing works without a GPU; calling into the library without
the built .so raises at once (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "BGCR_OK", "BGCR_NOT_CONVERGED", "BGCR_BREAKDOWN_DEFLATED", "BGCR_ERR_INVALID", "BGCR_ERR_NOMEM", "BGCR_ERR_HIP",
    "BGCR_ERR_NONFINITE", "BGCR_ERR_NUMERICAL", "BGCR_F64", "BGCR_C128", "BGCR_PLAIN_FP64",
    "BGCR_MIXED_FP32", "BGCR_MIXED_FP32_BF16", "BGCR_PRECOND_NONE", "BGCR_PRECOND_ILU0", "BgcrError", "bgcr_params", "bgcr_csr", "bgcr_stats", "lib", "LIB_PATH",
    "bgcr_create_sequence", "bgcr_solve", "bgcr_release", "bgcr_footprint_bytes", "bgcr_recycle_dim",
    "bgcr_get_recycle", "bgcr_set_recycle", "bgcr_get_cycle_log", "bgcr_spmm", "bgcr_strerror",
    "bgcr_set_profiling", "bgcr_get_profile", "bgcr_apply_projected", "bgcr_apply_projected_work_bytes",
    "bgcr_apply_projected_noalloc", "bgcr_stream_probe", "BGCR_NOALLOC_SCRATCH_BYTES", "KERNEL_CLASSES",
    "DeviceCSR", "Sequence", "EXPORTED_SYMBOLS",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbgcr.so")

BGCR_OK = 0
BGCR_NOT_CONVERGED = 1
BGCR_BREAKDOWN_DEFLATED = 2
BGCR_ERR_INVALID = -1
BGCR_ERR_NOMEM = -2
BGCR_ERR_HIP = -3
BGCR_ERR_NONFINITE = -4
BGCR_ERR_NUMERICAL = -5
BGCR_F64 = 0
BGCR_C128 = 1
BGCR_PLAIN_FP64 = 0
BGCR_MIXED_FP32 = 1
BGCR_MIXED_FP32_BF16 = 2
BGCR_PRECOND_NONE = 0
BGCR_PRECOND_ILU0 = 1

EXPORTED_SYMBOLS = [
    "bgcr_create_sequence", "bgcr_solve", "bgcr_release", "bgcr_footprint_bytes", "bgcr_recycle_dim",
    "bgcr_get_recycle", "bgcr_set_recycle", "bgcr_get_cycle_log", "bgcr_spmm", "bgcr_set_profiling",
    "bgcr_get_profile", "bgcr_strerror", "bgcr_apply_projected", "bgcr_apply_projected_work_bytes",
    "bgcr_apply_projected_noalloc", "bgcr_stream_probe",
]

# bytes of the library's own workspace of bgcr_apply_projected_noalloc (bgcr.h)
BGCR_NOALLOC_SCRATCH_BYTES = 20 << 20

# kernel classes of the per-kernel profile (bgcr_kernel_class)
KERNEL_CLASSES = ["arn_spmm", "arn_dot", "proj_dot", "proj_gram", "small", "combine", "residual", "tsdot", "spmm",
                  "host", "host_eig", "precond", "ilu", "arn_spmm_dot"]


class bgcr_params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
                ("select_largest", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("enlarge_cycles", ctypes.c_int32), ("ritz_vectors", ctypes.c_int32), ("precond", ctypes.c_int32)]


class bgcr_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p)]


class bgcr_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cycles", ctypes.c_int32), ("block_steps", ctypes.c_int32),
                ("spmm_calls", ctypes.c_int32), ("rel_res", ctypes.c_double), ("rel_res_max_col", ctypes.c_double),
                ("seconds", ctypes.c_double), ("alg_bytes", ctypes.c_double), ("k_eff", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("deflations", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BgcrError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: status {code} ({bgcr_strerror(code)})")


_lib = None


def lib():
    """Load libbgcr.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1604_01713_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        c = ctypes
        L.bgcr_create_sequence.argtypes = [c.POINTER(bgcr_params), c.c_int64, c.c_void_p, c.POINTER(c.c_void_p)]
        L.bgcr_solve.argtypes = [c.c_void_p, c.POINTER(bgcr_csr), c.c_void_p, c.c_int64, c.c_void_p, c.c_int64,
                                 c.c_double, c.POINTER(bgcr_stats)]
        L.bgcr_release.argtypes = [c.c_void_p]
        L.bgcr_footprint_bytes.argtypes = [c.POINTER(bgcr_params), c.c_int64, c.c_int64]
        L.bgcr_footprint_bytes.restype = c.c_size_t
        L.bgcr_recycle_dim.argtypes = [c.c_void_p, c.POINTER(c.c_int32)]
        L.bgcr_get_recycle.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p, c.c_int64]
        L.bgcr_set_recycle.argtypes = [c.c_void_p, c.c_void_p, c.c_int64, c.c_int32]
        L.bgcr_get_cycle_log.argtypes = [c.c_void_p, c.POINTER(c.c_int32), c.POINTER(c.c_double), c.c_int32,
                                         c.POINTER(c.c_int32)]
        L.bgcr_spmm.argtypes = [c.POINTER(bgcr_csr), c.c_int32, c.c_int32, c.c_void_p, c.c_void_p, c.c_void_p]
        L.bgcr_apply_projected.argtypes = [c.POINTER(bgcr_csr), c.c_int32, c.c_int32, c.c_void_p, c.c_void_p,
                                           c.c_void_p, c.c_int32, c.c_void_p, c.c_size_t, c.c_void_p]
        L.bgcr_apply_projected_noalloc.argtypes = [c.POINTER(bgcr_csr), c.c_int32, c.c_int32, c.c_void_p,
                                                   c.c_void_p, c.c_void_p, c.c_int32, c.c_void_p]
        L.bgcr_apply_projected_work_bytes.argtypes = [c.c_int64, c.c_int32, c.c_int32]
        L.bgcr_apply_projected_work_bytes.restype = c.c_size_t
        L.bgcr_set_profiling.argtypes = [c.c_void_p, c.c_int]
        L.bgcr_get_profile.argtypes = [c.c_void_p, c.POINTER(c.c_double), c.POINTER(c.c_double),
                                       c.POINTER(c.c_int64), c.c_int32]
        L.bgcr_stream_probe.argtypes = [c.POINTER(c.c_void_p), c.c_int32, c.POINTER(c.c_void_p), c.c_int32,
                                        c.c_int64, c.c_int32, c.c_void_p]
        L.bgcr_strerror.argtypes = [c.c_int]
        L.bgcr_strerror.restype = c.c_char_p
        for name in ["bgcr_create_sequence", "bgcr_solve", "bgcr_release", "bgcr_recycle_dim", "bgcr_get_recycle",
                     "bgcr_set_recycle", "bgcr_get_cycle_log", "bgcr_spmm", "bgcr_set_profiling",
                     "bgcr_get_profile", "bgcr_apply_projected", "bgcr_apply_projected_noalloc",
                     "bgcr_stream_probe"]:
            getattr(L, name).restype = c.c_int
        _lib = L
    return _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _check(code, what):
    if code < 0:
        raise BgcrError(code, what)
    return code


def bgcr_strerror(code):
    return lib().bgcr_strerror(int(code)).decode()


def bgcr_create_sequence(params: bgcr_params, n: int, stream=None):
    h = ctypes.c_void_p()
    _check(lib().bgcr_create_sequence(ctypes.byref(params), int(n), _stream_handle(stream), ctypes.byref(h)),
           "bgcr_create_sequence")
    return h


def bgcr_solve(seq, A: "DeviceCSR", B, X, tol: float):
    """X (in: X0, out: solution) and B are device tensors n x p (row-major, any ld)."""
    st = bgcr_stats()
    code = lib().bgcr_solve(seq, ctypes.byref(A.csr), _ptr(B), int(B.stride(0)), _ptr(X), int(X.stride(0)),
                            float(tol), ctypes.byref(st))
    _check(code, "bgcr_solve")
    return st


def bgcr_release(seq):
    return lib().bgcr_release(seq)


def bgcr_footprint_bytes(params: bgcr_params, n: int, nnz: int) -> int:
    return int(lib().bgcr_footprint_bytes(ctypes.byref(params), int(n), int(nnz)))


def bgcr_recycle_dim(seq) -> int:
    k = ctypes.c_int32()
    _check(lib().bgcr_recycle_dim(seq, ctypes.byref(k)), "bgcr_recycle_dim")
    return int(k.value)


def bgcr_get_recycle(seq, U_out=None, C_out=None):
    ld = (U_out if U_out is not None else C_out).stride(0)
    _check(lib().bgcr_get_recycle(seq, _ptr(U_out), _ptr(C_out), int(ld)), "bgcr_get_recycle")


def bgcr_set_recycle(seq, U):
    _check(lib().bgcr_set_recycle(seq, _ptr(U), int(U.stride(0)), int(U.shape[1])), "bgcr_set_recycle")


def bgcr_get_cycle_log(seq, cap=100000):
    steps = (ctypes.c_int32 * cap)()
    res = (ctypes.c_double * cap)()
    cnt = ctypes.c_int32()
    _check(lib().bgcr_get_cycle_log(seq, steps, res, cap, ctypes.byref(cnt)), "bgcr_get_cycle_log")
    c = min(cnt.value, cap)
    return list(steps[:c]), list(res[:c])


def bgcr_spmm(A: "DeviceCSR", V, W, stream=None):
    dtype = BGCR_C128 if V.is_complex() else BGCR_F64
    _check(lib().bgcr_spmm(ctypes.byref(A.csr), dtype, int(V.shape[1]), _ptr(V), _ptr(W), _stream_handle(stream)),
           "bgcr_spmm")


def bgcr_apply_projected_work_bytes(n: int, p: int, kc: int) -> int:
    return int(lib().bgcr_apply_projected_work_bytes(int(n), int(p), int(kc)))


def bgcr_apply_projected(A: "DeviceCSR", C, V, W, variant: int, work, stream=None):
    """W = (I - C C^T) A V; C holds kc blocks of n x p (tensor of shape (kc, n, p),
    or None for kc = 0); work: device tensor of at least
    bgcr_apply_projected_work_bytes(n, p, kc) bytes."""
    p = int(V.shape[1])
    kc = 0 if C is None else int(C.shape[0])
    nbytes = work.numel() * work.element_size()
    _check(lib().bgcr_apply_projected(ctypes.byref(A.csr), p, kc, None if C is None else _ptr(C), _ptr(V), _ptr(W),
                                      int(variant), _ptr(work), nbytes, _stream_handle(stream)),
           "bgcr_apply_projected")


def bgcr_apply_projected_noalloc(A: "DeviceCSR", C, V, W, variant: int, stream=None):
    """As bgcr_apply_projected, with the library's own device workspace (no
    allocation in the call; calls overlapping on one GPU race)."""
    p = int(V.shape[1])
    kc = 0 if C is None else int(C.shape[0])
    _check(lib().bgcr_apply_projected_noalloc(ctypes.byref(A.csr), p, kc, None if C is None else _ptr(C), _ptr(V),
                                              _ptr(W), int(variant), _stream_handle(stream)),
           "bgcr_apply_projected_noalloc")


def bgcr_stream_probe(ins, outs, nwg: int = 0, stream=None):
    """Streaming-rate probe (a measurement aid): every tensor of outs receives
    the elementwise sum of the tensors of ins; all are contiguous FP64 device
    tensors of one even number of elements."""
    count = int(ins[0].numel())
    for t in list(ins) + list(outs):
        if t.dtype.itemsize != 8 or t.is_complex() or not t.is_contiguous() or int(t.numel()) != count:
            raise ValueError("bgcr_stream_probe: contiguous FP64 tensors of one size")
    ip = (ctypes.c_void_p * len(ins))(*[t.data_ptr() for t in ins])
    op = (ctypes.c_void_p * max(1, len(outs)))(*([t.data_ptr() for t in outs] or [0]))
    _check(lib().bgcr_stream_probe(ip, len(ins), op if outs else None, len(outs), count, int(nwg),
                                   _stream_handle(stream)), "bgcr_stream_probe")


def bgcr_set_profiling(seq, on: bool):
    _check(lib().bgcr_set_profiling(seq, int(bool(on))), "bgcr_set_profiling")


def bgcr_get_profile(seq):
    """{class: {"ms": total ms, "bytes": algorithmic bytes, "launches": count}}"""
    nc = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * nc)()
    by = (ctypes.c_double * nc)()
    ln = (ctypes.c_int64 * nc)()
    _check(lib().bgcr_get_profile(seq, ms, by, ln, nc), "bgcr_get_profile")
    return {name: {"ms": ms[i], "bytes": by[i], "launches": ln[i]} for i, name in enumerate(KERNEL_CLASSES)}


class DeviceCSR:
    """CSR matrix resident on the device (int32 indices, FP64/complex128 values)."""

    def __init__(self, row_ptr, col_idx, values):
        self.row_ptr, self.col_idx, self.values = row_ptr, col_idx, values
        n = row_ptr.numel() - 1
        self.n = n
        self.csr = bgcr_csr(n, values.numel(), row_ptr.data_ptr(), col_idx.data_ptr(), values.data_ptr())

    @classmethod
    def from_scipy(cls, A, device="cuda"):
        import numpy as np
        import torch
        A = A.tocsr()
        rp = torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int32)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).to(device)
        dt = np.complex128 if np.iscomplexobj(A.data) else np.float64
        va = torch.from_numpy(np.ascontiguousarray(A.data, dtype=dt)).to(device)
        return cls(rp, ci, va)


class Sequence:
    """One sequence of related systems sharing a device-resident recycle space."""

    def __init__(self, n, p, m, k, dtype=BGCR_F64, precision=BGCR_PLAIN_FP64, max_cycles=1000,
                 select_largest=False, stream=None, block_size=0, enlarge_cycles=0, ritz_vectors=False,
                 precond=BGCR_PRECOND_NONE):
        self.params = bgcr_params(p, m, k, dtype, precision, max_cycles, int(bool(select_largest)), int(block_size),
                                  int(enlarge_cycles), int(bool(ritz_vectors)), int(precond))
        self.n = n
        self.stream = stream
        self.handle = bgcr_create_sequence(self.params, n, stream)

    def solve(self, A: DeviceCSR, B, X, tol):
        return bgcr_solve(self.handle, A, B, X, tol)

    def recycle_dim(self):
        return bgcr_recycle_dim(self.handle)

    def get_recycle(self, U_out=None, C_out=None):
        bgcr_get_recycle(self.handle, U_out, C_out)

    def set_recycle(self, U):
        bgcr_set_recycle(self.handle, U)

    def cycle_log(self):
        return bgcr_get_cycle_log(self.handle)

    def set_profiling(self, on=True):
        bgcr_set_profiling(self.handle, on)

    def profile(self):
        return bgcr_get_profile(self.handle)

    def footprint(self, nnz):
        return bgcr_footprint_bytes(self.params, self.n, nnz)

    def release(self):
        if self.handle is not None:
            bgcr_release(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.release()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
