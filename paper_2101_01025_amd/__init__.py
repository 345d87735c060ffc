"""Exact Low(A * phi(A)) over F_p and F_p[i]/(i^2+1) on AMD MI355X.

Thin Python binding of the C-ABI library ``libffa.so`` (``include/ffa.h``):
argument marshalling only.  Every step of the computation runs in the HIP
kernels of ``csrc/``; PyTorch only provides device memory and the current
stream.  If the library is not built this module raises on use: there is no
CPU path.
"""
from __future__ import annotations

import ctypes
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# FFA_LIBRARY names another build of the same library (the host-sanitizer build of
# the tests); by default the in-tree libffa.so
LIB_PATH = os.environ.get("FFA_LIBRARY") or os.path.join(_HERE, "libffa.so")

OK, EINVAL, EPRIME, ERANGE, ENOMEM, EDEVICE, EUNSUPPORTED, EBOUND = 0, -1, -2, -3, -4, -5, -6, -7
ESCRATCH, EWAIT = -8, -9
SCRATCH_BYTES = 64 << 20  # FFA_SCRATCH_BYTES: fixed scratch of syrk_modp_noalloc per GPU
I64, I32, U16, U8, F64, I8_CENTRED = 0, 1, 2, 3, 4, 5
ALGO_AUTO, ALGO_CLASSICAL, ALGO_RECURSIVE = 0, 1, 2
CARRIER_AUTO, CARRIER_INT8, CARRIER_F64 = 0, 1, 2
LAUNCH_GRAPH, LAUNCH_DIRECT = 0, 1
OPERANDS_AUTO, OPERANDS_PLANES, OPERANDS_RAW = 0, 1, 2
STREAMS_AUTO, STREAMS_ONE, STREAMS_TWO = 0, 1, 2
HERK_AUTO, HERK_2M, HERK_4M = 0, 1, 2
GENERAL_AUTO, GENERAL_CLASSICAL, GENERAL_WINOGRAD = 0, 1, 2
PERSIST_AUTO, PERSIST_OFF, PERSIST_ON = 0, 1, 2

SYMBOLS = [
    "ffa_create", "ffa_destroy", "ffa_set_stream", "ffa_last_device_error", "ffa_status_string",
    "ffa_skew_unitary", "ffa_syrk_modp", "ffa_herk_modp2", "ffa_batch_syrk_plan",
    "ffa_batch_offsets", "ffa_batch_syrk_exec", "ffa_batch_destroy", "ffa_plan_describe",
    "ffa_profile_enable", "ffa_profile_read", "ffa_profile_reset",
    "ffa_autotune_syrk", "ffa_batch_autotune", "ffa_tune_export", "ffa_tune_import",
    "ffa_batch_describe", "ffa_syrk_modp_ex", "ffa_batch_herk_plan", "ffa_batch_herk_exec",
    "ffa_syrk_modp_noalloc", "ffa_device_status",
]
PHASE_COND, PHASE_PRE, PHASE_PRODUCTS, PHASE_POST = 0, 1, 2, 3


class FfaError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"ffa status {status} ({status_string(status)}) {msg}")


class Opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("levels", ctypes.c_int32), ("cutoff", ctypes.c_int32),
                ("carrier", ctypes.c_int32), ("check_inputs", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("launch", ctypes.c_int32), ("operands", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("herk_base", ctypes.c_int32),
                ("general", ctypes.c_int32), ("wino_min", ctypes.c_int32),
                ("persist", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def make_opts(algo=ALGO_AUTO, levels=-1, cutoff=0, carrier=CARRIER_AUTO, check_inputs=False,
              kernel=0, launch=LAUNCH_GRAPH, operands=OPERANDS_AUTO, streams=STREAMS_AUTO,
              herk_base=0, general=0, wino_min=0, persist=0):
    return Opts(algo, levels, cutoff, carrier, int(bool(check_inputs)), kernel, launch, operands,
                streams, herk_base, general, wino_min, persist)


_lib = None


def lib():
    """The loaded libffa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, u32, P = ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p
        L.ffa_create.argtypes = [ctypes.POINTER(P), i32, P]
        L.ffa_destroy.argtypes = [P]
        L.ffa_set_stream.argtypes = [P, P]
        L.ffa_last_device_error.argtypes = [P]
        L.ffa_device_status.argtypes = [P]
        L.ffa_status_string.argtypes = [i32]
        L.ffa_status_string.restype = ctypes.c_char_p
        L.ffa_skew_unitary.argtypes = [u32, i32, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                       ctypes.POINTER(i32)]
        L.ffa_syrk_modp.argtypes = [P, i64, i64, u32, i32, P, i64, i32, P, i64, P]
        L.ffa_syrk_modp_noalloc.argtypes = [P, i64, i64, u32, i32, P, i64, i32, P, i64, P]
        L.ffa_syrk_modp_ex.argtypes = [P, i32, i64, i64, u32, u32, i32, P, i64, u32, i32, P, i64, P]
        L.ffa_herk_modp2.argtypes = [P, i64, i64, u32, i32, P, P, i64, i32, P, P, i64, P]
        L.ffa_batch_syrk_plan.argtypes = [P, i64, P, P, u32, i32, i32, P, ctypes.POINTER(P)]
        L.ffa_batch_offsets.argtypes = [P, P, P, P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.ffa_batch_syrk_exec.argtypes = [P, P, P]
        L.ffa_batch_herk_plan.argtypes = [P, i64, P, P, u32, i32, i32, P, ctypes.POINTER(P)]
        L.ffa_batch_herk_exec.argtypes = [P, P, P, P, P]
        L.ffa_batch_destroy.argtypes = [P]
        L.ffa_profile_enable.argtypes = [P, i32]
        L.ffa_profile_read.argtypes = [P, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.ffa_profile_reset.argtypes = [P]
        L.ffa_autotune_syrk.argtypes = [P, i64, i64, u32, i32, P, i64, i32, P, i64, i32, P,
                                         ctypes.POINTER(ctypes.c_double)]
        L.ffa_batch_autotune.argtypes = [P, P, P, i32, P, ctypes.POINTER(ctypes.c_double)]
        L.ffa_batch_describe.argtypes = [P, ctypes.c_char_p, i64]
        L.ffa_tune_export.argtypes = [P, ctypes.c_char_p, i64]
        L.ffa_tune_export.restype = i64
        L.ffa_tune_import.argtypes = [P, ctypes.c_char_p]
        L.ffa_plan_describe.argtypes = [i64, i64, u32, i32, i32, i32, i64, i64, P, ctypes.c_char_p,
                                        i64]
        _lib = L
    return _lib


def status_string(s):
    try:
        return lib().ffa_status_string(s).decode()
    except Exception:
        return "?"


def _check(st, msg=""):
    if st != OK:
        raise FfaError(st, msg)


def skew_unitary(p, hermitian=False):
    """(a, b, kind) of the skew-unitary Y used for p (Section 4 of the paper)."""
    a, b, k = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int()
    _check(lib().ffa_skew_unitary(p, int(hermitian), ctypes.byref(a), ctypes.byref(b),
                                  ctypes.byref(k)))
    return a.value, b.value, k.value


def plan_describe(n, k, p, hermitian=False, dA=I64, dC=I64, lda=None, ldc=None, opts=None):
    """Host-only plan summary (dict) and the status the call would return."""
    buf = ctypes.create_string_buffer(4096)
    o = ctypes.byref(opts) if opts is not None else None
    st = lib().ffa_plan_describe(n, k, p, int(hermitian), dA, dC, lda if lda is not None else k,
                                 ldc if ldc is not None else n, o, buf, 4096)
    return st, json.loads(buf.value.decode())


PROFILE_ALL = 15


def device_status(device_index=0):
    """Synchronises the device's context and raises FfaError(EWAIT) if a bounded wait
    inside a kernel of an earlier call gave up (the results of those calls are not valid)."""
    _check(lib().ffa_device_status(context(device_index)), "device status")


def profile_enable(device_index, on=True, phases=PROFILE_ALL):
    """Phase timing on (for the phases of the bit mask `phases`) or off."""
    _check(lib().ffa_profile_enable(context(device_index), phases if on else 0))


def profile_reset(device_index):
    _check(lib().ffa_profile_reset(context(device_index)))


def profile_read(device_index, phase):
    """(total milliseconds, calls) of a phase measured with HIP events."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().ffa_profile_read(context(device_index), phase, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ---------------------------------------------------------------- torch glue

def _torch():
    import torch
    return torch


def _dtype_code(t, for_output=False):
    torch = _torch()
    m = {torch.int64: I64, torch.int32: I32, torch.uint8: U8, torch.float64: F64}
    if not for_output:
        m[torch.int8] = I8_CENTRED
    if hasattr(torch, "uint16"):
        m[torch.uint16] = U16
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


_contexts = {}


def context(device_index: int):
    """Per-device ffa_ctx (created on first use, kept for the process)."""
    c = _contexts.get(device_index)
    if c is None:
        h = ctypes.c_void_p()
        _check(lib().ffa_create(ctypes.byref(h), device_index, None), "ffa_create")
        c = _contexts[device_index] = h
    return c


def _prep(A):
    torch = _torch()
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if A.dim() != 2 or (A.numel() > 0 and A.stride(1) != 1):
        raise ValueError("A must be a row-major 2-D tensor")
    ctx = context(A.device.index)
    lib().ffa_set_stream(ctx, ctypes.c_void_p(torch.cuda.current_stream(A.device).cuda_stream))
    return ctx


def _out(C, n, device, dtype):
    torch = _torch()
    if C is None:
        C = torch.zeros((n, n), dtype=dtype, device=device)
    if not C.is_cuda or C.device != device:
        raise ValueError(f"C must be a tensor on {device}")
    if C.dim() != 2 or C.shape[0] != n or C.shape[1] != n or (n > 0 and C.stride(1) != 1):
        raise ValueError("C must be a row-major n x n tensor")
    if n > 1 and C.stride(0) < n:
        raise ValueError("C's rows overlap (row stride below n)")
    return C


def _ld(T, width):
    """Row stride in elements of a row-major 2-D tensor with `width` columns (a
    single row or an empty tensor has no meaningful stride: width is used)."""
    if T.shape[0] <= 1 or width == 0:
        return max(width, 1)
    if T.stride(0) < width:
        raise ValueError("the tensor's rows overlap (row stride below its width)")
    return T.stride(0)


def default_out_dtype(p):
    torch = _torch()
    if p < 256:
        return torch.uint8
    if p < 65536 and hasattr(torch, "uint16"):
        return torch.uint16
    return torch.int32


def syrk_modp(A, p, C=None, out_dtype=None, opts=None, alpha=1, beta=0, trans=False, **kw):
    """C = alpha Low(op(A) op(A)^T) + beta Low(C) mod p (ffa_syrk_modp, or ffa_syrk_modp_ex
    for alpha != 1, beta != 0 or trans: op(A) = A^T, A is k x n).  The strict upper part
    of C is left as is."""
    ctx = _prep(A)
    k, n = A.shape if trans else A.shape[::-1]
    C = _out(C, n, A.device, out_dtype or default_out_dtype(p))
    # no options at all: NULL, so that the library applies an autotuned record for the shape
    o = opts if opts is not None else (make_opts(**kw) if kw else None)
    ob = ctypes.byref(o) if o is not None else None
    lda = _ld(A, A.shape[1])
    ldc = _ld(C, n)
    if alpha == 1 and beta == 0 and not trans:
        st = lib().ffa_syrk_modp(ctx, n, k, p, _dtype_code(A), ctypes.c_void_p(A.data_ptr()), lda,
                                 _dtype_code(C, True), ctypes.c_void_p(C.data_ptr()), ldc, ob)
    else:
        st = lib().ffa_syrk_modp_ex(ctx, int(bool(trans)), n, k, p, alpha, _dtype_code(A),
                                    ctypes.c_void_p(A.data_ptr()), lda, beta, _dtype_code(C, True),
                                    ctypes.c_void_p(C.data_ptr()), ldc, ob)
    _check(st, f"(device error {lib().ffa_last_device_error(ctx)})" if st == EDEVICE else "")
    return C


def syrk_modp_noalloc(A, p, C, opts=None, **kw):
    """C = Low(A A^T) mod p through ffa_syrk_modp_noalloc: the library allocates no device
    memory in this call (its workspace is a fixed scratch of SCRATCH_BYTES per GPU), so C
    must be given.  Raises FfaError(ESCRATCH) when the call needs more scratch."""
    ctx = _prep(A)
    n, k = A.shape
    C = _out(C, n, A.device, C.dtype)
    o = opts if opts is not None else (make_opts(**kw) if kw else None)
    ob = ctypes.byref(o) if o is not None else None
    st = lib().ffa_syrk_modp_noalloc(ctx, n, k, p, _dtype_code(A), ctypes.c_void_p(A.data_ptr()),
                                     _ld(A, k), _dtype_code(C, True), ctypes.c_void_p(C.data_ptr()),
                                     _ld(C, n), ob)
    _check(st, f"(device error {lib().ffa_last_device_error(ctx)})" if st == EDEVICE else "")
    return C


def herk_modp2(A_re, A_im, p, C_re=None, C_im=None, out_dtype=None, opts=None, **kw):
    """Lower triangle of A A^H over F_p[i]/(i^2+1), planar re/im (ffa_herk_modp2)."""
    ctx = _prep(A_re)
    if A_im.shape != A_re.shape or A_im.stride() != A_re.stride() or A_im.dtype != A_re.dtype:
        raise ValueError("A_re and A_im must have the same shape, strides and dtype")
    n, k = A_re.shape
    od = out_dtype or default_out_dtype(p)
    C_re = _out(C_re, n, A_re.device, od)
    C_im = _out(C_im, n, A_re.device, od)
    if C_im.stride() != C_re.stride() or C_im.dtype != C_re.dtype:
        raise ValueError("C_re and C_im must have the same strides and dtype")
    # no options at all: NULL, so that the library applies an autotuned record for the shape
    o = opts if opts is not None else (make_opts(**kw) if kw else None)
    ob = ctypes.byref(o) if o is not None else None
    st = lib().ffa_herk_modp2(ctx, n, k, p, _dtype_code(A_re), ctypes.c_void_p(A_re.data_ptr()),
                              ctypes.c_void_p(A_im.data_ptr()), _ld(A_re, k),
                              _dtype_code(C_re, True), ctypes.c_void_p(C_re.data_ptr()),
                              ctypes.c_void_p(C_im.data_ptr()), _ld(C_re, n), ob)
    _check(st, f"(device error {lib().ffa_last_device_error(ctx)})" if st == EDEVICE else "")
    return C_re, C_im


def autotune_syrk(A, p, C=None, out_dtype=None, reps=3):
    """Runs the autotuner for this call; returns (chosen Opts, ms per call).  Later
    calls with the same shape and formats and no explicit options use the choice."""
    ctx = _prep(A)
    n, k = A.shape
    C = _out(C, n, A.device, out_dtype or default_out_dtype(p))
    best = Opts()
    ms = ctypes.c_double()
    st = lib().ffa_autotune_syrk(ctx, n, k, p, _dtype_code(A), ctypes.c_void_p(A.data_ptr()),
                                 _ld(A, k), _dtype_code(C, True),
                                 ctypes.c_void_p(C.data_ptr()), _ld(C, n), reps,
                                 ctypes.byref(best), ctypes.byref(ms))
    _check(st, "autotune")
    return best, ms.value


def tune_export(device_index=0):
    """The context's autotuner records as a JSON string."""
    ctx = context(device_index)
    need = lib().ffa_tune_export(ctx, None, 0)
    if need < 0:
        raise FfaError(int(need), "tune export")
    buf = ctypes.create_string_buffer(need + 1)
    lib().ffa_tune_export(ctx, buf, need + 1)
    return buf.value.decode()


def tune_import(text, device_index=0):
    """Adds autotuner records from tune_export's JSON; returns how many were taken."""
    st = lib().ffa_tune_import(context(device_index), text.encode())
    if st < 0:
        raise FfaError(st, "tune import")
    return st


class BatchSyrk:
    """Batched Low(A_i A_i^T) mod p over a packed layout (ffa_batch_syrk_*)."""

    _plan_fn = "ffa_batch_syrk_plan"

    def __init__(self, ns, ks, p, dA, dC, device_index=0, opts=None, **kw):
        import numpy as np
        self.count = len(ns)
        self.ns = np.ascontiguousarray(ns, dtype=np.int64)
        self.ks = np.ascontiguousarray(ks, dtype=np.int64)
        self.p = p
        self.dA, self.dC = dA, dC
        self.device_index = device_index
        self.ctx = context(device_index)
        self.opts = opts if opts is not None else make_opts(**kw)
        h = ctypes.c_void_p()
        _check(getattr(lib(), self._plan_fn)(self.ctx, self.count, self.ns.ctypes.data,
                                             self.ks.ctypes.data, p, dA, dC, ctypes.byref(self.opts),
                                             ctypes.byref(h)), "batch plan")
        self.handle = h
        self.a_off = np.zeros(self.count, np.int64)
        self.lda = np.zeros(self.count, np.int64)
        self.c_off = np.zeros(self.count, np.int64)
        at, ct = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ffa_batch_offsets(h, self.a_off.ctypes.data, self.lda.ctypes.data,
                                       self.c_off.ctypes.data, ctypes.byref(at), ctypes.byref(ct)))
        self.a_total, self.c_total = at.value, ct.value

    def pack(self, mats, dtype=None):
        """Host array of the packed A layout holding mats[i] (n_i x k_i each);
        padding columns are zero."""
        import numpy as np
        out = np.zeros(self.a_total, dtype=dtype or np.asarray(mats[0]).dtype)
        for i, M in enumerate(mats):
            n, k = int(self.ns[i]), int(self.ks[i])
            if n == 0:
                continue
            ld = int(self.lda[i])
            view = out[self.a_off[i]:self.a_off[i] + n * ld].reshape(n, ld)
            view[:, :k] = M
        return out

    def _packed(self, T, code, total, what, output):
        """Checks one packed buffer against the plan: a contiguous tensor on the
        plan's device, of the plan's format, holding at least `total` elements."""
        if not self.handle:
            raise ValueError("the batch plan is closed")
        if not T.is_cuda or T.device.index != self.device_index:
            raise ValueError(f"{what} must be a tensor on cuda:{self.device_index}")
        if _dtype_code(T, output) != code:
            raise ValueError(f"{what} has dtype {T.dtype}, the plan expects format {code}")
        if not T.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if T.numel() < total:
            raise ValueError(f"{what} holds {T.numel()} elements, the packed layout needs {total}")

    def run(self, A_packed, C_packed):
        torch = _torch()
        self._packed(A_packed, self.dA, self.a_total, "A_packed", False)
        self._packed(C_packed, self.dC, self.c_total, "C_packed", True)
        lib().ffa_set_stream(self.ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        _check(lib().ffa_batch_syrk_exec(self.handle, ctypes.c_void_p(A_packed.data_ptr()),
                                         ctypes.c_void_p(C_packed.data_ptr())), "batch exec")

    def autotune(self, A_packed, C_packed, reps=3):
        """Re-plans with each kernel configuration / cutoff, keeps the fastest."""
        torch = _torch()
        self._packed(A_packed, self.dA, self.a_total, "A_packed", False)
        self._packed(C_packed, self.dC, self.c_total, "C_packed", True)
        lib().ffa_set_stream(self.ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        best = Opts()
        ms = ctypes.c_double()
        _check(lib().ffa_batch_autotune(self.handle, ctypes.c_void_p(A_packed.data_ptr()),
                                        ctypes.c_void_p(C_packed.data_ptr()), reps,
                                        ctypes.byref(best), ctypes.byref(ms)), "batch autotune")
        return best, ms.value

    def describe(self):
        buf = ctypes.create_string_buffer(4096)
        _check(lib().ffa_batch_describe(self.handle, buf, 4096), "batch describe")
        return json.loads(buf.value.decode())

    def close(self):
        if self.handle:
            lib().ffa_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchHerk(BatchSyrk):
    """Batched Low(A_i A_i^H) over F_p[i] (ffa_batch_herk_*): planar real and
    imaginary parts, each in the packed layout of the plan (the same offsets in
    the four buffers)."""

    _plan_fn = "ffa_batch_herk_plan"

    def run(self, A_re, A_im, C_re, C_im):
        torch = _torch()
        self._packed(A_re, self.dA, self.a_total, "A_re", False)
        self._packed(A_im, self.dA, self.a_total, "A_im", False)
        self._packed(C_re, self.dC, self.c_total, "C_re", True)
        self._packed(C_im, self.dC, self.c_total, "C_im", True)
        lib().ffa_set_stream(self.ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        _check(lib().ffa_batch_herk_exec(self.handle, ctypes.c_void_p(A_re.data_ptr()),
                                         ctypes.c_void_p(A_im.data_ptr()),
                                         ctypes.c_void_p(C_re.data_ptr()),
                                         ctypes.c_void_p(C_im.data_ptr())), "batch herk exec")

    def autotune(self, *a, **kw):
        raise FfaError(EUNSUPPORTED, "the batch autotuner covers A A^T batches")
