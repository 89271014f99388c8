"""ctypes binding of libqnae.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import threading
from typing import NamedTuple, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libqnae.so"

QNAE_U8 = 1
QNAE_U16 = 2
PREDICATES = {"nae": 0, "sat": 1}  # QNAE_PRED_NAE, QNAE_PRED_SAT
_STATUS = {0: "QNAE_OK", -1: "QNAE_EINVAL", -2: "QNAE_ENOMEM", -3: "QNAE_EHIP",
           -4: "QNAE_EBUSY", -5: "QNAE_ETIMEDOUT", -6: "QNAE_ECANCELED"}


class QNAEError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Result(NamedTuple):
    p_success: float
    expected_cost: float
    norm: float


class _CResult(ctypes.Structure):
    _fields_ = [("p_success", ctypes.c_double), ("expected_cost", ctypes.c_double),
                ("norm", ctypes.c_double)]


class _CCostJob(ctypes.Structure):
    _fields_ = [("clauses", ctypes.POINTER(ctypes.c_int32)), ("m", ctypes.c_int32), ("n", ctypes.c_int32),
                ("k", ctypes.c_int32), ("cost_dev", ctypes.c_void_p), ("cost_dtype", ctypes.c_int32),
                ("num_solutions", ctypes.POINTER(ctypes.c_uint64)), ("predicate", ctypes.c_int32),
                ("half", ctypes.c_int32)]


class _CInstance(ctypes.Structure):
    _fields_ = [("cost_dev", ctypes.c_void_p), ("cost_dtype", ctypes.c_int32), ("n", ctypes.c_int32),
                ("m", ctypes.c_int32), ("p", ctypes.c_int32), ("gammas", ctypes.POINTER(ctypes.c_double)),
                ("betas", ctypes.POINTER(ctypes.c_double)), ("state_dev", ctypes.c_void_p), ("half", ctypes.c_int32)]


_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)


def _np_view(carr, cls):
    """A numpy structured view of a ctypes array of `cls` (pointer fields as
    uint64 addresses), for filling many records without a Python loop."""
    kinds = {ctypes.c_int32: np.int32, ctypes.c_double: np.float64, ctypes.c_uint64: np.uint64}
    names, formats, offsets = [], [], []
    for fname, ftype in cls._fields_:
        names.append(fname)
        formats.append(kinds.get(ftype, np.uint64))
        offsets.append(getattr(cls, fname).offset)
    dt = np.dtype({"names": names, "formats": formats, "offsets": offsets, "itemsize": ctypes.sizeof(cls)})
    return np.frombuffer(carr, dtype=dt)


def _packed_angles(values, name):
    """Concatenated float64 angles of every item, their offsets and counts."""
    if all(type(x) is np.ndarray and x.ndim == 1 and x.dtype == np.float64 for x in values):
        counts = np.fromiter((x.shape[0] for x in values), dtype=np.int64, count=len(values))
        offsets = np.concatenate(([0], np.cumsum(counts)[:-1])) if len(values) else np.zeros(0, dtype=np.int64)
        flat = np.ascontiguousarray(np.concatenate(values)) if counts.sum() else np.zeros(1)
        return flat, offsets.astype(np.uint64), counts
    arrs = []
    for i, x in enumerate(values):
        a = np.asarray(x, dtype=np.float64)
        if a.ndim > 1:
            raise ValueError(f"instance {i}: {name} must be 1-D")
        arrs.append(a.reshape(-1))
    counts = np.fromiter((a.shape[0] for a in arrs), dtype=np.int64, count=len(arrs))
    offsets = np.concatenate(([0], np.cumsum(counts)[:-1])) if len(arrs) else np.zeros(0, dtype=np.int64)
    flat = np.ascontiguousarray(np.concatenate(arrs)) if counts.sum() else np.zeros(1)
    return flat, offsets.astype(np.uint64), counts


class _CGradJob(ctypes.Structure):
    _fields_ = [("cost_dev", ctypes.c_void_p), ("cost_dtype", ctypes.c_int32), ("n", ctypes.c_int32),
                ("m", ctypes.c_int32), ("p", ctypes.c_int32), ("gammas", _F64P), ("betas", _F64P),
                ("dgammas", _F64P), ("dbetas", _F64P)]


class _CTune(ctypes.Structure):
    _fields_ = [("tile_bits", ctypes.c_int32), ("low_run_bits", ctypes.c_int32), ("page_bit", ctypes.c_int32),
                ("split", ctypes.c_int32), ("ms_per_layer", ctypes.c_double)]


class _CKernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


_lib = None
_lock = threading.Lock()


def library_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


def load_library():
    """Load libqnae.so (built in-tree by ``paper_2401_02852_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run `python -m paper_2401_02852_amd.build`")
        lib = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        lib.qnae_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        lib.qnae_destroy.argtypes = [vp]
        lib.qnae_last_error.argtypes = [vp]
        lib.qnae_last_error.restype = ctypes.c_char_p
        lib.qnae_build_cost_diagonal.argtypes = [vp, _I32P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), vp]
        lib.qnae_build_cost_diagonal_pred.argtypes = [vp, _I32P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                      ctypes.c_int32, vp, ctypes.c_int32,
                                                      ctypes.POINTER(ctypes.c_uint64), vp]
        lib.qnae_qaoa_run.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _F64P, _F64P,
                                      ctypes.c_int32, vp, ctypes.POINTER(_CResult), vp]
        lib.qnae_profile_enable.argtypes = [vp, ctypes.c_int]
        lib.qnae_profile_read.argtypes = [vp, ctypes.POINTER(_CKernelStat), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]
        lib.qnae_build_cost_diagonal_batched.argtypes = [vp, ctypes.POINTER(_CCostJob), ctypes.c_int32, vp]
        lib.qnae_qaoa_run_batched.argtypes = [vp, ctypes.POINTER(_CInstance), ctypes.c_int32,
                                              ctypes.POINTER(_CResult), vp]
        lib.qnae_qaoa_grad.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _F64P, _F64P,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _F64P, _F64P,
                                       ctypes.POINTER(_CResult), vp]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.qnae_qaoa_grad_batched.argtypes = [vp, ctypes.POINTER(_CGradJob), ctypes.c_int32, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_CResult), vp]
        lib.qnae_build_cost_diagonal_z2.argtypes = [vp, _I32P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                                    ctypes.c_int32, u64p, vp]
        lib.qnae_qaoa_run_noalloc.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _F64P, _F64P,
                                              ctypes.c_int32, vp, ctypes.POINTER(_CResult), vp]
        lib.qnae_qaoa_run_z2.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _F64P, _F64P,
                                         ctypes.c_int32, vp, ctypes.POINTER(_CResult), vp]
        lib.qnae_sample.argtypes = [vp, vp, ctypes.c_int32, vp, ctypes.c_int32, _F64P, ctypes.c_int32, u64p, _I32P,
                                    vp]
        tp = ctypes.POINTER(_CTune)
        lib.qnae_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, tp, vp]
        lib.qnae_set_tune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, tp]
        lib.qnae_autotune_batched.argtypes = [vp, ctypes.POINTER(_CInstance), ctypes.c_int32, ctypes.c_int32, tp, vp]
        lib.qnae_get_tune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, tp]
        lib.qnae_server_create.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(vp)]
        lib.qnae_server_submit.argtypes = [vp, _I32P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _F64P, _F64P,
                                           ctypes.c_int32, u64p]
        lib.qnae_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(_CResult),
                                         ctypes.POINTER(ctypes.c_double)]
        lib.qnae_server_stats.argtypes = [vp, u64p, u64p, u64p, u64p, u64p, u64p]
        lib.qnae_server_destroy.argtypes = [vp]
        lib.qnae_server_cancel.argtypes = [vp, ctypes.c_uint64]
        lib.qnae_server_pool_in_use.argtypes = [vp, u64p]
        for fn in (lib.qnae_create, lib.qnae_destroy, lib.qnae_build_cost_diagonal, lib.qnae_qaoa_run,
                   lib.qnae_build_cost_diagonal_pred,
                   lib.qnae_profile_enable, lib.qnae_profile_read, lib.qnae_build_cost_diagonal_batched,
                   lib.qnae_qaoa_run_batched, lib.qnae_qaoa_grad, lib.qnae_server_create, lib.qnae_server_submit,
                   lib.qnae_server_wait, lib.qnae_server_stats, lib.qnae_server_destroy, lib.qnae_autotune,
                   lib.qnae_set_tune, lib.qnae_get_tune, lib.qnae_sample, lib.qnae_build_cost_diagonal_z2,
                   lib.qnae_qaoa_run_z2, lib.qnae_qaoa_grad_batched, lib.qnae_server_cancel, lib.qnae_qaoa_run_noalloc,
                   lib.qnae_autotune_batched,
                   lib.qnae_server_pool_in_use):
            fn.restype = ctypes.c_int
        _lib = lib
        return lib


def _check(status: int, ctx=None):
    if status != 0:
        msg = load_library().qnae_last_error(ctx).decode(errors="replace")
        raise QNAEError(status, msg)


def _stream(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Context:
    """Owns a qnae_ctx (device scratch, phase tables, pinned staging)."""

    def __init__(self, device: Optional[int] = None):
        import torch
        lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(lib.qnae_create(ctypes.byref(h), self.device))
        self._h = h

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise QNAEError(-1, "context destroyed")
        return self._h

    def profile(self, on: bool = True):
        """Enable or disable event timing of every kernel this context launches."""
        _check(load_library().qnae_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kind: (launches, total_ms, algorithmic_bytes)}; clears the tallies."""
        buf = (_CKernelStat * 16)()
        cnt = ctypes.c_int32(0)
        _check(load_library().qnae_profile_read(self.handle, buf, 16, ctypes.byref(cnt)))
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms), float(buf[i].bytes))
                for i in range(min(cnt.value, 16))}

    def autotune(self, n: int, cost_dtype: str = "u8", reps: int = 3, stream=None) -> dict:
        """Time the sweep tile shapes at n (scratch memory, two-layer runs)
        and keep the fastest for this context; returns it ({} for n <= 14)."""
        t = _CTune()
        _check(load_library().qnae_autotune(self.handle, int(n), _dtype_code(cost_dtype), int(reps), ctypes.byref(t),
                                            _stream(stream)))
        return _tune_dict(t) if t.tile_bits else {}

    def set_tune(self, n: int, tune: Optional[dict], cost_dtype: str = "u8"):
        """Use `tune` ({tile_bits, low_run_bits, page_bit[, split]}) at n; None
        restores the default."""
        t = None
        if tune is not None:
            t = _CTune(int(tune["tile_bits"]), int(tune["low_run_bits"]), int(tune["page_bit"]),
                       int(tune.get("split", 0)), float(tune.get("ms_per_layer", 0.0)))
        _check(load_library().qnae_set_tune(self.handle, int(n), _dtype_code(cost_dtype),
                                            ctypes.byref(t) if t is not None else None))

    def get_tune(self, n: int, cost_dtype: str = "u8") -> dict:
        t = _CTune()
        _check(load_library().qnae_get_tune(self.handle, int(n), _dtype_code(cost_dtype), ctypes.byref(t)))
        return _tune_dict(t)

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().qnae_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dtype_code(name) -> int:
    codes = {"u8": QNAE_U8, "uint8": QNAE_U8, "u16": QNAE_U16, "uint16": QNAE_U16}
    if name not in codes:
        raise ValueError(f"cost dtype {name!r} is not u8/u16")
    return codes[name]


def _tune_dict(t) -> dict:
    return {"tile_bits": int(t.tile_bits), "low_run_bits": int(t.low_run_bits), "page_bit": int(t.page_bit),
            "split": int(t.split), "ms_per_layer": float(t.ms_per_layer)}


_default = threading.local()


def default_context() -> Context:
    """The calling thread's context on the current device: calls on one
    context must not overlap, and ctypes releases the GIL during a call, so
    each thread gets its own."""
    import torch
    dev = torch.cuda.current_device()
    ctxs = getattr(_default, "by_device", None)
    if ctxs is None:
        ctxs = _default.by_device = {}
    if dev not in ctxs:
        ctxs[dev] = Context(dev)
    return ctxs[dev]


def _device_buffer(t, name: str, ctx: "Context", dtypes, numel: int) -> int:
    """Address of a tensor handed to the library as a device buffer, after
    checking what the kernels assume of it: on this context's GPU,
    contiguous, of one of `dtypes` and with exactly `numel` entries. A host
    tensor would hand the kernels a host address, a short one would be
    written past its end and a strided view would be read as dense, so each
    is rejected here, before any call."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU, got device {t.device}")
    if t.device.index != ctx.device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{ctx.device}")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected " + " or ".join(str(d) for d in dtypes))
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _device_buffers(ts, name: str, ctx: "Context", dtypes, numels):
    """_device_buffer over a list with one pass per property: (addresses,
    cost type codes) as arrays. The first failing entry is reported by
    _device_buffer itself."""
    import torch
    count = len(ts)
    if count == 0:
        return np.zeros(0, dtype=np.uint64), np.zeros(0, dtype=np.int32)
    codes = _DTYPE_CODES
    try:  # three passes: (device, contiguous), (entries, dtype), address
        dc = np.fromiter((2 * t.get_device() + t.is_contiguous() for t in ts), dtype=np.int64, count=count)
        nt = np.fromiter((4 * t.numel() + codes.get(t.dtype, 0) for t in ts), dtype=np.int64, count=count)
        ptr = np.fromiter((t.data_ptr() for t in ts), dtype=np.uint64, count=count)
    except AttributeError:
        dc = None
    if dc is None or not isinstance(ts[0], torch.Tensor):
        ptr, typ = None, None
        bad = range(count)
    else:
        typ = (nt & 3).astype(np.int32)
        allowed = np.array([codes[d] for d in dtypes], dtype=np.int32)
        bad = np.nonzero((dc != 2 * ctx.device + 1) | ~np.isin(typ, allowed) | ((nt >> 2) != np.asarray(numels)))[0]
    for i in bad:
        _device_buffer(ts[i], f"{name}[{i}]", ctx, dtypes, int(np.broadcast_to(numels, (count,))[i]))
    return ptr, typ


_DTYPE_CODES = {}


def _check_n(n):
    if not 1 <= int(n) <= 34:
        raise ValueError(f"n={n} outside [1, 34]")


def _cost_types():
    import torch
    if not _DTYPE_CODES:
        _DTYPE_CODES.update({torch.uint8: QNAE_U8, torch.uint16: QNAE_U16, torch.complex64: 3})
    return (torch.uint8, torch.uint16)


def _state_types():
    import torch
    _cost_types()
    return (torch.complex64,)


def _cost_code(t) -> int:
    import torch
    return QNAE_U8 if t.dtype == torch.uint8 else QNAE_U16


def cost_dtype_for(m: int):
    import torch
    return torch.uint8 if m <= 255 else torch.uint16


def _pred_code(predicate) -> int:
    if predicate not in PREDICATES:
        raise ValueError(f"predicate {predicate!r} is not 'nae' or 'sat'")
    return PREDICATES[predicate]


def build_cost_diagonal(clauses, n: int, *, out=None, count_solutions: bool = False, predicate: str = "nae",
                        ctx: Optional[Context] = None, stream=None):
    """C(x) for x in [0, 2^n) on the current device, uint8 when m <= 255 else
    uint16. ``clauses`` is an [m, k] int array of DIMACS-style literals;
    ``predicate`` "nae" (the paper's problem) or "sat" (plain k-SAT).
    Returns the tensor, or (tensor, #solutions) with count_solutions."""
    import torch
    cl = np.ascontiguousarray(np.asarray(clauses, dtype=np.int32))
    if cl.ndim != 2:
        raise ValueError("clauses must be an [m, k] literal array")
    m, k = cl.shape
    _check_n(n)
    ctx = ctx or default_context()
    if out is None:
        out = torch.empty(1 << n, dtype=cost_dtype_for(m), device=f"cuda:{ctx.device}")
    ptr = _device_buffer(out, "out", ctx, _cost_types(), 1 << n)
    sols = ctypes.c_uint64(0)
    _check(load_library().qnae_build_cost_diagonal_pred(
        ctx.handle, cl.ctypes.data_as(_I32P) if m else None, m, n, max(k, 1), _pred_code(predicate),
        ctypes.c_void_p(ptr), _cost_code(out),
        ctypes.byref(sols) if count_solutions else None, _stream(stream)))
    return (out, int(sols.value)) if count_solutions else out


def qaoa_run(cost, n: int, m: int, gammas, betas, *, state=None, ctx: Optional[Context] = None,
             stream=None) -> Result:
    """Depth-p QAOA from |+> on the cost diagonal; returns (p_success,
    expected_cost, norm). ``state``, if given, is a complex64 device tensor of
    2^n entries that receives the final state."""
    g = np.ascontiguousarray(np.atleast_1d(np.asarray(gammas, dtype=np.float64)))
    b = np.ascontiguousarray(np.atleast_1d(np.asarray(betas, dtype=np.float64)))
    if g.shape != b.shape or g.ndim != 1:
        raise ValueError("gammas and betas must be 1-D of equal length")
    _check_n(n)
    ctx = ctx or default_context()
    cptr = _device_buffer(cost, "cost", ctx, _cost_types(), 1 << n)
    sptr = _device_buffer(state, "state", ctx, _state_types(), 1 << n) if state is not None else None
    res = _CResult()
    p = g.shape[0]
    _check(load_library().qnae_qaoa_run(
        ctx.handle, ctypes.c_void_p(cptr), _cost_code(cost), n, m,
        g.ctypes.data_as(_F64P) if p else None, b.ctypes.data_as(_F64P) if p else None, p,
        ctypes.c_void_p(sptr) if sptr is not None else None,
        ctypes.byref(res), _stream(stream)))
    return Result(res.p_success, res.expected_cost, res.norm)


def qaoa_run_noalloc(cost, n: int, m: int, gammas, betas, *, state=None, ctx: Optional[Context] = None,
                     stream=None) -> Result:
    """qaoa_run through the entry point that allocates nothing (device
    scratch in the library's static array; for callers that cannot allocate).
    ``state`` (complex64, 2^n on the device) is required for n > 14."""
    g = np.ascontiguousarray(np.atleast_1d(np.asarray(gammas, dtype=np.float64)))
    b = np.ascontiguousarray(np.atleast_1d(np.asarray(betas, dtype=np.float64)))
    if g.shape != b.shape or g.ndim != 1:
        raise ValueError("gammas and betas must be 1-D of equal length")
    _check_n(n)
    ctx = ctx or default_context()
    cptr = _device_buffer(cost, "cost", ctx, _cost_types(), 1 << n)
    sptr = _device_buffer(state, "state", ctx, _state_types(), 1 << n) if state is not None else None
    res = _CResult()
    p = g.shape[0]
    _check(load_library().qnae_qaoa_run_noalloc(
        ctx.handle, ctypes.c_void_p(cptr), _cost_code(cost), n, m,
        g.ctypes.data_as(_F64P) if p else None, b.ctypes.data_as(_F64P) if p else None, p,
        ctypes.c_void_p(sptr) if sptr is not None else None, ctypes.byref(res), _stream(stream)))
    return Result(res.p_success, res.expected_cost, res.norm)


def _per_item(value, count, name):
    vals = list(value) if isinstance(value, (list, tuple)) else [value] * count
    if len(vals) != count:
        raise ValueError(f"{name} list has {len(vals)} entries, expected {count}")
    return vals


def build_cost_diagonals(clause_sets, ns, *, outs=None, count_solutions: bool = False, predicate="nae",
                         half=False, ctx: Optional[Context] = None, stream=None):
    """Batched build_cost_diagonal: one tensor per (clauses, n) pair, built
    with one launch per cost type. ``predicate`` is one name for all or a list
    of names; ``half`` (one flag or a list) builds the lower half only, as
    build_cost_diagonal_z2. Returns the list of tensors, or (tensors, solution
    counts) with count_solutions."""
    import torch
    arrs = [np.asarray(c, dtype=np.int32) for c in clause_sets]
    if len(arrs) != len(ns):
        raise ValueError("clause_sets and ns differ in length")
    halves = _per_item(half, len(arrs), "half")
    ctx = ctx or default_context()
    if outs is None:
        outs = [torch.empty(1 << (n - (1 if hf else 0)), dtype=cost_dtype_for(a.shape[0]), device=f"cuda:{ctx.device}")
                for a, n, hf in zip(arrs, ns, halves)]
    if len(outs) != len(arrs):
        raise ValueError("outs and clause_sets differ in length")
    count = len(arrs)
    preds = [predicate] * count if isinstance(predicate, str) else list(predicate)
    if len(preds) != count:
        raise ValueError("predicate list and clause_sets differ in length")
    if any(a.ndim != 2 for a in arrs):
        raise ValueError("clauses must be [m, k] literal arrays")
    mk = np.empty((count, 2), dtype=np.int64)
    mk[:, 0] = np.fromiter((a.shape[0] for a in arrs), dtype=np.int64, count=count)
    mk[:, 1] = np.fromiter((a.shape[1] for a in arrs), dtype=np.int64, count=count)
    # every job's literals in one buffer (one address, offsets by arithmetic)
    flat = np.concatenate([a.reshape(-1) for a in arrs]) if count and mk.prod(axis=1).sum() else np.zeros(1, np.int32)
    lit_at = np.concatenate(([0], np.cumsum(mk.prod(axis=1))[:-1])).astype(np.uint64) if count else np.zeros(0, np.uint64)
    hv = np.asarray(halves, dtype=bool)
    nv = np.asarray(ns, dtype=np.int64).reshape(count)
    if np.any(nv < 1) or np.any(nv > 34):
        i = int(np.nonzero((nv < 1) | (nv > 34))[0][0])
        raise ValueError(f"job {i}: n={int(nv[i])} outside [1, 34]")
    ptrs, codes = _device_buffers(outs, "outs", ctx, _cost_types(), np.left_shift(np.int64(1), nv - hv))
    sols = np.zeros(max(count, 1), dtype=np.uint64)
    jobs = (_CCostJob * count)()
    v = _np_view(jobs, _CCostJob)
    v["clauses"] = np.where(mk[:, 0] > 0, np.uint64(flat.ctypes.data) + np.uint64(4) * lit_at, np.uint64(0))
    v["m"] = mk[:, 0]
    v["n"] = nv
    v["k"] = np.maximum(mk[:, 1], 1)
    v["cost_dev"] = ptrs
    v["cost_dtype"] = codes
    v["num_solutions"] = (np.uint64(sols.ctypes.data) + np.uint64(8) * np.arange(count, dtype=np.uint64)
                          if count_solutions else np.uint64(0))
    v["predicate"] = np.fromiter((_pred_code(x) for x in preds), dtype=np.int32, count=count)
    v["half"] = hv
    _check(load_library().qnae_build_cost_diagonal_batched(ctx.handle, jobs, count, _stream(stream)))
    return (outs, [int(x) for x in sols[:count]]) if count_solutions else outs


def _instances(costs, ns, ms, gammas, betas, states, half, ctx):
    """The qnae_instance array of a batch (and the angle arrays it points
    into, which must outlive the call)."""
    count = len(costs)
    if not (len(ns) == len(ms) == len(gammas) == len(betas) == count):
        raise ValueError("argument lists differ in length")
    halves = np.asarray(_per_item(half, count, "half"), dtype=bool)
    G, goff, gcnt = _packed_angles(gammas, "gammas")
    B, boff, bcnt = _packed_angles(betas, "betas")
    bad = np.nonzero(gcnt != bcnt)[0]
    if bad.size:
        raise ValueError(f"instance {int(bad[0])}: gammas and betas must be 1-D of equal length")
    nv = np.asarray(ns, dtype=np.int64).reshape(count)
    if np.any(nv < 1) or np.any(nv > 34):
        i = int(np.nonzero((nv < 1) | (nv > 34))[0][0])
        raise ValueError(f"instance {i}: n={int(nv[i])} outside [1, 34]")
    stored = nv - halves
    cost_ptr, codes = _device_buffers(costs, "costs", ctx, _cost_types(), np.left_shift(np.int64(1), stored))
    state_ptr = np.zeros(count, dtype=np.uint64)
    if states is not None:
        if len(states) != count:
            raise ValueError("states and costs differ in length")
        for i, st in enumerate(states):
            if st is not None:
                state_ptr[i] = _device_buffer(st, f"states[{i}]", ctx, _state_types(), 1 << int(stored[i]))
    inst = (_CInstance * count)()
    v = _np_view(inst, _CInstance)
    v["cost_dev"] = cost_ptr
    v["cost_dtype"] = codes
    v["n"] = nv
    v["m"] = np.asarray(ms, dtype=np.int64).reshape(count)
    v["p"] = gcnt
    v["gammas"] = np.where(gcnt > 0, np.uint64(G.ctypes.data) + np.uint64(8) * goff, np.uint64(0))
    v["betas"] = np.where(gcnt > 0, np.uint64(B.ctypes.data) + np.uint64(8) * boff, np.uint64(0))
    v["state_dev"] = state_ptr
    v["half"] = halves
    return inst, (G, B)


def qaoa_run_batched(costs, ns, ms, gammas, betas, *, states=None, half=False, ctx: Optional[Context] = None,
                     stream=None):
    """Batched qaoa_run over many instances; returns a list of Result.
    ``half`` (one flag or a list) solves an instance on the half state as
    qaoa_run_z2 (its cost and state then hold 2^(n-1) entries)."""
    count = len(costs)
    ctx = ctx or default_context()
    inst, _keep = _instances(costs, ns, ms, gammas, betas, states, half, ctx)
    res = (_CResult * count)()
    _check(load_library().qnae_qaoa_run_batched(ctx.handle, inst, count, res, _stream(stream)))
    return list(map(Result._make, np.frombuffer(res, dtype=np.float64).reshape(count, 3).tolist()))


def autotune_batched(costs, ns, ms, gammas, betas, *, states=None, half=False, reps: int = 3,
                     ctx: Optional[Context] = None, stream=None) -> dict:
    """Tune the batched path's tile shape on this batch (every candidate
    shape, `reps` timed runs each) and keep the fastest on the context for
    every (n, cost type) of its instances with n > 14; returns it ({} when
    there are none)."""
    count = len(costs)
    ctx = ctx or default_context()
    inst, _keep = _instances(costs, ns, ms, gammas, betas, states, half, ctx)
    t = _CTune()
    _check(load_library().qnae_autotune_batched(ctx.handle, inst, count, int(reps), ctypes.byref(t), _stream(stream)))
    return _tune_dict(t) if t.tile_bits else {}


class PreparedCostBuild:
    """build_cost_diagonals with the arguments marshalled once: the device
    buffers are checked and the literals copied into one buffer when it is
    made, so build() is one library call (the library rebuilds the clause
    records and the diagonals every time). Later changes to the clause arrays
    are not seen."""

    def __init__(self, clause_sets, ns, *, outs=None, predicate="nae", half=False, ctx: Optional[Context] = None):
        import torch
        arrs = [np.asarray(c, dtype=np.int32) for c in clause_sets]
        count = len(arrs)
        if len(ns) != count:
            raise ValueError("clause_sets and ns differ in length")
        if any(a.ndim != 2 for a in arrs):
            raise ValueError("clauses must be [m, k] literal arrays")
        halves = np.asarray(_per_item(half, count, "half"), dtype=bool)
        ctx = ctx or default_context()
        nv = np.asarray(ns, dtype=np.int64).reshape(count)
        if np.any(nv < 1) or np.any(nv > 34):
            i = int(np.nonzero((nv < 1) | (nv > 34))[0][0])
            raise ValueError(f"job {i}: n={int(nv[i])} outside [1, 34]")
        if outs is None:
            outs = [torch.empty(1 << int(n - hf), dtype=cost_dtype_for(a.shape[0]), device=f"cuda:{ctx.device}")
                    for a, n, hf in zip(arrs, nv, halves)]
        if len(outs) != count:
            raise ValueError("outs and clause_sets differ in length")
        preds = [predicate] * count if isinstance(predicate, str) else list(predicate)
        if len(preds) != count:
            raise ValueError("predicate list and clause_sets differ in length")
        ptrs, codes = _device_buffers(outs, "outs", ctx, _cost_types(), np.left_shift(np.int64(1), nv - halves))
        mk = np.array([a.shape for a in arrs], dtype=np.int64).reshape(count, 2)
        size = mk.prod(axis=1)
        self._lits = np.concatenate([a.reshape(-1) for a in arrs]) if size.sum() else np.zeros(1, np.int32)
        lit_at = np.concatenate(([0], np.cumsum(size)[:-1])).astype(np.uint64) if count else np.zeros(0, np.uint64)
        self._sols = np.zeros(max(count, 1), dtype=np.uint64)
        self._jobs = (_CCostJob * count)()
        v = _np_view(self._jobs, _CCostJob)
        v["clauses"] = np.where(mk[:, 0] > 0, np.uint64(self._lits.ctypes.data) + np.uint64(4) * lit_at, np.uint64(0))
        v["m"] = mk[:, 0]
        v["n"] = nv
        v["k"] = np.maximum(mk[:, 1], 1)
        v["cost_dev"] = ptrs
        v["cost_dtype"] = codes
        v["predicate"] = np.fromiter((_pred_code(x) for x in preds), dtype=np.int32, count=count)
        v["half"] = halves
        self._view, self._count, self._ctx, self.outs = v, count, ctx, outs

    def build(self, *, count_solutions: bool = False, stream=None):
        """The diagonals into ``outs``; with count_solutions also the
        solution counts."""
        self._view["num_solutions"] = (np.uint64(self._sols.ctypes.data) + np.uint64(8) *
                                       np.arange(self._count, dtype=np.uint64) if count_solutions else np.uint64(0))
        _check(load_library().qnae_build_cost_diagonal_batched(self._ctx.handle, self._jobs, self._count,
                                                               _stream(stream)))
        return (self.outs, [int(x) for x in self._sols[:self._count]]) if count_solutions else self.outs


class PreparedBatch:
    """qaoa_run_batched with the instances marshalled once (device buffers
    checked, instance records built); run() takes the angles and makes one
    library call. Angles may be a [count, p] float64 array when every
    instance has the same p (no per-instance work at all), or per-instance
    1-D arrays as for qaoa_run_batched; each instance's p is fixed here."""

    def __init__(self, costs, ns, ms, ps, *, states=None, half=False, ctx: Optional[Context] = None):
        count = len(costs)
        ctx = ctx or default_context()
        pv = np.asarray(ps, dtype=np.int64).reshape(count)
        if np.any(pv < 0):
            raise ValueError("p must be >= 0")
        zero = [np.zeros(int(p)) for p in pv]
        self._inst, _ = _instances(costs, ns, ms, zero, zero, states, half, ctx)
        self._view = _np_view(self._inst, _CInstance)
        self._p = pv
        self._at = np.concatenate(([0], np.cumsum(pv)[:-1])).astype(np.uint64) if count else np.zeros(0, np.uint64)
        self._count, self._ctx = count, ctx
        self._keep = (costs, states)
        self._res = (_CResult * max(count, 1))()

    def _angles(self, values, name):
        if isinstance(values, np.ndarray) and values.ndim == 2:
            a = np.ascontiguousarray(values, dtype=np.float64)
            if a.shape[0] != self._count or np.any(self._p != a.shape[1]):
                raise ValueError(f"{name}: shape {a.shape} does not match the prepared p of every instance")
            return a, np.uint64(a.shape[1]) * np.arange(self._count, dtype=np.uint64)
        if len(values) != self._count:
            raise ValueError(f"{name}: {len(values)} entries, expected {self._count}")
        flat, off, cnt = _packed_angles(values, name)
        if np.any(cnt != self._p):
            i = int(np.nonzero(cnt != self._p)[0][0])
            raise ValueError(f"instance {i}: {name} has {int(cnt[i])} entries, prepared p={int(self._p[i])}")
        return flat, off

    def run(self, gammas, betas, *, stream=None) -> np.ndarray:
        """Results as a [count, 3] array: p_success, expected_cost, norm."""
        G, goff = self._angles(gammas, "gammas")
        B, boff = self._angles(betas, "betas")
        has = self._p > 0
        self._view["gammas"] = np.where(has, np.uint64(G.ctypes.data) + np.uint64(8) * goff, np.uint64(0))
        self._view["betas"] = np.where(has, np.uint64(B.ctypes.data) + np.uint64(8) * boff, np.uint64(0))
        _check(load_library().qnae_qaoa_run_batched(self._ctx.handle, self._inst, self._count, self._res,
                                                    _stream(stream)))
        return np.frombuffer(self._res, dtype=np.float64)[:3 * self._count].reshape(self._count, 3).copy()


def qaoa_grad(cost, n: int, m: int, gammas, betas, *, w_psucc: float = 1.0, w_energy: float = 0.0,
              checkpoint_every: int = 4, ctx: Optional[Context] = None, stream=None):
    """Adjoint gradient of w_psucc * p_succ + w_energy * E[C].

    Returns (dgammas, dbetas, Result) with float64 numpy arrays."""
    g = np.ascontiguousarray(np.atleast_1d(np.asarray(gammas, dtype=np.float64)))
    b = np.ascontiguousarray(np.atleast_1d(np.asarray(betas, dtype=np.float64)))
    if g.shape != b.shape or g.ndim != 1:
        raise ValueError("gammas and betas must be 1-D of equal length")
    _check_n(n)
    ctx = ctx or default_context()
    cptr = _device_buffer(cost, "cost", ctx, _cost_types(), 1 << n)
    p = g.shape[0]
    dg = np.zeros(p, dtype=np.float64)
    db = np.zeros(p, dtype=np.float64)
    res = _CResult()
    _check(load_library().qnae_qaoa_grad(
        ctx.handle, ctypes.c_void_p(cptr), _cost_code(cost), n, m,
        g.ctypes.data_as(_F64P) if p else None, b.ctypes.data_as(_F64P) if p else None, p,
        float(w_psucc), float(w_energy), int(checkpoint_every),
        dg.ctypes.data_as(_F64P) if p else None, db.ctypes.data_as(_F64P) if p else None,
        ctypes.byref(res), _stream(stream)))
    return dg, db, Result(res.p_success, res.expected_cost, res.norm)


def qaoa_grad_batched(costs, ns, ms, gammas, betas, *, w_psucc: float = 1.0, w_energy: float = 0.0,
                      checkpoint_every: int = 4, ctx: Optional[Context] = None, stream=None):
    """qaoa_grad for many instances; returns (dgammas list, dbetas list,
    Result list). Instances with n <= 13 share one launch."""
    count = len(costs)
    if not (len(ns) == len(ms) == len(gammas) == len(betas) == count):
        raise ValueError("argument lists differ in length")
    ctx = ctx or default_context()
    jobs = (_CGradJob * count)()
    keep, dgs, dbs = [], [], []
    for i in range(count):
        g = np.ascontiguousarray(np.atleast_1d(np.asarray(gammas[i], dtype=np.float64)))
        b = np.ascontiguousarray(np.atleast_1d(np.asarray(betas[i], dtype=np.float64)))
        if g.shape != b.shape or g.ndim != 1:
            raise ValueError(f"instance {i}: gammas and betas must be 1-D of equal length")
        if not 1 <= int(ns[i]) <= 34:
            raise ValueError(f"instance {i}: n={int(ns[i])} outside [1, 34]")
        cptr = _device_buffer(costs[i], f"costs[{i}]", ctx, _cost_types(), 1 << int(ns[i]))
        p = g.shape[0]
        dg, db = np.zeros(p), np.zeros(p)
        keep += [g, b]
        dgs.append(dg)
        dbs.append(db)
        jobs[i].cost_dev = cptr
        jobs[i].cost_dtype = _cost_code(costs[i])
        jobs[i].n, jobs[i].m, jobs[i].p = int(ns[i]), int(ms[i]), p
        if p:
            jobs[i].gammas, jobs[i].betas = g.ctypes.data_as(_F64P), b.ctypes.data_as(_F64P)
            jobs[i].dgammas, jobs[i].dbetas = dg.ctypes.data_as(_F64P), db.ctypes.data_as(_F64P)
    res = (_CResult * max(count, 1))()
    _check(load_library().qnae_qaoa_grad_batched(ctx.handle, jobs, count, float(w_psucc), float(w_energy),
                                                 int(checkpoint_every), res, _stream(stream)))
    return dgs, dbs, [Result(r.p_success, r.expected_cost, r.norm) for r in res[:count]]


def build_cost_diagonal_z2(clauses, n: int, *, out=None, count_solutions: bool = False,
                           ctx: Optional[Context] = None, stream=None):
    """Lower half (x < 2^(n-1)) of the NAE cost diagonal, for qaoa_run_z2;
    with count_solutions also the solution count of the whole diagonal."""
    import torch
    cl = np.ascontiguousarray(np.asarray(clauses, dtype=np.int32))
    if cl.ndim != 2:
        raise ValueError("clauses must be an [m, k] literal array")
    m, k = cl.shape
    if not 2 <= n <= 34:
        raise ValueError(f"n={n} outside [2, 34] for a half diagonal")
    ctx = ctx or default_context()
    if out is None:
        out = torch.empty(1 << (n - 1), dtype=cost_dtype_for(m), device=f"cuda:{ctx.device}")
    ptr = _device_buffer(out, "out", ctx, _cost_types(), 1 << (n - 1))
    sols = ctypes.c_uint64(0)
    _check(load_library().qnae_build_cost_diagonal_z2(
        ctx.handle, cl.ctypes.data_as(_I32P) if m else None, m, n, max(k, 1), ctypes.c_void_p(ptr), _cost_code(out),
        ctypes.byref(sols) if count_solutions else None, _stream(stream)))
    return (out, int(sols.value)) if count_solutions else out


def qaoa_run_z2(cost_half, n: int, m: int, gammas, betas, *, state=None, ctx: Optional[Context] = None,
                stream=None) -> Result:
    """qaoa_run on the half-state representation (NAE instances, n >= 15):
    ``cost_half`` from build_cost_diagonal_z2; ``state``, if given, receives
    the lower half of the final state (2^(n-1) complex64)."""
    g = np.ascontiguousarray(np.atleast_1d(np.asarray(gammas, dtype=np.float64)))
    b = np.ascontiguousarray(np.atleast_1d(np.asarray(betas, dtype=np.float64)))
    if g.shape != b.shape or g.ndim != 1:
        raise ValueError("gammas and betas must be 1-D of equal length")
    if not 2 <= n <= 34:
        raise ValueError(f"n={n} outside [2, 34] for a half state")
    ctx = ctx or default_context()
    cptr = _device_buffer(cost_half, "cost_half", ctx, _cost_types(), 1 << (n - 1))
    sptr = _device_buffer(state, "state", ctx, _state_types(), 1 << (n - 1)) if state is not None else None
    res = _CResult()
    p = g.shape[0]
    _check(load_library().qnae_qaoa_run_z2(
        ctx.handle, ctypes.c_void_p(cptr), _cost_code(cost_half), n, m,
        g.ctypes.data_as(_F64P) if p else None, b.ctypes.data_as(_F64P) if p else None, p,
        ctypes.c_void_p(sptr) if sptr is not None else None, ctypes.byref(res), _stream(stream)))
    return Result(res.p_success, res.expected_cost, res.norm)


def sample(state, n: int, uniforms, *, cost=None, ctx: Optional[Context] = None, stream=None):
    """Outcomes of measuring `state` (complex64, 2^n, on the device), one per
    uniform in [0, 1): the smallest x whose cumulative |psi|^2 mass in index
    order exceeds u times the total. Returns (samples uint64, costs int32 or
    None); costs are C(sample) when the cost diagonal is given."""
    if not 1 <= n <= 34:
        raise ValueError(f"n={n} outside [1, 34]")
    ctx = ctx or default_context()
    sptr = _device_buffer(state, "state", ctx, _state_types(), 1 << n)
    cptr = _device_buffer(cost, "cost", ctx, _cost_types(), 1 << n) if cost is not None else None
    u = np.ascontiguousarray(np.atleast_1d(np.asarray(uniforms, dtype=np.float64)))
    count = u.shape[0]
    out = np.zeros(count, dtype=np.uint64)
    costs = np.zeros(count, dtype=np.int32) if cost is not None else None
    _check(load_library().qnae_sample(
        ctx.handle, ctypes.c_void_p(sptr), n,
        ctypes.c_void_p(cptr) if cptr is not None else None, _cost_code(cost) if cost is not None else 0,
        u.ctypes.data_as(_F64P) if count else None, count,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if count else None,
        costs.ctypes.data_as(_I32P) if costs is not None and count else None, _stream(stream)))
    return out, costs


class Server:
    """Continuous-batching solve server (qnae_server_*): submit instances,
    collect results; requests share GPU launches while they are active."""

    def __init__(self, pool_bytes: int = 64 << 30, max_slots: int = 256, ctx: Optional[Context] = None):
        self._ctx = ctx or default_context()
        h = ctypes.c_void_p()
        _check(load_library().qnae_server_create(self._ctx.handle, int(pool_bytes), int(max_slots), ctypes.byref(h)))
        self._h = h

    def submit(self, clauses, n: int, gammas, betas) -> int:
        cl = np.ascontiguousarray(np.asarray(clauses, dtype=np.int32))
        if cl.ndim != 2:
            raise ValueError("clauses must be an [m, k] literal array")
        m, k = cl.shape
        g = np.ascontiguousarray(np.atleast_1d(np.asarray(gammas, dtype=np.float64)))
        b = np.ascontiguousarray(np.atleast_1d(np.asarray(betas, dtype=np.float64)))
        if g.shape != b.shape or g.ndim != 1:
            raise ValueError("gammas and betas must be 1-D of equal length")
        t = ctypes.c_uint64(0)
        p = g.shape[0]
        _check(load_library().qnae_server_submit(
            self._h, cl.ctypes.data_as(_I32P) if m else None, m, int(n), max(k, 1),
            g.ctypes.data_as(_F64P) if p else None, b.ctypes.data_as(_F64P) if p else None, p, ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(Result, latency seconds from submit to completion)."""
        res = _CResult()
        lat = ctypes.c_double(0.0)
        _check(load_library().qnae_server_wait(self._h, int(ticket), int(timeout_ms), ctypes.byref(res),
                                               ctypes.byref(lat)))
        return Result(res.p_success, res.expected_cost, res.norm), float(lat.value)

    def cancel(self, ticket: int) -> bool:
        """True if the request will not complete (wait then raises
        QNAEError with code -6), False if it had already completed."""
        rc = load_library().qnae_server_cancel(self._h, int(ticket))
        _check(rc if rc < 0 else 0)
        return rc == 0

    def pool_in_use(self) -> int:
        v = ctypes.c_uint64(0)
        _check(load_library().qnae_server_pool_in_use(self._h, ctypes.byref(v)))
        return int(v.value)

    def stats(self) -> dict:
        v = [ctypes.c_uint64(0) for _ in range(6)]
        _check(load_library().qnae_server_stats(self._h, *[ctypes.byref(x) for x in v]))
        keys = ["completed", "ticks", "launches", "peak_pool_bytes", "queued", "active"]
        return {k: int(x.value) for k, x in zip(keys, v)}

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().qnae_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
