"""Python binding of ``libgde.so`` (the C ABI declared in ``include/gde.h``).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  PyTorch is used, when given, for device memory (``tensor.data_ptr()``)
and streams (``torch.cuda.current_stream().cuda_stream``).  If the library has
not been built this module raises at import time; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgde.so")

OK, INVALID_ARG, ISOLATED_SEED, CAPACITY, NOT_CONVERGED, OOM, BUSY, DEVICE, UNSUPPORTED = range(9)
PPR, KATZ, HK, SERIES = 0, 1, 2, 3
LOCAL_GD, LOCAL_CH, LOCAL_SOR = 0, 1, 2
F32, F64 = 0, 1
HOST_PTRS, DEVICE_PTRS, COPY, BORROW = 0x1, 0x2, 0x4, 0x8
KATZ_SUBTRACT_SEED, TRACE, RESULT_DEVICE = 0x1, 0x2, 0x4
SCATTER_BINNED, SCATTER_ATOMIC, DETERMINISTIC = 0x8, 0x10, 0x20
SYM_NORM = 0x40  # M = D^-1/2 A D^-1/2 (APPNP) for PPR, HK and series
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024  # GDE_NOALLOC_SCRATCH_BYTES of gde.h
STATUS_NAMES = ["OK", "INVALID_ARG", "ISOLATED_SEED", "CAPACITY", "NOT_CONVERGED", "OOM", "BUSY", "DEVICE",
                "UNSUPPORTED"]
KINDS = {"ppr": PPR, "katz": KATZ, "hk": HK, "series": SERIES}
METHODS = {"gd": LOCAL_GD, "localgd": LOCAL_GD, "ch": LOCAL_CH, "localch": LOCAL_CH, "sor": LOCAL_SOR,
           "localsor": LOCAL_SOR, "appr": LOCAL_SOR}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2410_21634_amd.build` (hipcc, gfx950)")

# PyTorch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch
# first makes libgde.so bind to that same runtime, so that torch streams and
# device pointers are valid in the library and only one runtime owns the GPU.
try:
    import torch  # noqa: F401
except ImportError:  # the library also works without torch (host buffers)
    torch = None


class Params(C.Structure):
    _fields_ = [("kind", C.c_int32), ("method", C.c_int32), ("value_type", C.c_int32), ("K", C.c_int32),
                ("alpha", C.c_double), ("beta", C.c_double), ("tau", C.c_double), ("eps", C.c_double),
                ("lambda_bound", C.c_double), ("c", C.POINTER(C.c_double)), ("max_iters", C.c_int32),
                ("flags", C.c_uint32), ("omega", C.c_double)]


class Seed(C.Structure):
    _fields_ = [("nnz", C.c_int32), ("idx", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class Result(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("idx", C.c_void_p), ("val", C.c_void_p), ("trace_capacity", C.c_int64),
                ("trace_size", C.c_void_p), ("trace_vol", C.c_void_p), ("trace_nodes_capacity", C.c_int64),
                ("trace_nodes", C.c_void_p), ("nnz", C.c_int64), ("residual_l1", C.c_double),
                ("residual_dinf", C.c_double), ("iters", C.c_int32), ("status", C.c_int32), ("ops", C.c_int64),
                ("pushes", C.c_int64), ("trace_len", C.c_int64), ("trace_nodes_len", C.c_int64)]


class ServerCfg(C.Structure):
    _fields_ = [("lanes_per_group", C.c_int32), ("max_groups", C.c_int32), ("iters_per_step", C.c_int32),
                ("queue_capacity", C.c_int32), ("value_type", C.c_int32), ("result_capacity", C.c_int32),
                ("max_insert_edges", C.c_int64)]


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("edges", C.c_int64), ("entries", C.c_int64),
                ("batch_launches", C.c_int64), ("batch_ms", C.c_double), ("batch_lane_edges", C.c_int64),
                ("batch_entries", C.c_int64), ("batch_push_launches", C.c_int64), ("batch_push_ms", C.c_double),
                ("batch_rows", C.c_int64), ("batch_row_vol", C.c_int64)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("iters", C.c_int32), ("nnz", C.c_int64),
                ("idx", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_float)), ("residual_l1", C.c_double),
                ("residual_dinf", C.c_double), ("submit_time_s", C.c_double), ("done_time_s", C.c_double)]


_lib = C.CDLL(LIB_PATH)
_vp, _i32, _i64 = C.c_void_p, C.c_int32, C.c_int64
_SIGS = {
    "gde_abi_version": ([], C.c_int),
    "gde_last_error": ([], C.c_char_p),
    "gde_ctx_create": ([C.c_int, C.POINTER(_vp)], C.c_int),
    "gde_ctx_destroy": ([_vp], C.c_int),
    "gde_graph_create": ([_vp, _i32, _i64, _vp, _vp, C.c_uint32, _vp, C.POINTER(_vp)], C.c_int),
    "gde_graph_destroy": ([_vp], C.c_int),
    "gde_graph_info": ([_vp, C.POINTER(_i32), C.POINTER(_i64)], C.c_int),
    "gde_graph_download": ([_vp, _vp, _vp], C.c_int),
    "gde_graph_lambda_max": ([_vp, _vp, C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), _vp],
                             C.c_int),
    "gde_validate": ([_i32, _i64, _vp, _vp, C.POINTER(Params), C.POINTER(Seed)], C.c_int),
    "gde_ctx_profile": ([_vp, C.c_int, C.POINTER(KernelProfile), C.c_int], C.c_int),
    "gde_solve": ([_vp, _vp, C.POINTER(Params), C.POINTER(Seed), C.POINTER(Result), _vp], C.c_int),
    "gde_solve_global": ([_vp, _vp, C.POINTER(Params), C.POINTER(Seed), C.POINTER(Result), _vp], C.c_int),
    "gde_solve_noalloc": ([_vp, C.POINTER(Params), C.POINTER(Seed), C.POINTER(Result), _vp], C.c_int),
    "gde_solve_noalloc_bytes": ([_vp, C.POINTER(Params), C.POINTER(Seed)], C.c_size_t),
    "gde_dyn_create": ([_vp, _vp, _i32, C.POINTER(_vp)], C.c_int),
    "gde_dyn_graph": ([_vp], _vp),
    "gde_dyn_add": ([_vp, C.POINTER(Params), C.POINTER(Seed), C.POINTER(_i32)], C.c_int),
    "gde_dyn_update": ([_vp, _i32, _vp, _vp, _i32, _vp, _vp], C.c_int),
    "gde_dyn_read": ([_vp, _i32, C.POINTER(Result), C.c_uint32], C.c_int),
    "gde_dyn_destroy": ([_vp], C.c_int),
    "gde_batch_tuned": ([_vp, _vp, _i32, _i32, _i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "gde_solve_batch": ([_vp, _vp, _i32, C.POINTER(Params), C.POINTER(Seed), C.POINTER(Result), C.c_char_p, _vp],
                        C.c_int),
    "gde_server_create": ([_vp, _vp, C.POINTER(ServerCfg), C.POINTER(_vp)], C.c_int),
    "gde_server_submit": ([_vp, C.POINTER(Params), C.POINTER(Seed), C.POINTER(C.c_uint64)], C.c_int),
    "gde_server_poll": ([_vp, C.POINTER(Completion), _i32, C.POINTER(_i32)], C.c_int),
    "gde_server_insert_edges": ([_vp, _i32, _vp, _vp], C.c_int),
    "gde_server_destroy": ([_vp], C.c_int),
}
for _name, (_args, _ret) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _ret
EXPORTED = tuple(_SIGS)


class GDEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


def last_error() -> str:
    return (_lib.gde_last_error() or b"").decode()


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise GDEError(rc, last_error())
    return rc


def abi_version() -> int:
    return _lib.gde_abi_version()


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def make_params(kind="ppr", method="gd", *, alpha=0.1, beta=0.0, tau=5.0, K=30, eps=1e-6, lambda_bound=0.0,
                value_type=F32, max_iters=10000, flags=0, c=None, omega=0.0) -> Params:
    """Query parameters.  ``c``: the K + 1 coefficients of kind "series" (K is
    taken from their count); the returned struct keeps the array alive."""
    k = KINDS[kind] if isinstance(kind, str) else int(kind)
    m = METHODS[method] if isinstance(method, str) else int(method)
    vt = {"f32": F32, "f64": F64}.get(value_type, value_type) if isinstance(value_type, str) else int(value_type)
    coef = None
    if c is not None:
        coef = np.ascontiguousarray(c, dtype=np.float64)
        K = len(coef) - 1
    p = Params(k, m, vt, int(K), float(alpha), float(beta), float(tau), float(eps), float(lambda_bound),
               coef.ctypes.data_as(C.POINTER(C.c_double)) if coef is not None else None, int(max_iters), int(flags),
               float(omega))
    p._coef = coef
    return p


class _SeedHolder:
    """Keeps the numpy arrays behind a Seed struct alive."""

    def __init__(self, idx, val=None):
        self.idx = np.ascontiguousarray(np.atleast_1d(idx), dtype=np.int32)
        if val is None:
            val = np.ones(len(self.idx))
        self.val = np.ascontiguousarray(np.atleast_1d(val), dtype=np.float64)
        self.seed = Seed(len(self.idx), self.idx.ctypes.data_as(C.POINTER(C.c_int32)),
                         self.val.ctypes.data_as(C.POINTER(C.c_double)))


def validate(row_ptr, col_idx, params: Params, seed_idx, seed_val=None) -> int:
    """Host-only validation (no device work)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    sh = _SeedHolder(seed_idx, seed_val)
    return _lib.gde_validate(len(rp) - 1, int(rp[-1]) if len(rp) else 0, rp.ctypes.data_as(_vp),
                             ci.ctypes.data_as(_vp), C.byref(params), C.byref(sh.seed))


class Context:
    def __init__(self, device: int = 0):
        h = _vp()
        _check(_lib.gde_ctx_create(int(device), C.byref(h)))
        self.handle = h
        self.device = device

    def batch_tuned(self, graph, kind, value_type, B):
        """(lanes, blocks_per_cu) chosen by the "auto" schedule for such batches, or None."""
        ln, bp = C.c_int32(0), C.c_int32(0)
        k = KINDS[kind] if isinstance(kind, str) else int(kind)
        rc = _lib.gde_batch_tuned(self.handle, graph.handle, k, int(value_type), int(B), C.byref(ln), C.byref(bp))
        return (ln.value, bp.value) if rc == OK else None

    def profile(self, enable: bool = True, reset: bool = True) -> dict:
        """Push-kernel event timing: returns the totals so far, then sets the mode."""
        kp = KernelProfile()
        _check(_lib.gde_ctx_profile(self.handle, int(enable), C.byref(kp), int(reset)))
        return {name: getattr(kp, name) for name, _ in KernelProfile._fields_}

    def close(self):
        if self.handle:
            _lib.gde_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _download_csr(handle):
    n, nnz = _i32(), _i64()
    _check(_lib.gde_graph_info(handle, C.byref(n), C.byref(nnz)))
    rp = np.zeros(n.value + 1, np.int32)
    ci = np.zeros(max(nnz.value, 1), np.int32)
    _check(_lib.gde_graph_download(handle, rp.ctypes.data_as(_vp), ci.ctypes.data_as(_vp)))
    return rp, ci[:nnz.value]


class Graph:
    """A CSR graph on the context's device.  numpy arrays are copied; torch
    device tensors are borrowed (they must stay alive with the graph)."""

    def __init__(self, ctx: Context, row_ptr, col_idx, stream=None):
        self.ctx = ctx
        h = _vp()
        if hasattr(row_ptr, "data_ptr") and getattr(row_ptr, "is_cuda", False):
            self._keep = (row_ptr, col_idx)
            n = row_ptr.numel() - 1
            nnz = col_idx.numel()
            rc = _lib.gde_graph_create(ctx.handle, n, nnz, _vp(row_ptr.data_ptr()), _vp(col_idx.data_ptr()),
                                       DEVICE_PTRS | BORROW, _stream_ptr(stream), C.byref(h))
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            ci = np.ascontiguousarray(col_idx, dtype=np.int32)
            n, nnz = len(rp) - 1, len(ci)
            rc = _lib.gde_graph_create(ctx.handle, n, nnz, rp.ctypes.data_as(_vp), ci.ctypes.data_as(_vp),
                                       HOST_PTRS | COPY, _stream_ptr(stream), C.byref(h))
        _check(rc)
        self.handle = h
        self.n = int(n)
        self.nnz = int(nnz)

    def csr(self):
        """(row_ptr, col_idx) copied to host numpy arrays."""
        return _download_csr(self.handle)

    def lambda_max(self, max_iters=500, rtol=1e-3, stream=None):
        lo, hi = C.c_double(), C.c_double()
        _check(_lib.gde_graph_lambda_max(self.ctx.handle, self.handle, int(max_iters), float(rtol), C.byref(lo),
                                         C.byref(hi), _stream_ptr(stream)))
        return lo.value, hi.value

    def close(self):
        if self.handle:
            _lib.gde_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SolveResult:
    idx: object
    val: object
    status: int
    residual_l1: float
    residual_dinf: float
    iters: int
    ops: int
    pushes: int
    trace_size: np.ndarray | None = None
    trace_vol: np.ndarray | None = None
    trace_nodes: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    def dense(self, n):
        x = np.zeros(n)
        idx = self.idx.cpu().numpy() if hasattr(self.idx, "cpu") else self.idx
        val = self.val.cpu().numpy() if hasattr(self.val, "cpu") else self.val
        x[idx] = val
        return x


def _result_struct(params, capacity, out_idx, out_val, trace_cap, nodes_cap):
    r = Result()
    r.capacity = capacity
    r.idx = out_idx
    r.val = out_val
    keep = []
    if params.flags & TRACE:
        ts = np.zeros(max(trace_cap, 1), np.int64)
        tv = np.zeros(max(trace_cap, 1), np.int64)
        tn = np.zeros(max(nodes_cap, 1), np.int32)
        r.trace_capacity = trace_cap
        r.trace_size = ts.ctypes.data
        r.trace_vol = tv.ctypes.data
        r.trace_nodes_capacity = nodes_cap
        r.trace_nodes = tn.ctypes.data if nodes_cap else None
        keep = [ts, tv, tn]
    return r, keep


def solve(ctx: Context, graph: Graph, params: Params, seed_idx, seed_val=None, *, capacity=None, out=None,
          trace_cap=4096, nodes_cap=0, stream=None, raise_on_error=True, _entry="gde_solve") -> SolveResult:
    """One query.  ``out``: optional (idx, val) torch device tensors (the result
    stays in HBM, GDE_RESULT_DEVICE); otherwise numpy host arrays are returned."""
    sh = _SeedHolder(seed_idx, seed_val)
    vdt = np.float64 if params.value_type == F64 else np.float32
    p = Params.from_buffer_copy(params)
    if out is not None:
        p.flags |= RESULT_DEVICE
        oi, ov = out
        cap = oi.numel() if capacity is None else capacity
        r, keep = _result_struct(p, cap, oi.data_ptr(), ov.data_ptr(), trace_cap, nodes_cap)
    else:
        cap = graph.n if capacity is None else capacity
        oi = np.zeros(max(cap, 1), np.int32)
        ov = np.zeros(max(cap, 1), vdt)
        r, keep = _result_struct(p, cap, oi.ctypes.data, ov.ctypes.data, trace_cap, nodes_cap)
    rc = getattr(_lib, _entry)(ctx.handle, graph.handle, C.byref(p), C.byref(sh.seed), C.byref(r),
                               _stream_ptr(stream))
    if raise_on_error:
        _check(rc, (OK, NOT_CONVERGED))
    nnz = int(r.nnz) if rc in (OK, NOT_CONVERGED) else 0
    res = SolveResult(oi[:nnz], ov[:nnz], rc, r.residual_l1, r.residual_dinf, r.iters, r.ops, r.pushes)
    res.extra["nnz_needed"] = int(r.nnz)
    if p.flags & TRACE:
        m = min(int(r.trace_len), trace_cap)
        res.trace_size = keep[0][:m].copy()
        res.trace_vol = keep[1][:m].copy()
        if nodes_cap:
            res.trace_nodes = keep[2][: min(int(r.trace_nodes_len), nodes_cap)].copy()
    return res


def solve_global(ctx: Context, graph: Graph, params: Params, seed_idx, seed_val=None, **kw) -> SolveResult:
    """gde_solve_global: GD or Chebyshev (params.method) over all nodes in every
    iteration; same arguments and result as ``solve``."""
    return solve(ctx, graph, params, seed_idx, seed_val, _entry="gde_solve_global", **kw)


def solve_noalloc(graph: Graph, params: Params, seed_idx, seed_val=None, *, out, capacity=None, stream=None,
                  raise_on_error=True) -> SolveResult:
    """gde_solve_noalloc: one query on the library's fixed device array (no
    allocation in the call).  ``out`` = (idx, val) torch device tensors."""
    sh = _SeedHolder(seed_idx, seed_val)
    p = Params.from_buffer_copy(params)
    p.flags |= RESULT_DEVICE
    oi, ov = out
    cap = oi.numel() if capacity is None else capacity
    r, _ = _result_struct(p, cap, oi.data_ptr(), ov.data_ptr(), 0, 0)
    rc = _lib.gde_solve_noalloc(graph.handle, C.byref(p), C.byref(sh.seed), C.byref(r), _stream_ptr(stream))
    if raise_on_error:
        _check(rc, (OK, NOT_CONVERGED))
    nnz = int(r.nnz) if rc in (OK, NOT_CONVERGED) else 0
    res = SolveResult(oi[:nnz], ov[:nnz], rc, r.residual_l1, r.residual_dinf, r.iters, r.ops, r.pushes)
    res.extra["nnz_needed"] = int(r.nnz)
    return res


def noalloc_bytes(graph: Graph, params: Params, seed_idx, seed_val=None) -> int:
    """Bytes of the fixed array gde_solve_noalloc would use for this query."""
    sh = _SeedHolder(seed_idx, seed_val)
    return int(_lib.gde_solve_noalloc_bytes(graph.handle, C.byref(params), C.byref(sh.seed)))


def _np_dtype(struct):
    """numpy view of a ctypes Structure (pointers as uint64), for vectorised filling."""
    conv = {C.c_int32: "<i4", C.c_uint32: "<u4", C.c_int64: "<i8", C.c_uint64: "<u8", C.c_double: "<f8"}
    names, formats, offsets = [], [], []
    for name, ctype in struct._fields_:
        names.append(name)
        formats.append(conv.get(ctype, "<u8"))
        offsets.append(getattr(struct, name).offset)
    return np.dtype({"names": names, "formats": formats, "offsets": offsets, "itemsize": C.sizeof(struct)})


_PAR_DT, _SEED_DT, _RES_DT = _np_dtype(Params), _np_dtype(Seed), _np_dtype(Result)


class BatchResults:
    """Results of one gde_solve_batch call.  Per-query fields are numpy arrays
    (status, nnz, iters, ops, pushes, residual_l1, residual_dinf); indexing or
    iterating gives SolveResult objects, built on first access."""

    def __init__(self, rv, idx_of, val_of, traces):
        self._rv = rv
        self._idx_of, self._val_of, self._traces = idx_of, val_of, traces
        self._cache = {}
        self.status = rv["status"].copy()
        self.nnz = rv["nnz"].copy()
        self.iters = rv["iters"].copy()
        self.ops = rv["ops"].copy()
        self.pushes = rv["pushes"].copy()
        self.residual_l1 = rv["residual_l1"].copy()
        self.residual_dinf = rv["residual_dinf"].copy()

    def __len__(self):
        return len(self.status)

    def __getitem__(self, i):
        if i < 0:
            i += len(self)
        if i not in self._cache:
            st = int(self.status[i])
            nnz = int(self.nnz[i]) if st in (OK, NOT_CONVERGED) else 0
            sr = SolveResult(self._idx_of(i, nnz), self._val_of(i, nnz), st, float(self.residual_l1[i]),
                             float(self.residual_dinf[i]), int(self.iters[i]), int(self.ops[i]), int(self.pushes[i]))
            sr.extra["nnz_needed"] = int(self.nnz[i])
            if i in self._traces:
                ts, tv, tn, tcap, ncap = self._traces[i]
                m = min(int(self._rv["trace_len"][i]), tcap)
                sr.trace_size = ts[:m].copy()
                sr.trace_vol = tv[:m].copy()
                if ncap:
                    sr.trace_nodes = tn[: min(int(self._rv["trace_nodes_len"][i]), ncap)].copy()
            self._cache[i] = sr
        return self._cache[i]

    def __iter__(self):
        return (self[i] for i in range(len(self)))


def params_array(params_list):
    """A ctypes ``Params * B`` array of the queries, for repeated solve_batch calls
    on the same queries (built once instead of per call)."""
    return (Params * len(params_list))(*params_list)


def solve_batch(ctx: Context, graph: Graph, params_list, seeds, *, capacity=None, schedule=None, stream=None,
                raise_on_error=True, trace_cap=4096, nodes_cap=0, out=None) -> BatchResults:
    """B queries in one call.  ``params_list``: a sequence of Params, or a ctypes
    ``Params * B`` array (copied, not changed).  ``seeds``: a list of (idx, val)
    pairs (val None = ones), or a 1-D integer array with one seed node per query
    (value 1).  ``out``: optional flat (idx, val) torch device tensors split evenly
    between the queries (the results stay in HBM).  Argument structs are filled
    vectorised."""
    B = len(params_list)
    P = (Params * B)()
    if isinstance(params_list, C.Array) and params_list._type_ is Params:
        C.memmove(P, params_list, C.sizeof(P))
    else:
        P = (Params * B)(*params_list)
    pv = np.frombuffer(P, dtype=_PAR_DT)
    if out is not None:
        pv["flags"] |= RESULT_DEVICE
    if isinstance(seeds, np.ndarray) and seeds.ndim == 1:  # one seed node per query
        if len(seeds) != B:
            raise ValueError("one seed node per query expected")
        lens = np.ones(B, np.int64)
        offs = np.arange(B, dtype=np.int64)
        cat_idx = np.ascontiguousarray(seeds, dtype=np.int32)
        cat_val = np.ones(B, np.float64)
    else:
        idx_l = [np.atleast_1d(np.asarray(i, dtype=np.int32)) for i, _ in seeds]
        lens = np.fromiter((len(x) for x in idx_l), dtype=np.int64, count=B)
        offs = np.zeros(B, np.int64)
        offs[1:] = np.cumsum(lens)[:-1]
        cat_idx = np.ascontiguousarray(np.concatenate(idx_l), dtype=np.int32)
        cat_val = np.ascontiguousarray(np.concatenate([np.ones(len(x)) if v is None else
                                                       np.atleast_1d(np.asarray(v, np.float64))
                                                       for x, (_, v) in zip(idx_l, seeds)]), dtype=np.float64)
    S = (Seed * B)()
    sv = np.frombuffer(S, dtype=_SEED_DT)
    sv["nnz"] = lens
    sv["idx"] = cat_idx.ctypes.data + 4 * offs
    sv["val"] = cat_val.ctypes.data + 8 * offs
    R = (Result * B)()
    rv = np.frombuffer(R, dtype=_RES_DT)
    vt = pv["value_type"].copy()
    if out is not None:
        cap = out[0].numel() // B if capacity is None else capacity
        esize = out[1].element_size()
        rv["capacity"] = cap
        rv["idx"] = out[0].data_ptr() + 4 * cap * np.arange(B, dtype=np.uint64)
        rv["val"] = out[1].data_ptr() + esize * cap * np.arange(B, dtype=np.uint64)

        def idx_of(i, nnz):
            return out[0][i * cap:i * cap + nnz]

        def val_of(i, nnz):
            return out[1][i * cap:i * cap + nnz]
        host = None
    else:
        cap = graph.n if capacity is None else capacity
        rv["capacity"] = cap
        if (vt == vt[0]).all():  # one block of host buffers
            vdt = np.float64 if vt[0] == F64 else np.float32
            host = (np.zeros((B, max(cap, 1)), np.int32), np.zeros((B, max(cap, 1)), vdt))
            rv["idx"] = host[0].ctypes.data + 4 * max(cap, 1) * np.arange(B, dtype=np.uint64)
            rv["val"] = host[1].ctypes.data + host[1].itemsize * max(cap, 1) * np.arange(B, dtype=np.uint64)
        else:  # mixed value types: one buffer pair per query
            host = ([np.zeros(max(cap, 1), np.int32) for _ in range(B)],
                    [np.zeros(max(cap, 1), np.float64 if t == F64 else np.float32) for t in vt])
            rv["idx"] = [a.ctypes.data for a in host[0]]
            rv["val"] = [a.ctypes.data for a in host[1]]

        def idx_of(i, nnz):
            return host[0][i][:nnz]

        def val_of(i, nnz):
            return host[1][i][:nnz]
    traces = {}
    for i in np.flatnonzero(pv["flags"] & TRACE):
        ts = np.zeros(max(trace_cap, 1), np.int64)
        tv = np.zeros(max(trace_cap, 1), np.int64)
        tn = np.zeros(max(nodes_cap, 1), np.int32)
        R[i].trace_capacity = trace_cap
        R[i].trace_size = ts.ctypes.data
        R[i].trace_vol = tv.ctypes.data
        R[i].trace_nodes_capacity = nodes_cap
        R[i].trace_nodes = tn.ctypes.data if nodes_cap else None
        traces[int(i)] = (ts, tv, tn, trace_cap, nodes_cap)
    sched = schedule.encode() if isinstance(schedule, str) else schedule
    rc = _lib.gde_solve_batch(ctx.handle, graph.handle, B, P, S, R, sched, _stream_ptr(stream))
    if raise_on_error:
        _check(rc, (OK, NOT_CONVERGED))
    res = BatchResults(rv, idx_of, val_of, traces)
    res._keep = (P, S, R, cat_idx, cat_val, host)
    return res


class _GraphView:
    """A graph handle owned by another object (the current version of a Dynamic)."""

    def __init__(self, ctx, handle, n):
        self.ctx, self.handle, self.n = ctx, handle, n

    def csr(self):
        """(row_ptr, col_idx) of this version copied to host numpy arrays (rows ascending)."""
        return _download_csr(self.handle)


class Dynamic:
    """Standing PPR / Katz LocalGD queries on a graph changed by edge batches
    (gde_dyn_*): the Insert / Delete corrections of Sec. 4 followed by a warm
    re-solve, with x and r resident on the device."""

    def __init__(self, ctx: Context, graph: Graph, value_type=F64):
        self.ctx, self.n, self.value_type = ctx, graph.n, value_type
        h = _vp()
        _check(_lib.gde_dyn_create(ctx.handle, graph.handle, int(value_type), C.byref(h)))
        self.handle = h

    @property
    def graph(self):
        """The current version, for gde_solve / gde_solve_global comparisons."""
        return _GraphView(self.ctx, _lib.gde_dyn_graph(self.handle), self.n)

    def add(self, params: Params, seed_idx, seed_val=None) -> int:
        sh = _SeedHolder(seed_idx, seed_val)
        q = _i32()
        _check(_lib.gde_dyn_add(self.handle, C.byref(params), C.byref(sh.seed), C.byref(q)))
        return int(q.value)

    def update(self, insert=(), delete=()):
        """insert / delete: edges as (k, 2) arrays or sequences of pairs."""
        ins = np.asarray(insert, dtype=np.int32).reshape(-1, 2)
        dels = np.asarray(delete, dtype=np.int32).reshape(-1, 2)
        iu, iv = np.ascontiguousarray(ins[:, 0]), np.ascontiguousarray(ins[:, 1])
        du, dv = np.ascontiguousarray(dels[:, 0]), np.ascontiguousarray(dels[:, 1])
        _check(_lib.gde_dyn_update(self.handle, len(iu), iu.ctypes.data_as(_vp), iv.ctypes.data_as(_vp), len(du),
                                   du.ctypes.data_as(_vp), dv.ctypes.data_as(_vp)))

    def read(self, qid: int) -> SolveResult:
        vdt = np.float64 if self.value_type == F64 else np.float32
        oi = np.zeros(max(self.n, 1), np.int32)
        ov = np.zeros(max(self.n, 1), vdt)
        r = Result()
        r.capacity = self.n
        r.idx = oi.ctypes.data
        r.val = ov.ctypes.data
        _check(_lib.gde_dyn_read(self.handle, int(qid), C.byref(r), 0), (OK, NOT_CONVERGED))
        nnz = int(r.nnz)
        return SolveResult(oi[:nnz].copy(), ov[:nnz].copy(), int(r.status), r.residual_l1, r.residual_dinf, r.iters,
                           r.ops, r.pushes)

    def close(self):
        if getattr(self, "handle", None):
            _lib.gde_dyn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (gde_server_*): submit queries, insert edges,
    poll completions.  Each completion is returned as a dict with its sparse x."""

    def __init__(self, ctx: Context, graph: Graph, lanes_per_group=16, max_groups=8, iters_per_step=4,
                 queue_capacity=1 << 20, result_capacity=None, max_insert_edges=0):
        cfg = ServerCfg(int(lanes_per_group), int(max_groups), int(iters_per_step), int(queue_capacity), F32,
                        int(result_capacity if result_capacity is not None else graph.n), int(max_insert_edges))
        h = _vp()
        _check(_lib.gde_server_create(ctx.handle, graph.handle, C.byref(cfg), C.byref(h)))
        self.handle = h
        self.ctx = ctx
        self._buf = (Completion * 4096)()

    def submit(self, params: Params, seed_idx, seed_val=None) -> int:
        sh = _SeedHolder(seed_idx, seed_val)
        t = C.c_uint64()
        _check(_lib.gde_server_submit(self.handle, C.byref(params), C.byref(sh.seed), C.byref(t)))
        return int(t.value)

    def insert_edges(self, u, v):
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        _check(_lib.gde_server_insert_edges(self.handle, len(u), u.ctypes.data_as(_vp), v.ctypes.data_as(_vp)))

    def poll(self) -> list:
        n = C.c_int32()
        _check(_lib.gde_server_poll(self.handle, self._buf, len(self._buf), C.byref(n)))
        out = []
        for i in range(n.value):
            c = self._buf[i]
            k = int(c.nnz)
            idx = np.ctypeslib.as_array(c.idx, shape=(k,)).copy() if k else np.zeros(0, np.int32)
            val = np.ctypeslib.as_array(c.val, shape=(k,)).copy() if k else np.zeros(0, np.float32)
            out.append(dict(ticket=int(c.ticket), status=int(c.status), iters=int(c.iters), idx=idx, val=val,
                            residual_l1=c.residual_l1, residual_dinf=c.residual_dinf,
                            submit_time_s=c.submit_time_s, done_time_s=c.done_time_s))
        return out

    def close(self):
        if self.handle:
            _lib.gde_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
