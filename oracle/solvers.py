"""ctypes wrapper of the FP64 C oracle (``gde_oracle.c``) -- TEST INFRASTRUCTURE.

Each function takes a CSR graph (``row_ptr``, ``col_idx`` as numpy arrays) and
returns plain numpy arrays / dicts.  Residuals are returned in the generic form
``r = b - Q x`` of Sec. 3.1, Eq. (4); ``residual_l1`` / ``residual_dinf`` are in
the reported scale (PPR divides by alpha, so they match the stop rule
``||D^-1 r||_inf < eps`` of Sec. 5 and App. B).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

PPR, KATZ, HK = 0, 1, 2
OK, NOT_CONVERGED = 0, 4

_p64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_p32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_pf = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with the plain Makefile next to this file."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["make", "-s", "-C", _HERE] + (["-B"] if force else [])
        subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = C.CDLL(_LIB_PATH)
            i64, i32, d, vp = C.c_int64, C.c_int32, C.c_double, C.c_void_p
            lib.oracle_localgd.argtypes = [i64, _p64, _p32, C.c_int, d, d, i32, _p32, _pf, i32, _pf, _pf,
                                           _p64, _pf, i64, vp, vp, vp, vp, i64, vp, vp]
            lib.oracle_localch.argtypes = [i64, _p64, _p32, C.c_int, d, d, d, i32, _p32, _pf, i32, _pf, _pf,
                                           _p64, _pf, i64, vp, vp, i64, vp, vp]
            lib.oracle_replay_gd_ch.argtypes = [i64, _p64, _p32, C.c_int, C.c_int, d, d, d, i32, _p32, _pf, i64,
                                                _p64, _p32, d, _pf, _pf, _p64, _pf, _p64]
            lib.oracle_push_fifo.argtypes = [i64, _p64, _p32, C.c_int, d, d, d, i32, _p32, _pf, i64, _pf, _pf,
                                             _p64, _pf]
            lib.oracle_hk.argtypes = [i64, _p64, _p32, d, i32, d, i32, _p32, _pf, _pf, _p64, _pf, _pf, i64, vp,
                                      vp, i64, vp, vp, i64, vp, vp, d, vp]
            lib.oracle_localgd_warm.argtypes = [i64, _p64, _p32, C.c_int, d, d, i32, _pf, _pf, _p64, _pf]
            lib.oracle_edge_events.argtypes = [i64, C.c_int, d, _pf, _pf, _p64, i64, _p32, _p32, C.c_int]
            lib.oracle_series.argtypes = [i64, _p64, _p32, i32, _pf, d, i32, _p32, _pf, _pf, _p64, _pf, _pf, i64,
                                          vp, vp, i64, vp, vp, i64, vp, vp, d, vp]
            lib.oracle_global.argtypes = [i64, _p64, _p32, C.c_int, C.c_int, d, d, d, i32, _p32, _pf, i32, _pf,
                                          _pf, _p64, _pf]
            for f in (lib.oracle_localgd, lib.oracle_localch, lib.oracle_replay_gd_ch, lib.oracle_push_fifo,
                      lib.oracle_hk, lib.oracle_localgd_warm, lib.oracle_edge_events, lib.oracle_global,
                      lib.oracle_series):
                f.restype = C.c_int
            _lib = lib
    return _lib


def _graph(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    return len(rp) - 1, rp, ci


def _seed(seed_idx, seed_val=None):
    idx = np.ascontiguousarray(np.atleast_1d(seed_idx), dtype=np.int32)
    if seed_val is None:
        seed_val = np.ones(len(idx))
    val = np.ascontiguousarray(np.atleast_1d(seed_val), dtype=np.float64)
    return len(idx), idx, val


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc):
    if rc not in (OK, NOT_CONVERGED):
        raise ValueError(f"oracle rejected the input (status {rc})")


def _nodes_result(buf, nlen, sizes):
    """(offsets, nodes) of the recorded S_t lists, or None if the buffer was short."""
    if buf is None or nlen[0] > len(buf) or len(sizes) == 0 and nlen[0] > 0:
        return None
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    return off, buf[: nlen[0]].copy()


def localgd(row_ptr, col_idx, kind, param, eps, seed_idx, seed_val=None, max_iters=100000, trace_cap=0,
            nodes_cap=0):
    """LocalGD, Eq. (9): x <- x + r_S, r <- r - Q r_S (synchronous over S_t)."""
    lib = _load()
    n, rp, ci = _graph(row_ptr, col_idx)
    k, idx, val = _seed(seed_idx, seed_val)
    x, r = np.zeros(n), np.zeros(n)
    stats, norms = np.zeros(4, np.int64), np.zeros(2)
    tr = [np.zeros(trace_cap, np.int64), np.zeros(trace_cap, np.int64), np.zeros(trace_cap), np.zeros(trace_cap)]
    nb = np.zeros(nodes_cap, np.int32) if nodes_cap else None
    nlen = np.zeros(1, np.int64)
    rc = lib.oracle_localgd(n, rp, ci, kind, param, eps, k, idx, val, max_iters, x, r, stats, norms, trace_cap,
                            *(_ptr(a) for a in tr), nodes_cap, _ptr(nb), _ptr(nlen))
    _check(rc)
    T = int(stats[0])
    m = min(T, trace_cap)
    out = dict(x=x, r=r, status=rc, iters=T, ops=int(stats[1]), pushes=int(stats[2]), residual_l1=norms[0],
               residual_dinf=norms[1], trace_size=tr[0][:m], trace_vol=tr[1][:m], trace_rs_l1=tr[2][:m],
               trace_r_l1=tr[3][:m])
    if nodes_cap and m == T:
        out["trace_nodes"] = _nodes_result(nb, nlen, tr[0][:m])
    return out


def localch(row_ptr, col_idx, kind, param, eps, seed_idx, seed_val=None, lam=0.0, max_iters=100000, trace_cap=0,
            nodes_cap=0):
    """LocalCH (Sec. 3.3; App. B implementation details), Chebyshev update restricted to S_t."""
    lib = _load()
    n, rp, ci = _graph(row_ptr, col_idx)
    k, idx, val = _seed(seed_idx, seed_val)
    x, r = np.zeros(n), np.zeros(n)
    stats, norms = np.zeros(4, np.int64), np.zeros(2)
    ts, tv = np.zeros(trace_cap, np.int64), np.zeros(trace_cap, np.int64)
    nb = np.zeros(nodes_cap, np.int32) if nodes_cap else None
    nlen = np.zeros(1, np.int64)
    rc = lib.oracle_localch(n, rp, ci, kind, param, lam, eps, k, idx, val, max_iters, x, r, stats, norms,
                            trace_cap, _ptr(ts), _ptr(tv), nodes_cap, _ptr(nb), _ptr(nlen))
    _check(rc)
    T = int(stats[0])
    m = min(T, trace_cap)
    out = dict(x=x, r=r, status=rc, iters=T, ops=int(stats[1]), pushes=int(stats[2]), residual_l1=norms[0],
               residual_dinf=norms[1], trace_size=ts[:m], trace_vol=tv[:m])
    if nodes_cap and m == T:
        out["trace_nodes"] = _nodes_result(nb, nlen, ts[:m])
    return out


def push_fifo(row_ptr, col_idx, kind, param, eps, seed_idx, seed_val=None, omega=1.0, max_pops=10**12):
    """FIFO push: APPR (Algorithm 1) / AKatz for omega = 1, LocalSOR (Eq. (7)) otherwise."""
    lib = _load()
    n, rp, ci = _graph(row_ptr, col_idx)
    k, idx, val = _seed(seed_idx, seed_val)
    x, r = np.zeros(n), np.zeros(n)
    stats, norms = np.zeros(4, np.int64), np.zeros(2)
    rc = lib.oracle_push_fifo(n, rp, ci, kind, param, eps, omega, k, idx, val, max_pops, x, r, stats, norms)
    _check(rc)
    return dict(x=x, r=r, status=rc, pops=int(stats[0]), ops=int(stats[1]), epochs=int(stats[2]),
                residual_l1=norms[0], residual_dinf=norms[1])


def hk(row_ptr, col_idx, tau, K, eps, seed_idx, seed_val=None, trace_cap=64, replay=None, kappa=0.0, nodes_cap=0):
    """Heat-kernel level push on the Kronecker system (AHK, Sec. 2).

    ``replay``: optional ``(offsets, nodes)`` of recorded per-level active sets;
    the run then uses them and grades each decision (flips, violations)."""
    lib = _load()
    n, rp, ci = _graph(row_ptr, col_idx)
    k, idx, val = _seed(seed_idx, seed_val)
    x = np.zeros(n)
    stats, norms, psi = np.zeros(4, np.int64), np.zeros(2), np.zeros(K + 1)
    ts, tv = np.zeros(trace_cap, np.int64), np.zeros(trace_cap, np.int64)
    fv = np.zeros(2, np.int64)
    if replay is not None:
        off = np.ascontiguousarray(replay[0], dtype=np.int64)
        nodes = np.ascontiguousarray(replay[1], dtype=np.int32)
        if len(nodes) == 0:
            nodes = np.zeros(1, np.int32)
        T_rec = len(off) - 1
    else:
        off = nodes = None
        T_rec = 0
    nb = np.zeros(nodes_cap, np.int32) if nodes_cap else None
    nlen = np.zeros(1, np.int64)
    rc = lib.oracle_hk(n, rp, ci, tau, K, eps, k, idx, val, x, stats, norms, psi, trace_cap, _ptr(ts), _ptr(tv),
                       nodes_cap, _ptr(nb), _ptr(nlen), T_rec, _ptr(off), _ptr(nodes), kappa, _ptr(fv))
    _check(rc)
    T = int(stats[0])
    m = min(T, trace_cap)
    out = dict(x=x, status=rc, iters=T, ops=int(stats[1]), pushes=int(stats[2]), residual_l1=norms[0],
               residual_dinf=norms[1], psi=psi, trace_size=ts[:m], trace_vol=tv[:m], flips=int(fv[0]),
               violations=int(fv[1]))
    if nodes_cap and m == T:
        out["trace_nodes"] = _nodes_result(nb, nlen, ts[:m])
    return out


def series(row_ptr, col_idx, c, eps, seed_idx, seed_val=None, trace_cap=64, replay=None, kappa=0.0, nodes_cap=0):
    """Level push of f_K = sum_k c_k (A D^-1)^k s for positive coefficients c
    (length K + 1): the heat-kernel push with general level ratios (Eq. (1),
    Table 1).  Arguments and result as ``hk``."""
    lib = _load()
    n, rp, ci = _graph(row_ptr, col_idx)
    k, idx, val = _seed(seed_idx, seed_val)
    cc = np.ascontiguousarray(c, dtype=np.float64)
    K = len(cc) - 1
    x = np.zeros(n)
    stats, norms, psi = np.zeros(4, np.int64), np.zeros(2), np.zeros(K + 1)
    ts, tv = np.zeros(trace_cap, np.int64), np.zeros(trace_cap, np.int64)
    fv = np.zeros(2, np.int64)
    if replay is not None:
        off = np.ascontiguousarray(replay[0], dtype=np.int64)
        nodes = np.ascontiguousarray(replay[1], dtype=np.int32)
        if len(nodes) == 0:
            nodes = np.zeros(1, np.int32)
        T_rec = len(off) - 1
    else:
        off = nodes = None
        T_rec = 0
    nb = np.zeros(nodes_cap, np.int32) if nodes_cap else None
    nlen = np.zeros(1, np.int64)
    rc = lib.oracle_series(n, rp, ci, K, cc, eps, k, idx, val, x, stats, norms, psi, trace_cap, _ptr(ts), _ptr(tv),
                           nodes_cap, _ptr(nb), _ptr(nlen), T_rec, _ptr(off), _ptr(nodes), kappa, _ptr(fv))
    _check(rc)
    T = int(stats[0])
    m = min(T, trace_cap)
    out = dict(x=x, status=rc, iters=T, ops=int(stats[1]), pushes=int(stats[2]), residual_l1=norms[0],
               residual_dinf=norms[1], psi=psi, trace_size=ts[:m], trace_vol=tv[:m], flips=int(fv[0]),
               violations=int(fv[1]))
    if nodes_cap and m == T:
        out["trace_nodes"] = _nodes_result(nb, nlen, ts[:m])
    return out


def symmetric(fn, row_ptr, col_idx, *args, seed_idx, seed_val=None, **kw):
    """``fn`` (localgd, localch, hk or series) with the propagation matrix
    D^-1/2 A D^-1/2 of Table 1 (APPNP) in place of A D^-1.  Since
    (D^-1/2 A D^-1/2)^k = D^-1/2 (A D^-1)^k D^1/2, the series equals
    D^-1/2 f(D^1/2 s) with f the A D^-1 form (the symmetrisation of Sec. 3.3):
    ``fn`` runs on the source D^1/2 s, then x is scaled by D^-1/2.  ``args`` are
    fn's arguments before the seed; the stop rule, counts and residuals stay
    those of the A D^-1 form."""
    d = np.diff(np.asarray(row_ptr, dtype=np.int64)).astype(np.float64)
    idx = np.atleast_1d(np.asarray(seed_idx, dtype=np.int32))
    val = np.ones(len(idx)) if seed_val is None else np.asarray(seed_val, dtype=np.float64)
    out = fn(row_ptr, col_idx, *args, idx, val * np.sqrt(d[idx]), **kw)
    x = out["x"]
    out["x"] = np.where(d > 0, x / np.sqrt(np.where(d > 0, d, 1.0)), 0.0)
    return out


def replay_gd_ch(row_ptr, col_idx, method, kind, param, eps, seed_idx, seed_val, offsets, nodes, kappa, lam=0.0):
    """Re-run LocalGD (method 0) / LocalCH (method 1) in FP64 on recorded active sets.

    Every decision of the recording is graded against the band
    ``[theta (1-kappa), theta (1+kappa))`` of the FP64 residual."""
    lib = _load()
    n, rp, ci = _graph(row_ptr, col_idx)
    k, idx, val = _seed(seed_idx, seed_val)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nd = np.ascontiguousarray(nodes, dtype=np.int32)
    if len(nd) == 0:
        nd = np.zeros(1, np.int32)
    x, r = np.zeros(n), np.zeros(n)
    stats, norms, fv = np.zeros(4, np.int64), np.zeros(2), np.zeros(2, np.int64)
    rc = lib.oracle_replay_gd_ch(n, rp, ci, method, kind, param, lam, eps, k, idx, val, len(off) - 1, off, nd,
                                 kappa, x, r, stats, norms, fv)
    _check(rc)
    return dict(x=x, r=r, status=rc, iters=int(stats[0]), ops=int(stats[1]), pushes=int(stats[2]),
                residual_l1=norms[0], residual_dinf=norms[1], flips=int(fv[0]), violations=int(fv[1]))


def localgd_warm(row_ptr, col_idx, kind, param, eps, x, r, max_iters=100000):
    """LocalGD continued from a given (x, r) (no forced S_0, signed residuals): the
    re-solve after the edge-event corrections of the dynamic algorithms (Sec. 4).
    Returns new arrays; the inputs are not modified."""
    lib = _load()
    n, rp, ci = _graph(row_ptr, col_idx)
    x = np.array(x, dtype=np.float64, copy=True)
    r = np.array(r, dtype=np.float64, copy=True)
    stats, norms = np.zeros(4, np.int64), np.zeros(2)
    rc = lib.oracle_localgd_warm(n, rp, ci, kind, param, eps, max_iters, x, r, stats, norms)
    _check(rc)
    return dict(x=x, r=r, status=rc, iters=int(stats[0]), ops=int(stats[1]), pushes=int(stats[2]),
                residual_l1=norms[0], residual_dinf=norms[1])


def edge_events(kind, param, x, r, deg, u, v, sign):
    """Insert (sign=+1) or delete (sign=-1) the undirected edges (u[i], v[i]) in
    (x, r) (generic form r = b - Q x), each as the directed events u->v then v->u
    (the Insert / Delete procedures of Sec. 4; Katz derived).  ``deg`` holds the
    degrees before the batch.  Returns new (x, r, deg)."""
    lib = _load()
    x = np.array(x, dtype=np.float64, copy=True)
    r = np.array(r, dtype=np.float64, copy=True)
    deg = np.array(deg, dtype=np.int64, copy=True)
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    rc = lib.oracle_edge_events(len(x), kind, param, x, r, deg, len(u), u, v, int(sign))
    if rc != OK:
        raise ValueError(f"oracle rejected the edge events (status {rc})")
    return x, r, deg


def global_gd_ch(row_ptr, col_idx, method, kind, param, eps, seed_idx, seed_val=None, lam=0.0, max_iters=100000):
    """The standard counterparts of LocalGD / LocalCH (method 0 / 1): the same
    update with S_t = V in every iteration, until no node is active (Table 2,
    the eps sweep of Sec. 5).  ops = T * nnz, pushes = T * n."""
    lib = _load()
    n, rp, ci = _graph(row_ptr, col_idx)
    k, idx, val = _seed(seed_idx, seed_val)
    x, r = np.zeros(n), np.zeros(n)
    stats, norms = np.zeros(4, np.int64), np.zeros(2)
    rc = lib.oracle_global(n, rp, ci, method, kind, param, lam, eps, k, idx, val, max_iters, x, r, stats, norms)
    _check(rc)
    return dict(x=x, r=r, status=rc, iters=int(stats[0]), ops=int(stats[1]), pushes=int(stats[2]),
                residual_l1=norms[0], residual_dinf=norms[1])
