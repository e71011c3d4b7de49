"""ctypes binding of libspand (the C ABI declared in include/spand.h).

Argument marshalling only: every step of the factorization, apply and PCG
runs inside the library.  Device buffers are passed as integer addresses
(``tensor.data_ptr()`` of a torch tensor on the GPU works, as does any object
with a ``data_ptr()`` method); host arrays are numpy arrays.

The library must be built (``python -m paper_2007_00789_amd.build``); loading
raises OSError when it is missing, so no caller can fall back silently.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspand.so")

SPAND_OK = 0
FIRST_ORDER, SECOND_ORDER, SUPERFINE = 1, 2, 3
SCHEMES = {"FO": FIRST_ORDER, "SO": SECOND_ORDER, "SF": SUPERFINE}
FP64, FP32, FP32_BF16 = 0, 1, 2
PRECISIONS = {"FP64": FP64, "FP32": FP32, "FP32_BF16": FP32_BF16}

STATUS = {
    0: "SPAND_OK", -1: "SPAND_E_INVALID", -2: "SPAND_E_NOT_SYMMETRIC", -3: "SPAND_E_NOT_SPD",
    -4: "SPAND_E_NO_CONVERGENCE", -5: "SPAND_E_OOM", -6: "SPAND_E_HIP", -7: "SPAND_E_STATE",
    -8: "SPAND_E_LIMIT",
}


class Opts(C.Structure):
    _fields_ = [("depth", C.c_int32), ("skip", C.c_int32), ("eps", C.c_double),
                ("scheme", C.c_int32), ("precision", C.c_int32), ("debug_stop_step", C.c_int32),
                ("qr_group", C.c_int32), ("qr_list_cap", C.c_int32),
                ("qr_xcd_local", C.c_int32), ("qr_lds_cols", C.c_int32),
                ("prescale", C.c_int32), ("top_fp64_levels", C.c_int32),
                ("gemm_tile", C.c_int32), ("apply_graph", C.c_int32),
                ("qr_single_launch", C.c_int32), ("hbm_budget_bytes", C.c_int64)]


class FactorStats(C.Structure):
    _fields_ = [("nnz_L", C.c_int64), ("flops", C.c_double), ("factor_seconds", C.c_double),
                ("factor_bytes", C.c_int64), ("root_size", C.c_int32)]


class SpandError(RuntimeError):
    def __init__(self, status, message=""):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)

# name -> (restype, argtypes); mirrors include/spand.h
SIGNATURES = {
    "spand_default_opts": (None, [C.POINTER(Opts)]),
    "spand_status_string": (C.c_char_p, [C.c_int]),
    "spand_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "spand_destroy": (None, [_P]),
    "spand_last_error": (C.c_char_p, [_P]),
    "spand_analyze": (C.c_int, [_P, C.c_int64, _I64P, _I32P, _DP, C.c_int32, C.POINTER(Opts),
                                C.POINTER(_P)]),
    "spand_destroy_plan": (None, [_P]),
    "spand_analyze_batch": (C.c_int, [_P, C.c_int32, _I64P, C.POINTER(_I64P), C.POINTER(_I32P),
                                      C.POINTER(_DP), _I32P, _I32P, C.POINTER(Opts),
                                      C.POINTER(_P)]),
    "spand_plan_segments": (C.c_int, [_P, _I32P, _I64P]),
    "spand_plan_sizes": (C.c_int, [_P, _I64P, _I64P, _I32P]),
    "spand_plan_vertices": (C.c_int, [_P, _I32P, _I64P, _I64P]),
    "spand_plan_step_counts": (C.c_int, [_P, C.c_int32, _I32P, _I32P, _I64P, _I64P, _I32P]),
    "spand_plan_step_arrays": (C.c_int, [_P, C.c_int32, _I64P, _I64P, _I64P, _I32P, _I32P,
                                         _I64P, _I32P]),
    "spand_factor": (C.c_int, [_P, _P, _P, C.POINTER(Opts), C.POINTER(_P)]),
    "spand_destroy_factor": (None, [_P]),
    "spand_factor_batch": (C.c_int, [_P, C.c_int32, C.POINTER(_P), C.POINTER(_P), C.POINTER(Opts),
                                     C.POINTER(_P)]),
    "spand_pcg_batch": (C.c_int, [_P, C.c_int32, C.POINTER(_P), _I32P, C.POINTER(_P), C.POINTER(_P),
                                  C.c_double, C.c_int32, _I32P, _DP]),
    "spand_factor_ranks": (C.c_int, [_P, C.c_int32, _I32P, _I32P, _I32P, _I32P]),
    "spand_factor_info": (C.c_int, [_P, C.POINTER(FactorStats)]),
    "spand_apply": (C.c_int, [_P, _P, C.c_int32, _P, _P]),
    "spand_apply_noalloc": (C.c_int, [_P, _P, C.c_int32, _P, _P]),
    "spand_pcg": (C.c_int, [_P, _P, C.c_int32, _P, _P, C.c_double, C.c_int32, _I32P, _DP]),
    "spand_debug_block": (C.c_int, [_P, C.c_int32, C.c_int32, _DP, _I32P, _I32P]),
    "spand_server_create": (C.c_int, [C.c_int32, C.POINTER(Opts), C.c_double, C.c_int32,
                                      C.c_int64, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "spand_server_submit": (C.c_int, [_P, C.c_int64, C.c_int64, _I64P, _I32P, _DP, C.c_int32,
                                      _DP, C.c_int32, _DP, _I64P]),
    "spand_server_poll": (C.c_int, [_P, C.c_int64, C.c_int32, _I32P, _DP, _I32P, _DP, _DP]),
    "spand_server_stats": (C.c_int, [_P, _I64P]),
    "spand_server_error": (C.c_char_p, [_P]),
    "spand_server_destroy": (None, [_P]),
    "spand_gemm_tuning": (C.c_int, [_P, C.c_int32, _I32P, C.POINTER(C.c_float)]),
    "spand_profile": (C.c_int, [_P, C.c_int32]),
    "spand_profile_only": (C.c_int, [_P, C.c_char_p]),
    "spand_profile_entries": (C.c_int, [_P, _I32P]),
    "spand_profile_entry": (C.c_int, [_P, C.c_int32, C.c_char_p, C.c_int32, _DP, _I64P, _DP]),
}

_lib = None

# Live library objects, released in dependency order (factors, plans, servers,
# then contexts) before the interpreter tears down the HIP runtime, so that no
# device memory or stream is released from a finalizer running after it.
_live = {"factor": weakref.WeakSet(), "plan": weakref.WeakSet(), "server": weakref.WeakSet(),
         "ctx": weakref.WeakSet()}


def release_all():
    """Destroy every live factor, plan, server and context (also run at exit)."""
    for kind in ("factor", "plan", "server", "ctx"):
        for obj in list(_live[kind]):
            obj.close()


atexit.register(release_all)


def load(path: str = LIB_PATH):
    """Load libspand.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with python -m paper_2007_00789_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return C.c_void_p(x.data_ptr())
    return C.c_void_p(int(x))


def _np(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.POINTER(np.ctypeslib.as_ctypes_type(dtype)))


def make_opts(depth=0, skip=4, eps=1e-2, scheme="SO", precision=FP64, debug_stop_step=-1,
              qr_group=0, qr_list_cap=-1, qr_xcd_local=1, qr_lds_cols=0, prescale=0,
              top_fp64_levels=None, hbm_budget_bytes=0, apply_graph=0, gemm_tile=0,
              qr_single_launch=1) -> Opts:
    o = Opts()
    load().spand_default_opts(C.byref(o))
    o.depth = int(depth)
    o.skip = int(skip)
    o.eps = float(eps)
    o.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.debug_stop_step = int(debug_stop_step)
    o.qr_group = int(qr_group)
    o.qr_list_cap = int(qr_list_cap)
    o.qr_xcd_local = int(qr_xcd_local)
    o.qr_lds_cols = int(qr_lds_cols)
    o.prescale = int(prescale)
    if top_fp64_levels is not None:
        o.top_fp64_levels = int(top_fp64_levels)
    o.hbm_budget_bytes = int(hbm_budget_bytes)
    o.apply_graph = int(apply_graph)
    o.gemm_tile = int(gemm_tile)
    o.qr_single_launch = int(qr_single_launch)
    return o


class Context:
    """spand_create / spand_destroy.  stream: a hipStream_t address or None."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.spand_create(C.byref(h), int(device), _ptr(stream))
        if st != SPAND_OK:
            raise SpandError(st, "spand_create failed")
        self.h = h
        _live["ctx"].add(self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.spand_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, st):
        if st != SPAND_OK:
            raise SpandError(st, self.lib.spand_last_error(self.h).decode())

    def profile(self, enable: bool, only: str | None = None):
        """spand_profile: clear and start (or stop) per-kernel event timing;
        only: time the launches of this kernel name alone."""
        self._check(self.lib.spand_profile_only(self.h, only.encode() if only else None))
        self._check(self.lib.spand_profile(self.h, 1 if enable else 0))

    def gemm_tuning(self, precision: int = 0):
        """spand_gemm_tuning: {block size class: (tile, ms 64-tile, ms 128-tile)}
        or None before the first factorization in that precision."""
        tiles = np.zeros(4, np.int32)
        ms = np.zeros(8, np.float32)
        st = self.lib.spand_gemm_tuning(self.h, int(precision), tiles.ctypes.data_as(_I32P),
                                        ms.ctypes.data_as(C.POINTER(C.c_float)))
        if st != SPAND_OK:
            return None
        return {sz: (int(tiles[i]), float(ms[2 * i]), float(ms[2 * i + 1]))
                for i, sz in enumerate((64, 128, 256, 512))}

    def profile_entries(self) -> dict:
        """{kernel: (total_ms, launches, work)} accumulated since profile(True)."""
        n = C.c_int32()
        self._check(self.lib.spand_profile_entries(self.h, C.byref(n)))
        out = {}
        buf = C.create_string_buffer(64)
        for i in range(n.value):
            ms, calls, work = C.c_double(), C.c_int64(), C.c_double()
            self._check(self.lib.spand_profile_entry(self.h, i, buf, 64, C.byref(ms),
                                                     C.byref(calls), C.byref(work)))
            out[buf.value.decode()] = (ms.value, calls.value, work.value)
        return out

    def factor(self, plan: "Plan", vals, opts: Opts) -> "Factor":
        """spand_factor; vals: device buffer of nnz float64 values."""
        h = C.c_void_p()
        self._check(self.lib.spand_factor(self.h, plan.h, _ptr(vals), C.byref(opts), C.byref(h)))
        return Factor(self.lib, h, plan)

    def factor_batch(self, plans, vals, opts: Opts) -> list:
        """spand_factor_batch: plans from analyze() (one problem each) and one
        device buffer of CSR values per problem; returns one Factor handle per
        problem, all viewing the same batch factor."""
        cnt = len(plans)
        hp = (_P * cnt)(*[p.h for p in plans])
        vp = (_P * cnt)(*[_ptr(v) for v in vals])
        out = (_P * cnt)()
        self._check(self.lib.spand_factor_batch(self.h, cnt, hp, vp, C.byref(opts), out))
        return [Factor(self.lib, C.c_void_p(out[i]), plans[i]) for i in range(cnt)]

    def pcg_batch(self, facs, nrhs, bs, xs, tol=1e-10, maxit=1000, check=True):
        """spand_pcg_batch: per problem i, nrhs[i] columns of bs[i] / xs[i]
        (device buffers); returns per problem (iters, relres) arrays."""
        cnt = len(facs)
        nr = np.ascontiguousarray(nrhs, dtype=np.int32)
        tot = int(nr.sum())
        it = np.zeros(tot, dtype=np.int32)
        rr = np.zeros(tot, dtype=np.float64)
        fp = (_P * cnt)(*[f.h for f in facs])
        bp = (_P * cnt)(*[_ptr(b) for b in bs])
        xp = (_P * cnt)(*[_ptr(x) for x in xs])
        st = self.lib.spand_pcg_batch(self.h, cnt, fp, nr.ctypes.data_as(_I32P), bp, xp, float(tol),
                                      int(maxit), it.ctypes.data_as(_I32P), rr.ctypes.data_as(_DP))
        if check or st not in (SPAND_OK, -4):
            self._check(st)
        off = np.concatenate([[0], np.cumsum(nr)])
        return [(it[off[i]:off[i + 1]], rr[off[i]:off[i + 1]]) for i in range(cnt)]

    def apply(self, fac: "Factor", nrhs: int, x, y):
        """spand_apply: y = M x (device buffers, n x nrhs column-major)."""
        self._check(self.lib.spand_apply(self.h, fac.h, int(nrhs), _ptr(x), _ptr(y)))

    def apply_noalloc(self, fac: "Factor", nrhs: int, x, y):
        """spand_apply_noalloc: y = M x with the library's fixed device scratch
        (no device allocation)."""
        self._check(self.lib.spand_apply_noalloc(self.h, fac.h, int(nrhs), _ptr(x), _ptr(y)))

    def pcg(self, fac: "Factor", nrhs: int, b, x, tol=1e-10, maxit=1000, check=True):
        """spand_pcg; returns (iters, relres) numpy arrays of nrhs entries, or of
        (problems, nrhs) for a batch plan."""
        nseg = fac.plan.segments()[0]
        it = np.zeros(nseg * nrhs, dtype=np.int32)
        rr = np.zeros(nseg * nrhs, dtype=np.float64)
        st = self.lib.spand_pcg(self.h, fac.h, int(nrhs), _ptr(b), _ptr(x), float(tol), int(maxit),
                                it.ctypes.data_as(_I32P), rr.ctypes.data_as(_DP))
        if check or st not in (SPAND_OK, -4):
            self._check(st)
        if nseg > 1:
            return it.reshape(nseg, nrhs), rr.reshape(nseg, nrhs)
        return it, rr


def analyze(n, rowptr, colind, coords, opts: Opts, ctx: Context | None = None) -> "Plan":
    """spand_analyze (host work; ctx optional)."""
    lib = load()
    rp, rp_p = _np(rowptr, np.int64)
    ci, ci_p = _np(colind, np.int32)
    if coords is None:   # coordinate-free analysis
        xy, xy_p, dim = None, None, 0
    else:
        xy, xy_p = _np(coords, np.float64)
        dim = 1 if xy.ndim == 1 else xy.shape[1]
    h = C.c_void_p()
    st = lib.spand_analyze(ctx.h if ctx else None, int(n), rp_p, ci_p, xy_p, dim, C.byref(opts),
                           C.byref(h))
    if st != SPAND_OK:
        msg = lib.spand_last_error(ctx.h).decode() if ctx else ""
        raise SpandError(st, msg or "spand_analyze failed")
    return Plan(lib, h)


def analyze_batch(problems, opts: Opts, ctx: Context | None = None, depths=None) -> "Plan":
    """spand_analyze_batch: problems is a list of (n, rowptr, colind, coords);
    depths an optional list of per-problem depths (default: opts.depth rule)."""
    lib = load()
    keep = []
    cnt = len(problems)
    ns = np.ascontiguousarray([int(p[0]) for p in problems], dtype=np.int64)
    rp_arr = (_I64P * cnt)()
    ci_arr = (_I32P * cnt)()
    xy_arr = (_DP * cnt)()
    dims = np.zeros(cnt, dtype=np.int32)
    for i, (n, rowptr, colind, coords) in enumerate(problems):
        rp, rp_p = _np(rowptr, np.int64)
        ci, ci_p = _np(colind, np.int32)
        if coords is None:   # coordinate-free analysis of this problem
            xy, xy_p = None, None
            dims[i] = 0
        else:
            xy, xy_p = _np(coords, np.float64)
            dims[i] = 1 if xy.ndim == 1 else xy.shape[1]
        keep += [rp, ci, xy]
        rp_arr[i], ci_arr[i], xy_arr[i] = rp_p, ci_p, xy_p
    dp = None
    if depths is not None:
        dpa = np.ascontiguousarray(depths, dtype=np.int32)
        keep.append(dpa)
        dp = dpa.ctypes.data_as(_I32P)
    h = C.c_void_p()
    st = lib.spand_analyze_batch(ctx.h if ctx else None, cnt, ns.ctypes.data_as(_I64P), rp_arr,
                                 ci_arr, xy_arr, dims.ctypes.data_as(_I32P), dp, C.byref(opts),
                                 C.byref(h))
    if st != SPAND_OK:
        msg = lib.spand_last_error(ctx.h).decode() if ctx else ""
        raise SpandError(st, msg or "spand_analyze_batch failed")
    return Plan(lib, h)


class Plan:
    def __init__(self, lib, h):
        self.lib, self.h = lib, h
        _live["plan"].add(self)
        n, nnz, d = C.c_int64(), C.c_int64(), C.c_int32()
        lib.spand_plan_sizes(h, C.byref(n), C.byref(nnz), C.byref(d))
        self.n, self.nnz, self.depth = n.value, nnz.value, d.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.spand_destroy_plan(self.h)
            self.h = None

    __del__ = close

    def segments(self):
        """(count, offsets[count+1]) of the plan's independent problems."""
        cnt = C.c_int32()
        self.lib.spand_plan_segments(self.h, C.byref(cnt), None)
        off = np.zeros(cnt.value + 1, np.int64)
        self.lib.spand_plan_segments(self.h, C.byref(cnt), off.ctypes.data_as(_I64P))
        return cnt.value, off

    def vertices(self):
        lvl = np.zeros(self.n, np.int32)
        path = np.zeros(self.n, np.int64)
        perm = np.zeros(self.n, np.int64)
        self.lib.spand_plan_vertices(self.h, lvl.ctypes.data_as(_I32P), path.ctypes.data_as(_I64P),
                                     perm.ctypes.data_as(_I64P))
        return lvl, path, perm

    def step(self, l: int) -> dict:
        nc, ni, na, nch, sp = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64(), C.c_int32()
        st = self.lib.spand_plan_step_counts(self.h, l, C.byref(nc), C.byref(ni), C.byref(na),
                                             C.byref(nch), C.byref(sp))
        if st != SPAND_OK:
            raise SpandError(st, f"step {l}")
        nc, na, nch = nc.value, na.value, nch.value
        out = dict(n_clusters=nc, n_interior=ni.value, sparsified=bool(sp.value),
                   key_lvl=np.zeros(nc, np.int64), key_prefix=np.zeros(nc, np.int64),
                   adj_ptr=np.zeros(nc + 1, np.int64), adj=np.zeros(max(na, 1), np.int32),
                   colour=np.zeros(nc, np.int32), child_ptr=np.zeros(nc + 1, np.int64),
                   child=np.zeros(max(nch, 1), np.int32))
        self.lib.spand_plan_step_arrays(
            self.h, l, out["key_lvl"].ctypes.data_as(_I64P), out["key_prefix"].ctypes.data_as(_I64P),
            out["adj_ptr"].ctypes.data_as(_I64P), out["adj"].ctypes.data_as(_I32P),
            out["colour"].ctypes.data_as(_I32P), out["child_ptr"].ctypes.data_as(_I64P),
            out["child"].ctypes.data_as(_I32P))
        out["adj"] = out["adj"][:na]
        out["child"] = out["child"][:nch]
        return out


class Factor:
    def __init__(self, lib, h, plan):
        self.lib, self.h, self.plan = lib, h, plan
        _live["factor"].add(self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.spand_destroy_factor(self.h)
            self.h = None

    __del__ = close

    def ranks(self, l: int, n_clusters: int):
        arrs = [np.zeros(n_clusters, np.int32) for _ in range(4)]
        st = self.lib.spand_factor_ranks(self.h, l, *[a.ctypes.data_as(_I32P) for a in arrs])
        if st != SPAND_OK:
            raise SpandError(st, f"ranks of step {l}")
        return dict(zip(("a", "k", "r", "r2"), arrs))

    def info(self) -> dict:
        s = FactorStats()
        self.lib.spand_factor_info(self.h, C.byref(s))
        return {k: getattr(s, k) for k, _ in FactorStats._fields_}

    def debug_block(self, ci: int, cj: int) -> np.ndarray:
        r, c = C.c_int32(), C.c_int32()
        st = self.lib.spand_debug_block(self.h, ci, cj, None, C.byref(r), C.byref(c))
        if st != SPAND_OK:
            raise SpandError(st, "debug block")
        out = np.zeros((r.value, c.value), order="F")
        self.lib.spand_debug_block(self.h, ci, cj, out.ctypes.data_as(_DP), C.byref(r), C.byref(c))
        return out


class Server:
    """spand_server_*: a request loop on one device (continuous batching of
    new matrices, resident factors within a byte budget, one PCG per factor
    and slot).  submit() returns a request id; result() waits for it."""

    def __init__(self, opts: Opts, device: int = 0, tol=1e-10, maxit=1000,
                 max_bytes: int = 64 << 30, slots: int = 2, max_batch: int = 32):
        self.lib = load()
        self.h = C.c_void_p()
        st = self.lib.spand_server_create(int(device), C.byref(opts), float(tol), int(maxit),
                                          int(max_bytes), int(slots), int(max_batch),
                                          C.byref(self.h))
        if st != SPAND_OK:
            raise SpandError(st, "spand_server_create failed")
        self._n = {}
        _live["server"].add(self)

    def close(self):
        if self.h:
            self.lib.spand_server_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, key: int, b, matrix=None) -> int:
        """Queue a solve with the matrix of `key`; b is (n,) or (n, nrhs).
        matrix = (n, rowptr, colind, coords, vals) on the first request with a
        key (host arrays), None afterwards."""
        b = np.asarray(b, dtype=np.float64)
        nrhs = 1 if b.ndim == 1 else b.shape[1]
        bb, b_p = _np(b.reshape(b.shape[0], nrhs).T, np.float64)   # column-major
        rid = C.c_int64()
        if matrix is not None:
            n, rowptr, colind, coords, vals = matrix
            rp, rp_p = _np(rowptr, np.int64)
            ci, ci_p = _np(colind, np.int32)
            xy, xy_p = _np(coords, np.float64)
            va, va_p = _np(vals, np.float64)
            dim = 1 if xy.ndim == 1 else xy.shape[1]
            st = self.lib.spand_server_submit(self.h, int(key), int(n), rp_p, ci_p, xy_p, dim,
                                              va_p, nrhs, b_p, C.byref(rid))
            if st == SPAND_OK:
                self._n[int(key)] = int(n)
        else:
            st = self.lib.spand_server_submit(self.h, int(key), 0, None, None, None, 0, None,
                                              nrhs, b_p, C.byref(rid))
        if st != SPAND_OK:
            raise SpandError(st, "spand_server_submit failed")
        return rid.value, self._n[int(key)], nrhs

    def result(self, req, wait: bool = True, check=True):
        """(x (n, nrhs), iters, relres, latency seconds, status), or None if
        not done and wait is False."""
        rid, n, nrhs = req
        done = C.c_int32()
        x = np.zeros(n * nrhs, dtype=np.float64)
        it = np.zeros(nrhs, dtype=np.int32)
        rr = np.zeros(nrhs, dtype=np.float64)
        lat = C.c_double()
        st = self.lib.spand_server_poll(self.h, int(rid), int(bool(wait)), C.byref(done),
                                        x.ctypes.data_as(_DP), it.ctypes.data_as(_I32P),
                                        rr.ctypes.data_as(_DP), C.byref(lat))
        if st not in (SPAND_OK, -4) or (check and st != SPAND_OK):
            raise SpandError(st, self.lib.spand_server_error(self.h).decode())
        if not done.value:
            return None
        return x.reshape(nrhs, n).T, it, rr, lat.value, st

    def stats(self) -> dict:
        c = np.zeros(9, dtype=np.int64)
        self.lib.spand_server_stats(self.h, c.ctypes.data_as(_I64P))
        keys = ["resident_bytes", "resident_factors", "queued", "factor_batches",
                "factored_matrices", "pcg_calls"]
        out = {k: int(v) for k, v in zip(keys, c)}
        out.update(analyze_s=c[6] * 1e-6, factor_s=c[7] * 1e-6, pcg_s=c[8] * 1e-6)
        return out
