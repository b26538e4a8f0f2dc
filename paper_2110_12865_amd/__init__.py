"""Python binding of libspchol (MI355X sparse Cholesky on a fixed pattern).

Argument marshalling only: every numeric step runs in the library's HIP
kernels; PyTorch provides device memory and the current stream.  The
names follow the C ABI in include/spchol.h:

    plan = analyze(colptr, rowind, perm)        # host, once per pattern
    num  = plan.numeric(batch, "f64")           # device storage
    num.factor(values)                          # values: cuda f64 [batch, nnzA]
    num.solve(b)                                # b: cuda f64 [batch, nrhs, n], in place

    group = analyze_group([(colptr, rowind, perm), ...])   # uneven batch:
    # one block-diagonal plan over several patterns (see sc_analyze_group)

Importing this package fails loudly if the library has not been built
(``python paper_2110_12865_amd/build.py``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspchol.so")

SC_OK, SC_EINVAL, SC_EPATTERN, SC_ENOMEM, SC_EDEVICE, SC_ENOTSPD, SC_ENOCONV, SC_ESCRATCH = \
    0, -1, -2, -3, -4, -5, -6, -7
SC_NOALLOC_SCRATCH_BYTES = 32 << 20
SC_F64, SC_F32 = 0, 1
SC_REFINE_CLASSICAL, SC_REFINE_PCG = 0, 1
SC_ORDER_NATURAL, SC_ORDER_GIVEN, SC_ORDER_ND = 0, 1, 2
_ORDERINGS = {"natural": SC_ORDER_NATURAL, "given": SC_ORDER_GIVEN, "nd": SC_ORDER_ND}
_METHODS = {"classical": SC_REFINE_CLASSICAL, "pcg": SC_REFINE_PCG}
_DTYPES = {"f64": SC_F64, "f32": SC_F32}

# names exported by the library, in the order of the header
EXPORTS = [
    "sc_status_string", "sc_options_default", "sc_analyze", "sc_analyze_group",
    "sc_plan_info", "sc_plan_export_blocks", "sc_plan_export_symbolic",
    "sc_plan_export_supernodes", "sc_plan_destroy", "sc_numeric_create", "sc_numeric_destroy",
    "sc_factor", "sc_factor_info", "sc_solve", "sc_solve_noalloc", "sc_refine_solve",
    "sc_numeric_get_columns", "sc_numeric_get_block", "sc_numeric_profile",
    "sc_numeric_profile_read",
    "sc_step_graph_create", "sc_step_graph_launch", "sc_step_graph_stats", "sc_step_graph_destroy",
    "sc_autotune", "sc_adjoint", "sc_autotune_group",
]


class SpcholError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, status_string(status), status))


class Options(ctypes.Structure):
    _fields_ = [("relax", ctypes.c_int32), ("relax_cols", ctypes.c_int32),
                ("relax_zeros", ctypes.c_double), ("small_front", ctypes.c_int32),
                ("soa_min_batch", ctypes.c_int32), ("soa_seg_max", ctypes.c_int32),
                ("soa_subtree_min", ctypes.c_int32),
                ("ordering", ctypes.c_int32), ("panel_inverse", ctypes.c_int32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("opt", Options), ("factor_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("score", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


class RefineStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("clause", ctypes.c_int32),
                ("relres", ctypes.c_double), ("rnorm", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("xnorm", ctypes.c_double)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnzA", ctypes.c_int64),
                ("nnzL", ctypes.c_int64), ("nfund", ctypes.c_int64),
                ("nsuper", ctypes.c_int64), ("nlevels", ctypes.c_int64),
                ("L_store", ctypes.c_int64), ("U_store", ctypes.c_int64),
                ("max_front", ctypes.c_int64), ("max_width", ctypes.c_int64),
                ("flops", ctypes.c_double), ("etree_height", ctypes.c_int64),
                ("nblocks", ctypes.c_int64)]


def _load():
    # torch ships its own HIP runtime with the same soname as the system
    # one; load it first so that this library and torch share one runtime
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libspchol.so is not built (%s); run "
                          "`python paper_2110_12865_amd/build.py`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "sc_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "sc_options_default": ([P], ctypes.c_int),
        "sc_analyze": ([I64, P, P, P, P, P], ctypes.c_int),
        "sc_analyze_group": ([I32, P, P, P, P, P, P], ctypes.c_int),
        "sc_plan_info": ([P, P], ctypes.c_int),
        "sc_plan_export_blocks": ([P, P, P], ctypes.c_int),
        "sc_plan_export_symbolic": ([P, P, P, P, P], ctypes.c_int),
        "sc_plan_export_supernodes": ([P, P, P, P, P, P], ctypes.c_int),
        "sc_plan_destroy": ([P], None),
        "sc_numeric_create": ([P, I32, ctypes.c_int, P], ctypes.c_int),
        "sc_numeric_destroy": ([P], None),
        "sc_factor": ([P, P, P, I64, P], ctypes.c_int),
        "sc_factor_info": ([P, P, P], ctypes.c_int),
        "sc_solve": ([P, P, P, I32, I64, P], ctypes.c_int),
        "sc_solve_noalloc": ([P, P, P, I32, I64, P], ctypes.c_int),
        "sc_refine_solve": ([P, P, P, I64, P, P, I32, I64, ctypes.c_double, I32, I32, P, P],
                            ctypes.c_int),
        "sc_numeric_get_columns": ([P, P, I32, I64, P, P], ctypes.c_int),
        "sc_numeric_get_block": ([P, P, I32, I32, P], ctypes.c_int),
        "sc_numeric_profile": ([P, I32], ctypes.c_int),
        "sc_numeric_profile_read": ([P, I32, P, P], ctypes.c_int),
        "sc_step_graph_create": ([P, P, P, I64, P, P, I32, I64, ctypes.c_double, I32, I32, P],
                                 ctypes.c_int),
        "sc_step_graph_launch": ([P, P], ctypes.c_int),
        "sc_step_graph_stats": ([P, P, P], ctypes.c_int),
        "sc_step_graph_destroy": ([P], None),
        "sc_autotune": ([I64, P, P, P, P, I64, I32, ctypes.c_int, P, I32, I64, ctypes.c_double, P,
                         P, I32, P, P], ctypes.c_int),
        "sc_adjoint": ([P, P, P, P, P, I64, P, I32, I64, P], ctypes.c_int),
        "sc_autotune_group": ([I32, P, P, P, P, P, I64, I32, ctypes.c_int, P, I32, I64,
                               ctypes.c_double, P, P, I32, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def status_string(s: int) -> str:
    return _lib.sc_status_string(int(s)).decode()


def _check(st: int, what: str):
    if st != SC_OK:
        raise SpcholError(st, what)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def default_options(**kw) -> Options:
    o = Options()
    _check(_lib.sc_options_default(ctypes.byref(o)), "sc_options_default")
    for k, v in kw.items():
        if k == "ordering" and isinstance(v, str):
            v = _ORDERINGS[v]
        setattr(o, k, v)
    return o


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype_name: str):
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != getattr(torch, dtype_name):
        raise ValueError("expected %s, got %s" % (dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Symbolic analysis of one pattern (see sc_analyze)."""

    def __init__(self, n, colptr, rowind, perm=None, options: Optional[Options] = None):
        self.n = int(n)
        colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        rowind = np.ascontiguousarray(rowind, dtype=np.int32)
        perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(_lib.sc_analyze(self.n, _ptr(colptr), _ptr(rowind), _ptr(perm),
                               None if options is None else ctypes.byref(options),
                               ctypes.byref(h)), "sc_analyze")
        self._h = h
        self.nblocks = 1

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:  # (the module may be torn down first at exit)
            _lib.sc_plan_destroy(h)
            self._h = None

    def info(self) -> dict:
        st = PlanStats()
        _check(_lib.sc_plan_info(self._h, ctypes.byref(st)), "sc_plan_info")
        return {k: getattr(st, k) for k, _ in PlanStats._fields_}

    def export_symbolic(self):
        inf = self.info()
        n, nnzL = inf["n"], inf["nnzL"]
        perm = np.empty(n, np.int32)
        parent = np.empty(n, np.int32)
        Lcolptr = np.empty(n + 1, np.int64)
        Lrowind = np.empty(nnzL, np.int32)
        _check(_lib.sc_plan_export_symbolic(self._h, _ptr(perm), _ptr(parent),
                                            _ptr(Lcolptr), _ptr(Lrowind)),
               "sc_plan_export_symbolic")
        return perm, parent, Lcolptr, Lrowind

    def export_supernodes(self):
        """(first, parent, level, rowptr, rows) of the amalgamated supernodes."""
        ns = self.info()["nsuper"]
        first = np.empty(ns + 1, np.int32)
        parent = np.empty(ns, np.int32)
        level = np.empty(ns, np.int32)
        rowptr = np.empty(ns + 1, np.int64)
        _check(_lib.sc_plan_export_supernodes(self._h, _ptr(first), _ptr(parent), _ptr(level),
                                              _ptr(rowptr), None), "sc_plan_export_supernodes")
        rows = np.empty(int(rowptr[-1]), np.int32)
        _check(_lib.sc_plan_export_supernodes(self._h, None, None, None, None, _ptr(rows)),
               "sc_plan_export_supernodes")
        return first, parent, level, rowptr, rows

    def export_blocks(self):
        """(col0, val0): column and value offsets of the blocks, nblocks + 1 each."""
        col0 = np.empty(self.nblocks + 1, np.int64)
        val0 = np.empty(self.nblocks + 1, np.int64)
        _check(_lib.sc_plan_export_blocks(self._h, _ptr(col0), _ptr(val0)),
               "sc_plan_export_blocks")
        return col0, val0

    def numeric(self, batch: int = 1, dtype: str = "f64") -> "Numeric":
        return Numeric(self, batch, dtype)


class GroupPlan(Plan):
    """One plan over several patterns, the block-diagonal matrix of all of
    them (see sc_analyze_group).  Values and vectors of the group are the
    concatenations of the patterns' values and vectors (export_blocks gives
    the offsets)."""

    def __init__(self, patterns, options: Optional[Options] = None):
        npat = len(patterns)
        if npat < 1:
            raise ValueError("no patterns")
        cps = [np.ascontiguousarray(p[0], dtype=np.int64) for p in patterns]
        ris = [np.ascontiguousarray(p[1], dtype=np.int32) for p in patterns]
        pms = [None if len(p) < 3 or p[2] is None else np.ascontiguousarray(p[2], dtype=np.int32)
               for p in patterns]
        ns = np.array([len(c) - 1 for c in cps], np.int64)
        VP = ctypes.c_void_p * npat
        cpa = VP(*[c.ctypes.data for c in cps])
        ria = VP(*[r.ctypes.data for r in ris])
        pma = VP(*[0 if q is None else q.ctypes.data for q in pms])
        h = ctypes.c_void_p()
        _check(_lib.sc_analyze_group(npat, _ptr(ns), cpa, ria, pma,
                                     None if options is None else ctypes.byref(options),
                                     ctypes.byref(h)), "sc_analyze_group")
        self._h = h
        self.n = int(ns.sum())
        self.nblocks = npat


def analyze(colptr, rowind, perm=None, n=None, **opts) -> Plan:
    n = len(colptr) - 1 if n is None else n
    return Plan(n, colptr, rowind, perm, default_options(**opts) if opts else None)


def autotune(colptr, rowind, perm, values, b, dtype: str = "f64",
             solves_per_factor: float = 1.0, stream=None):
    """Pick analysis/kernel options for this workload by timing candidates
    (sc_autotune).  values: device float64 [batch, nnzA]; b: device float64
    [batch, nrhs, n] (not modified).  Returns (options dict, table) where
    table lists every candidate with its factor and solve times."""
    colptr = np.ascontiguousarray(colptr, np.int64)
    rowind = np.ascontiguousarray(rowind, np.int32)
    perm = None if perm is None else np.ascontiguousarray(perm, np.int32)
    n = len(colptr) - 1
    best = Options()
    cap = 64
    table = (TuneEntry * cap)()
    cnt = ctypes.c_int32(0)
    _check(_lib.sc_autotune(n, _ptr(colptr), _ptr(rowind), _ptr(perm),
                            _dev_ptr(values, "float64"), int(values.shape[1]),
                            int(values.shape[0]), _DTYPES[dtype], _dev_ptr(b, "float64"),
                            int(b.shape[1]), int(b.shape[2]), float(solves_per_factor),
                            ctypes.byref(best), table, cap, ctypes.byref(cnt),
                            _stream_handle(stream)), "sc_autotune")
    as_dict = lambda o: {k: getattr(o, k) for k, _ in Options._fields_}
    rows = [dict(as_dict(table[i].opt), factor_ms=table[i].factor_ms,
                 solve_ms=table[i].solve_ms, score=table[i].score) for i in range(cnt.value)]
    return as_dict(best), rows


def autotune_group(patterns, values, b, dtype: str = "f64", solves_per_factor: float = 1.0,
                   stream=None):
    """sc_autotune_group: the autotuner on the group plan of `patterns`
    (sequence of (colptr, rowind) or (colptr, rowind, perm)); values and b
    are the concatenated device arrays of the group.  Returns (options dict,
    table) as autotune()."""
    keep = []
    cps, ris, pms, ns = [], [], [], []
    for pat in patterns:
        cp = np.ascontiguousarray(pat[0], np.int64)
        ri = np.ascontiguousarray(pat[1], np.int32)
        pm = None if len(pat) < 3 or pat[2] is None else np.ascontiguousarray(pat[2], np.int32)
        keep += [cp, ri, pm]
        cps.append(cp.ctypes.data)
        ris.append(ri.ctypes.data)
        pms.append(pm.ctypes.data if pm is not None else None)
        ns.append(len(cp) - 1)
    npat = len(ns)
    ns = np.array(ns, np.int64)
    cpa = (ctypes.c_void_p * npat)(*cps)
    ria = (ctypes.c_void_p * npat)(*ris)
    pma = (ctypes.c_void_p * npat)(*pms)
    best = Options()
    cap = 64
    table = (TuneEntry * cap)()
    cnt = ctypes.c_int32(0)
    _check(_lib.sc_autotune_group(npat, _ptr(ns), cpa, ria, pma, _dev_ptr(values, "float64"),
                                  int(values.shape[1]), int(values.shape[0]), _DTYPES[dtype],
                                  _dev_ptr(b, "float64"), int(b.shape[1]), int(b.shape[2]),
                                  float(solves_per_factor), ctypes.byref(best), table, cap,
                                  ctypes.byref(cnt), _stream_handle(stream)),
           "sc_autotune_group")
    as_dict = lambda o: {k: getattr(o, k) for k, _ in Options._fields_}
    rows = [dict(as_dict(table[i].opt), factor_ms=table[i].factor_ms,
                 solve_ms=table[i].solve_ms, score=table[i].score) for i in range(cnt.value)]
    return as_dict(best), rows


def analyze_group(patterns, **opts) -> GroupPlan:
    """patterns: sequence of (colptr, rowind) or (colptr, rowind, perm)."""
    return GroupPlan(patterns, default_options(**opts) if opts else None)


class Numeric:
    """Device storage for a batch of factors of one plan."""

    def __init__(self, plan: Plan, batch: int, dtype: str):
        self.plan = plan
        self.batch = int(batch)
        self.dtype = dtype
        h = ctypes.c_void_p()
        _check(_lib.sc_numeric_create(plan._h, self.batch, _DTYPES[dtype], ctypes.byref(h)),
               "sc_numeric_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.sc_numeric_destroy(h)
            self._h = None

    def factor(self, values, stream=None):
        """values: device float64 tensor [batch, ldv] (ldv >= nnzA)."""
        if values.dim() != 2 or values.shape[0] != self.batch:
            raise ValueError("values must be [batch, nnzA]")
        # contiguous [batch, ldv]: the row pitch is the row length (a size-1
        # batch dimension may report any stride)
        _check(_lib.sc_factor(self.plan._h, self._h, _dev_ptr(values, "float64"),
                              int(values.shape[1]), _stream_handle(stream)), "sc_factor")

    def info(self, stream=None) -> np.ndarray:
        """Breakdown steps: [batch] for a plan of one pattern, [batch, nblocks]
        for a group plan (0 = factor complete)."""
        nb = self.plan.nblocks
        out = np.empty(self.batch * nb, np.int32)
        st = _lib.sc_factor_info(self._h, _ptr(out), _stream_handle(stream))
        if st not in (SC_OK, SC_ENOTSPD):
            raise SpcholError(st, "sc_factor_info")
        return out if nb == 1 else out.reshape(self.batch, nb)

    def solve(self, b, stream=None):
        """b: device float64 tensor [batch, nrhs, n]; overwritten by x."""
        if b.dim() != 3 or b.shape[0] != self.batch:
            raise ValueError("b must be [batch, nrhs, n]")
        _check(_lib.sc_solve(self.plan._h, self._h, _dev_ptr(b, "float64"), int(b.shape[1]),
                             int(b.shape[2]), _stream_handle(stream)), "sc_solve")
        return b

    def solve_noalloc(self, b, stream=None):
        """As solve(), through sc_solve_noalloc: no device allocation, the
        solve vectors in the library's static scratch (SC_ESCRATCH when they
        do not fit)."""
        if b.dim() != 3 or b.shape[0] != self.batch:
            raise ValueError("b must be [batch, nrhs, n]")
        _check(_lib.sc_solve_noalloc(self.plan._h, self._h, _dev_ptr(b, "float64"),
                                     int(b.shape[1]), int(b.shape[2]), _stream_handle(stream)),
               "sc_solve_noalloc")
        return b

    def refine_solve(self, values, b, x, tol: float = 1e-10, maxit: int = 10,
                     method: str = "classical", stream=None):
        """x <- refined solution of A x = b (see sc_refine_solve).  values:
        the factored float64 values [batch, nnzA]; b, x: float64
        [batch, nrhs, n] device tensors.  Returns (status, stats) where stats
        is a list of dicts per system, ordered (matrix, rhs, block)."""
        if b.shape != x.shape or b.dim() != 3 or b.shape[0] != self.batch:
            raise ValueError("b and x must be [batch, nrhs, n]")
        nsys = self.batch * int(b.shape[1]) * self.plan.nblocks
        st = (RefineStats * nsys)()
        rc = _lib.sc_refine_solve(self.plan._h, self._h, _dev_ptr(values, "float64"),
                                  int(values.shape[1]), _dev_ptr(b, "float64"),
                                  _dev_ptr(x, "float64"), int(b.shape[1]), int(b.shape[2]),
                                  float(tol), int(maxit), _METHODS[method], st,
                                  _stream_handle(stream))
        if rc not in (SC_OK, SC_ENOCONV):
            raise SpcholError(rc, "sc_refine_solve")
        return rc, [{k: getattr(st[i], k) for k, _ in RefineStats._fields_}
                    for i in range(nsys)]

    def adjoint(self, x, gx, stream=None):
        """(dL/dvalues [batch, nnzA], dL/db [batch, nrhs, n]) for x = A^{-1} b
        solved with the stored factor and the upstream gradient gx = dL/dx
        (see sc_adjoint)."""
        import torch
        if x.shape != gx.shape or x.dim() != 3 or x.shape[0] != self.batch:
            raise ValueError("x and gx must be [batch, nrhs, n]")
        gx = gx.contiguous()
        gv = torch.empty((self.batch, self.plan.info()["nnzA"]), dtype=torch.float64,
                         device=x.device)
        gb = torch.empty_like(gx)
        _check(_lib.sc_adjoint(self.plan._h, self._h, _dev_ptr(x, "float64"),
                               _dev_ptr(gx, "float64"), _dev_ptr(gv, "float64"),
                               int(gv.shape[1]), _dev_ptr(gb, "float64"), int(x.shape[1]),
                               int(x.shape[2]), _stream_handle(stream)), "sc_adjoint")
        return gv, gb

    def step_graph(self, values, b, x, tol: float = 1e-10, iters: int = 3,
                   method: str = "classical") -> "StepGraph":
        """Capture factor(values) + refined solve b -> x with exactly `iters`
        refinement steps as one HIP graph (see sc_step_graph_create).  The
        tensors must stay alive and unmoved while the graph is used."""
        if b.shape != x.shape or b.dim() != 3 or b.shape[0] != self.batch:
            raise ValueError("b and x must be [batch, nrhs, n]")
        h = ctypes.c_void_p()
        _check(_lib.sc_step_graph_create(self.plan._h, self._h, _dev_ptr(values, "float64"),
                                         int(values.shape[1]), _dev_ptr(b, "float64"),
                                         _dev_ptr(x, "float64"), int(b.shape[1]),
                                         int(b.shape[2]), float(tol), int(iters),
                                         _METHODS[method], ctypes.byref(h)),
               "sc_step_graph_create")
        return StepGraph(self, h, self.batch * int(b.shape[1]) * self.plan.nblocks,
                         (values, b, x))

    def get_columns(self, b: int, cols) -> np.ndarray:
        """Values of L on the exact pattern for the given columns (host)."""
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        _, _, Lcolptr, _ = self._lcolptr()
        total = int(np.sum(Lcolptr[cols + 1] - Lcolptr[cols])) if cols.size else 0
        out = np.empty(total, np.float64)
        _check(_lib.sc_numeric_get_columns(self.plan._h, self._h, int(b), int(cols.size),
                                           _ptr(cols), _ptr(out)), "sc_numeric_get_columns")
        return out

    def get_block(self, b: int, s: int) -> np.ndarray:
        """The whole stored c x w block of supernode s of factor b (host,
        float64, [w, c]: row t of the result is column t of the block)."""
        if not hasattr(self.plan, "_sn"):
            self.plan._sn = self.plan.export_supernodes()
        first, _, _, rowptr, _ = self.plan._sn
        c, w = int(rowptr[s + 1] - rowptr[s]), int(first[s + 1] - first[s])
        out = np.empty(c * w, np.float64)
        _check(_lib.sc_numeric_get_block(self.plan._h, self._h, int(b), int(s), _ptr(out)),
               "sc_numeric_get_block")
        return out.reshape(w, c)

    def profile(self, enable: bool = True):
        """Time every later launch with HIP events (see sc_numeric_profile)."""
        _check(_lib.sc_numeric_profile(self._h, 1 if enable else 0), "sc_numeric_profile")

    def profile_read(self) -> dict:
        """Per-kernel totals {name: {launches, ms, flops, bytes}}; clears them."""
        arr = (KernelStat * 32)()
        cnt = ctypes.c_int32()
        _check(_lib.sc_numeric_profile_read(self._h, 32, arr, ctypes.byref(cnt)),
               "sc_numeric_profile_read")
        return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms,
                                       "flops": arr[i].flops, "bytes": arr[i].bytes,
                                       "alg_bytes": arr[i].alg_bytes}
                for i in range(cnt.value)}

    def _lcolptr(self):
        if not hasattr(self.plan, "_Lcolptr"):
            inf = self.plan.info()
            Lcolptr = np.empty(inf["n"] + 1, np.int64)
            _check(_lib.sc_plan_export_symbolic(self.plan._h, None, None, _ptr(Lcolptr), None),
                   "sc_plan_export_symbolic")
            self.plan._Lcolptr = Lcolptr
        return None, None, self.plan._Lcolptr, None


class StepGraph:
    """A captured factor + refined-solve step (sc_step_graph_*)."""

    def __init__(self, num: "Numeric", h, nsys: int, keep):
        self.num = num
        self._h = h
        self.nsys = nsys
        self._keep = keep  # the captured buffers stay alive with the graph

    def __del__(self):
        self.destroy()

    def destroy(self):
        """Release the graph (sc_step_graph_destroy); later calls on the
        numeric object may then grow its workspaces again."""
        if getattr(self, "_h", None):
            _lib.sc_step_graph_destroy(self._h)
            self._h = None

    def launch(self, stream=None):
        _check(_lib.sc_step_graph_launch(self._h, _stream_handle(stream)), "sc_step_graph_launch")

    def stats(self, stream=None):
        st = (RefineStats * self.nsys)()
        rc = _lib.sc_step_graph_stats(self._h, st, _stream_handle(stream))
        if rc not in (SC_OK, SC_ENOCONV):
            raise SpcholError(rc, "sc_step_graph_stats")
        return rc, [{k: getattr(st[i], k) for k, _ in RefineStats._fields_}
                    for i in range(self.nsys)]


def _autograd_function():
    import torch

    class SolveFn(torch.autograd.Function):
        """x = A^{-1} b for a batch on a fixed pattern, differentiable in the
        stored values of A and in b.  forward factors `values` into `num`
        and solves; backward runs the adjoint with the same factor (one more
        solve, sc_adjoint), so `num` must not be refactored in between."""

        @staticmethod
        def forward(ctx, values, b, num):
            num.factor(values.detach())
            x = b.detach().clone()
            num.solve(x)
            ctx.num = num
            ctx.save_for_backward(x)
            return x

        @staticmethod
        def backward(ctx, gx):
            (x,) = ctx.saved_tensors
            gv, gb = ctx.num.adjoint(x, gx)
            return gv, gb, None

    return SolveFn


def solve_fn(num: "Numeric", values, b):
    """Differentiable solve: x = A(values)^{-1} b with autograd support in
    values [batch, nnzA] and b [batch, nrhs, n] (float64 device tensors)."""
    global SolveFn
    if SolveFn is None:
        SolveFn = _autograd_function()
    return SolveFn.apply(values, b, num)


SolveFn = None
