"""CPU oracle for sparse Cholesky LL^T and triangular solves (FP64).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is independent of
the GPU library (no shared code, headers or tables); the two only share the
seeded input generators in ``workloads``.

The arithmetic lives in ``oracle.c`` (plain serial C, built with
``-O2 -ffp-contract=off -fno-fast-math``).  This module marshals numpy
arrays and adds the error measures used to compare results, all in FP64:

  relres = ||b - A x||_2 / ||b||_2
  eta    = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)
  forward error  ||x - x_o||_inf / ||x_o||_inf
  factor error   max_j ||L[:, j] - L_o[:, j]||_inf / ||L_o[:, j]||_inf

and the gradients of a loss through the solve (``solve_gradients``): for
x = A^{-1} b and upstream gradient g_x, differentiating A x = b gives
dx = A^{-1} (db - dA x), so g_b = A^{-T} g_x = lambda (A symmetric: one more
solve with the same factor) and dL/dA_ij = -lambda_i x_j; a stored lower
entry v_k stands for A_ij and A_ji, hence -(lambda_i x_j + lambda_j x_i)
off the diagonal and -lambda_i x_i on it (summed over right-hand sides).
It also estimates kappa_1 = ||A||_1 ||A^{-1}||_1, with ||A^{-1}||_1 from
Hager's method (Higham's safeguards) over oracle solves, and evaluates the
stop rule of a refined solution: relres <= tol, or the residual at the FP64
evaluation floor ||r||_2 <= 2 u ||A||_inf ||x||_2 (u = 2^-53).

Parity status: every function here is pinned by tests/test_oracle.py
(dense LAPACK Cholesky, closed forms of the 1D Laplacian, exact results for
diagonal matrices, brute-force boolean elimination for the pattern; the
gradients by central finite differences and by the closed-form inverse of
the 1D Laplacian; the error measures and norms by hand-computed 3x3 and 4x4
cases; the condition estimate by numpy's exact one-norm condition number on
dense cases and the closed-form ||A^{-1}||_1 of the 1D Laplacian).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=c11"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
U64 = 2.0 ** -53   # unit roundoff of FP64


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.or_symbolic.argtypes = [I64, P, P, P, I64, P, P, P]
        lib.or_symbolic.restype = ctypes.c_int
        lib.or_factor.argtypes = [I64, P, P, P, P, I64, P, P, P, P]
        lib.or_factor.restype = ctypes.c_int
        lib.or_solve.argtypes = [I64, P, P, P, P, P, I64]
        lib.or_solve.restype = None
        lib.or_spmv.argtypes = [I64, P, P, P, P, P, I64]
        lib.or_spmv.restype = None
        lib.or_inv_norm1_est.argtypes = [I64, P, P, P, P]
        lib.or_inv_norm1_est.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Symbolic:
    n: int
    nrows: int
    perm: Optional[np.ndarray]
    parent: np.ndarray   # int32[n]
    Lcolptr: np.ndarray  # int64[n+1]
    Lrowind: np.ndarray  # int32[nnzL]

    @property
    def nnzL(self) -> int:
        return int(self.Lcolptr[-1])

    @property
    def counts(self) -> np.ndarray:
        return np.diff(self.Lcolptr)

    def flops(self) -> float:
        """Sum of squared column counts (multiply-add counted as 2 flops)."""
        c = self.counts.astype(np.float64)
        return float(np.sum(c * c))


def symbolic(n, colptr, rowind, perm=None, nrows=None) -> Symbolic:
    """Elimination tree and pattern of L for P A P^T (rows < nrows only)."""
    lib = _load()
    colptr = _c(colptr, np.int64)
    rowind = _c(rowind, np.int32)
    perm = _c(perm, np.int32)
    nr = n if nrows is None else int(nrows)
    parent = np.empty(n, dtype=np.int32)
    Lcolptr = np.empty(n + 1, dtype=np.int64)
    rc = lib.or_symbolic(n, _p(colptr), _p(rowind), _p(perm), nr, _p(parent),
                         _p(Lcolptr), None)
    if rc:
        raise MemoryError("or_symbolic")
    Lrowind = np.empty(int(Lcolptr[-1]), dtype=np.int32)
    rc = lib.or_symbolic(n, _p(colptr), _p(rowind), _p(perm), nr, _p(parent),
                         _p(Lcolptr), _p(Lrowind))
    if rc:
        raise MemoryError("or_symbolic")
    return Symbolic(n=n, nrows=nr, perm=perm, parent=parent, Lcolptr=Lcolptr,
                    Lrowind=Lrowind)


def factor(n, colptr, rowind, values, sym: Symbolic):
    """Numeric factor.  Returns (Lx, info) with info = 0 or the 1-based row
    whose pivot failed."""
    lib = _load()
    colptr = _c(colptr, np.int64)
    rowind = _c(rowind, np.int32)
    values = _c(values, np.float64)
    Lx = np.zeros(sym.nnzL, dtype=np.float64)
    info = lib.or_factor(n, _p(colptr), _p(rowind), _p(values), _p(sym.perm),
                         sym.nrows, _p(sym.parent), _p(sym.Lcolptr),
                         _p(sym.Lrowind), _p(Lx))
    if info < 0:
        raise MemoryError("or_factor")
    return Lx, int(info)


def solve(sym: Symbolic, Lx, b):
    """x = A^{-1} b for b of shape [n] or [nrhs, n]."""
    lib = _load()
    b = np.array(b, dtype=np.float64, copy=True, order="C")
    shape = b.shape
    b2 = b.reshape(-1, sym.n)
    Lx = _c(Lx, np.float64)
    lib.or_solve(sym.n, _p(sym.Lcolptr), _p(sym.Lrowind), _p(Lx), _p(sym.perm),
                 _p(b2), b2.shape[0])
    return b2.reshape(shape)


def spmv(n, colptr, rowind, values, x):
    """A x with A given by its lower CSC triangle; x of shape [n] or [k, n]."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    shape = x.shape
    x2 = x.reshape(-1, n)
    y = np.empty_like(x2)
    lib.or_spmv(n, _p(_c(colptr, np.int64)), _p(_c(rowind, np.int32)),
                _p(_c(values, np.float64)), _p(x2), _p(y), x2.shape[0])
    return y.reshape(shape)


def norm_inf_sym(n, colptr, rowind, values) -> float:
    """||A||_inf of the symmetric matrix stored by its lower triangle."""
    colptr = np.asarray(colptr, np.int64)
    rowind = np.asarray(rowind, np.int64)
    values = np.asarray(values, np.float64)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    s = np.zeros(n)
    np.add.at(s, rowind, np.abs(values))
    off = rowind != cols
    np.add.at(s, cols[off], np.abs(values[off]))
    return float(s.max()) if n else 0.0


def residual_measures(n, colptr, rowind, values, x, b):
    """Per right-hand side: (relres, eta).  x, b: [nrhs, n] (or [n])."""
    x2 = np.asarray(x, np.float64).reshape(-1, n)
    b2 = np.asarray(b, np.float64).reshape(-1, n)
    r = b2 - spmv(n, colptr, rowind, values, x2)
    an = norm_inf_sym(n, colptr, rowind, values)
    relres = np.linalg.norm(r, axis=1) / np.maximum(np.linalg.norm(b2, axis=1), 1e-300)
    eta = np.abs(r).max(1) / (an * np.abs(x2).max(1) + np.abs(b2).max(1))
    return relres, eta


def stop_clause(n, colptr, rowind, values, x, b, tol):
    """Per right-hand side, which clause of the stop rule holds: 1 if
    ||b - A x||_2 <= tol ||b||_2, else 2 if ||b - A x||_2 <= 2 u ||A||_inf
    ||x||_2 (u = 2^-53), else 0.  x, b: [nrhs, n] (or [n])."""
    x2 = np.asarray(x, np.float64).reshape(-1, n)
    b2 = np.asarray(b, np.float64).reshape(-1, n)
    r = b2 - spmv(n, colptr, rowind, values, x2)
    rn = np.linalg.norm(r, axis=1)
    an = norm_inf_sym(n, colptr, rowind, values)
    c1 = rn <= tol * np.linalg.norm(b2, axis=1)
    c2 = rn <= 2.0 * U64 * an * np.linalg.norm(x2, axis=1)
    return np.where(c1, 1, np.where(c2, 2, 0)).astype(np.int32)


def inv_norm1_estimate(sym: Symbolic, Lx) -> float:
    """Lower-bound estimate of ||A^{-1}||_1 by Hager's method with Higham's
    safeguards (oracle.c, or_inv_norm1_est), from solves with the factor."""
    lib = _load()
    v = lib.or_inv_norm1_est(sym.n, _p(sym.Lcolptr), _p(sym.Lrowind),
                             _p(_c(Lx, np.float64)), _p(sym.perm))
    if v < 0:
        raise MemoryError("or_inv_norm1_est")
    return float(v)


def kappa1_estimate(n, colptr, rowind, values, sym: Symbolic, Lx) -> float:
    """kappa_1(A) = ||A||_1 ||A^{-1}||_1 with the second factor estimated
    (Hager/Higham); A is symmetric, so ||A||_1 = ||A||_inf."""
    return norm_inf_sym(n, colptr, rowind, values) * inv_norm1_estimate(sym, Lx)


def within_conditioning(xerr: float, tol: float, kappa1: float) -> bool:
    """Acceptance of a solution's forward error against the oracle: at most
    `tol`, or, when the system is too ill-conditioned for two correct FP64
    solvers to agree to `tol`, at most 10 kappa_1 u (the conditioning limit
    of a backward-stable solve)."""
    return xerr <= tol or xerr <= 10.0 * kappa1 * U64


def forward_error(x, x_ref) -> float:
    x = np.asarray(x, np.float64).ravel()
    x_ref = np.asarray(x_ref, np.float64).ravel()
    return float(np.abs(x - x_ref).max() / max(np.abs(x_ref).max(), 1e-300))


def factor_error(Lcolptr, Lx, Lx_ref) -> float:
    """max over columns of ||dL[:, j]||_inf / ||L_ref[:, j]||_inf."""
    Lcolptr = np.asarray(Lcolptr, np.int64)
    d = np.abs(np.asarray(Lx, np.float64) - np.asarray(Lx_ref, np.float64))
    a = np.abs(np.asarray(Lx_ref, np.float64))
    n = len(Lcolptr) - 1
    counts = np.diff(Lcolptr)
    nz = counts > 0
    starts = Lcolptr[:-1][nz]
    dm = np.maximum.reduceat(d, starts) if d.size else np.zeros(0)
    am = np.maximum.reduceat(a, starts) if a.size else np.zeros(0)
    if dm.size == 0:
        return 0.0
    return float(np.max(dm / np.maximum(am, 1e-300)))


def to_dense_permuted(n, colptr, rowind, values, perm=None) -> np.ndarray:
    """Dense P A P^T (for small test cases only)."""
    A = np.zeros((n, n))
    colptr = np.asarray(colptr, np.int64)
    for c in range(n):
        for p in range(colptr[c], colptr[c + 1]):
            r = int(rowind[p])
            A[r, c] = values[p]
            A[c, r] = values[p]
    if perm is not None:
        perm = np.asarray(perm, np.int64)
        A = A[np.ix_(perm, perm)]
    return A


def L_dense(sym: Symbolic, Lx) -> np.ndarray:
    L = np.zeros((sym.n, sym.n))
    for j in range(sym.n):
        for q in range(sym.Lcolptr[j], sym.Lcolptr[j + 1]):
            L[sym.Lrowind[q], j] = Lx[q]
    return L


def solve_gradients(n, colptr, rowind, values, sym: Symbolic, Lx, x, gx):
    """Gradients of a loss L(x), x = A^{-1} b, with respect to the stored
    lower-triangle values of A and to b, given x [nrhs, n] and the upstream
    gradient gx = dL/dx [nrhs, n].  Returns (g_values [nnz], g_b [nrhs, n]).
    lambda = A^{-1} gx (A = A^T), g_b = lambda, and for a stored entry (i, j):
    -(lambda_i x_j + lambda_j x_i) if i != j, -lambda_i x_i if i == j, summed
    over the right-hand sides."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, n)
    gx = np.asarray(gx, dtype=np.float64).reshape(-1, n)
    lam = solve(sym, Lx, gx).reshape(-1, n)
    colptr = np.asarray(colptr, np.int64)
    rows = np.asarray(rowind, np.int64)
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(colptr))
    g = np.zeros(rows.size)
    for r in range(x.shape[0]):
        t = lam[r, rows] * x[r, cols]
        g -= np.where(rows == cols, t, t + lam[r, cols] * x[r, rows])
    return g, lam


def cotan_values(n, colptr, rowind, pos, tris, mass, mass_coeff, clip_lo, clip_hi,
                 edge_scale=None):
    """Values (lower CSC order) of A = K + c diag(m) for a triangle mesh,
    K the cotangent stiffness matrix (the operator the paper assembles in
    its cotan construction, Sec. 5.3), written out from its definition:

      cot of the angle at corner o of a triangle, opposite edge (p, q):
          u = x_p - x_o,  v = x_q - x_o,  cot = (u . v) / |u_0 v_1 - u_1 v_0|
      w_pq = clip(1/2 * sum of cot over the (one or two) triangles with
                  edge (p, q), clip_lo, clip_hi)
      per value set s: w^s_pq = clip(w_pq * scale_s[pq], clip_lo, clip_hi)
                       (skipped when edge_scale is None)
      K_pq = -w^s_pq (p != q),  K_pp = sum_q w^s_pq,  A = K + c diag(m).

    The sum of a diagonal entry runs over the neighbours q > p in ascending
    order, then the neighbours q < p in ascending order (a fixed order, so
    the result is reproducible to the bit); sums of two terms do not depend
    on order.  Every stored off-diagonal entry must be a mesh edge.
    pos: [nv, 2] or [batch, nv, 2]; tris: [ntri, 3]; edge_scale:
    [batch, nedge] in the storage order of the off-diagonal entries, or
    None.  Returns values [batch, nnz] (batch 1 without scales and with one
    position set)."""
    colptr = np.asarray(colptr, np.int64)
    rowind = np.asarray(rowind, np.int64)
    tris = np.asarray(tris, np.int64)
    mass = np.asarray(mass, np.float64)
    pos = np.asarray(pos, np.float64)
    nnz = int(colptr[-1])
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(colptr))
    off = rowind != cols
    key_store = cols[off] * n + rowind[off]           # (lo, hi), lo = column
    nedge = key_store.size
    batch = 1
    if edge_scale is not None:
        edge_scale = np.asarray(edge_scale, np.float64).reshape(-1, nedge)
        batch = edge_scale.shape[0]
    if pos.ndim == 3:
        batch = max(batch, pos.shape[0])
    out = np.zeros((batch, nnz))
    # the three corners of every triangle and their opposite edges
    corners = []
    for c in range(3):
        o, p, q = tris[:, c], tris[:, (c + 1) % 3], tris[:, (c + 2) % 3]
        corners.append((o, np.minimum(p, q), np.maximum(p, q)))
    for s in range(batch):
        x = pos[s] if pos.ndim == 3 else pos
        w = np.zeros(nedge)
        hit = np.zeros(nedge, np.int64)
        for o, lo, hi in corners:
            u = x[lo] - x[o]
            v = x[hi] - x[o]
            dot = u[:, 0] * v[:, 0] + u[:, 1] * v[:, 1]
            cross = np.abs(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0])
            e = np.searchsorted(key_store, lo * n + hi)
            if np.any(e >= nedge) or np.any(key_store[np.minimum(e, nedge - 1)] != lo * n + hi):
                raise ValueError("a triangle edge is not a stored entry")
            np.add.at(w, e, 0.5 * (dot / cross))
            np.add.at(hit, e, 1)
        if np.any(hit == 0) or np.any(hit > 2):
            raise ValueError("every stored entry must be an edge of one or two triangles")
        w = np.clip(w, clip_lo, clip_hi)
        if edge_scale is not None:
            w = np.clip(w * edge_scale[s], clip_lo, clip_hi)
        vals = np.zeros(nnz)
        vals[off] = -w
        # diagonal: neighbours above (q > p, column p) ascending, then below
        lo_e = key_store // n
        hi_e = key_store % n
        deg = np.zeros(n)
        np.add.at(deg, lo_e, w)     # column p: its rows q > p, ascending
        order = np.lexsort((lo_e, hi_e))
        np.add.at(deg, hi_e[order], w[order])   # row p: columns q < p, ascending
        diag = ~off
        vals[diag] = (deg + mass_coeff * mass)[rowind[diag]]
        out[s] = vals
    return out


def sparse_product(m, n, A, B, transB=False, D=None):
    """C = A B (transB False) or A B^T (transB True), plus D when given, for
    CSR matrices given as (rowptr, colind, values): the sparse products the
    paper evaluates with its generated kernels (Sec. 5.2, Table tab:Lpow).
    A is m x p; B is p x n (or n x p when transposed); D is m x n.  The
    product itself is scipy's sparse matrix product in FP64 (a library
    routine as one step); D is added after it.  Returns C as a scipy CSR
    matrix with sorted indices (explicit zeros of the pattern kept out)."""
    import scipy.sparse as sp
    Ar, Ac, Av = A
    Br, Bc, Bv = B
    Am = sp.csr_matrix((np.asarray(Av, np.float64), np.asarray(Ac), np.asarray(Ar)),
                       shape=(m, int(np.max(Ac)) + 1 if len(Ac) else 0))
    nb_rows = len(Br) - 1
    Bm = sp.csr_matrix((np.asarray(Bv, np.float64), np.asarray(Bc), np.asarray(Br)),
                       shape=(nb_rows, int(np.max(Bc)) + 1 if len(Bc) else 0))
    if transB:
        Bm = Bm.T
    p = max(Am.shape[1], Bm.shape[0])
    Am = sp.csr_matrix((Am.data, Am.indices, Am.indptr), shape=(m, p))
    Bm = sp.csr_matrix(Bm.tocsr(), shape=(p, Bm.shape[1]))
    Bm = sp.csr_matrix((Bm.data, Bm.indices, Bm.indptr), shape=(p, n))
    C = (Am @ Bm).tocsr()
    if D is not None:
        Dr, Dc, Dv = D
        C = C + sp.csr_matrix((np.asarray(Dv, np.float64), np.asarray(Dc), np.asarray(Dr)),
                              shape=(m, n))
    C = C.tocsr()
    C.sort_indices()
    return C


def sparse_product_pattern(m, n, A_rowptr, A_colind, B_rowptr, B_colind, transB=False,
                           D_rowptr=None, D_colind=None):
    """Structural pattern (rowptr, colind) of A B (or A B^T) union D: entry
    (i, j) is present when some k has A_ik and B_kj (B_jk) stored, whatever
    the values; written as a plain loop over the rows (small cases)."""
    Ar = np.asarray(A_rowptr); Ac = np.asarray(A_colind)
    Br = np.asarray(B_rowptr); Bc = np.asarray(B_colind)
    if transB:
        # rows of B^T: the columns of B
        nbr = len(Br) - 1
        brows = {}
        for j in range(nbr):
            for q in range(Br[j], Br[j + 1]):
                brows.setdefault(int(Bc[q]), []).append(j)
    else:
        brows = {k: [int(c) for c in Bc[Br[k]:Br[k + 1]]] for k in range(len(Br) - 1)}
    rowptr = [0]
    colind = []
    for i in range(m):
        cols = set()
        for q in range(Ar[i], Ar[i + 1]):
            cols.update(brows.get(int(Ac[q]), []))
        if D_rowptr is not None:
            cols.update(int(c) for c in D_colind[D_rowptr[i]:D_rowptr[i + 1]])
        colind.extend(sorted(cols))
        rowptr.append(len(colind))
    return np.array(rowptr, np.int64), np.array(colind, np.int32)
