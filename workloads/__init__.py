"""Seeded synthetic SPD systems on fixed sparsity patterns.

This module builds inputs only: lower-triangular CSC patterns, value sets,
right-hand sides and a geometric nested-dissection permutation. It contains
none of the factorization arithmetic, so both the CPU oracle and the GPU
library can be fed from it without sharing any code of the method.

Conventions (used by every caller):
  * A symmetric matrix is passed by its lower triangle in CSC form:
    ``colptr`` int64[n+1], ``rowind`` int32[nnz], rows sorted ascending inside
    each column, diagonal entry first.  ``values`` is float64[batch, nnz] in
    the same entry order.
  * ``perm`` is int32[n] with ``perm[k]`` = original index of the vertex that
    is eliminated k-th (new k <- old perm[k]).

The workloads stand in for the mesh-derived systems of the paper's
evaluation (cotangent Laplacian plus mass matrix, Sec. 5.3; the
factor/solve that follows assembly in Sec. 5.5 and 5.6).  No mesh or dataset
from the paper is used; every input is generated from a seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "SymPattern",
    "Workload",
    "grid_edges",
    "lower_csc_from_edges",
    "grid_nd_perm",
    "laplacian_values",
    "rhs",
    "trimesh_edges_weights",
    "trimesh_geometry",
    "config",
    "small_grid",
    "random_spd",
    "block_vector_workload",
]


@dataclass
class SymPattern:
    """Lower-triangular CSC pattern of a symmetric matrix (diagonal first)."""

    n: int
    colptr: np.ndarray  # int64[n+1]
    rowind: np.ndarray  # int32[nnz]
    # For every stored entry: its (row, col) in original numbering.
    rows: np.ndarray = field(repr=False, default=None)
    cols: np.ndarray = field(repr=False, default=None)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def offdiag_mask(self) -> np.ndarray:
        return self.rows != self.cols


@dataclass
class Workload:
    """One pattern with a batch of value sets and right-hand sides."""

    name: str
    pattern: SymPattern
    perm: Optional[np.ndarray]  # int32[n] or None (natural order)
    values: np.ndarray  # float64[batch, nnz]
    b: np.ndarray  # float64[batch, nrhs, n]
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return int(self.values.shape[0])

    @property
    def nrhs(self) -> int:
        return int(self.b.shape[1])


# ---------------------------------------------------------------------------
# patterns
# ---------------------------------------------------------------------------

def grid_edges(dims: Sequence[int]) -> Tuple[int, np.ndarray]:
    """Edges of the 5-point (2D) or 7-point (3D) grid stencil.

    Vertex (x, y, z) has index x + nx*(y + ny*z).  Returns (n, edges[m, 2])
    with edges[:, 0] < edges[:, 1].
    """
    dims = tuple(int(d) for d in dims)
    while len(dims) < 3:
        dims = dims + (1,)
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    edges = []
    if nx > 1:
        edges.append(np.stack([idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()], 1))
    if ny > 1:
        edges.append(np.stack([idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()], 1))
    if nz > 1:
        edges.append(np.stack([idx[:-1, :, :].ravel(), idx[1:, :, :].ravel()], 1))
    if edges:
        e = np.concatenate(edges, 0)
    else:
        e = np.zeros((0, 2), dtype=np.int64)
    return n, e


def lower_csc_from_edges(n: int, edges: np.ndarray) -> SymPattern:
    """Lower CSC pattern with a diagonal plus one entry per undirected edge."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    lo = np.minimum(edges[:, 0], edges[:, 1])
    hi = np.maximum(edges[:, 0], edges[:, 1])
    if np.any(lo == hi):
        raise ValueError("self loops are not edges")
    diag = np.arange(n, dtype=np.int64)
    cols = np.concatenate([diag, lo])
    rows = np.concatenate([diag, hi])
    order = np.lexsort((rows, cols))
    cols = cols[order]
    rows = rows[order]
    if len(rows) > 1:
        dup = (cols[1:] == cols[:-1]) & (rows[1:] == rows[:-1])
        if np.any(dup):
            raise ValueError("duplicate edges")
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)
    return SymPattern(n=n, colptr=colptr, rowind=rows.astype(np.int32),
                      rows=rows, cols=cols)


def grid_nd_perm(dims: Sequence[int], leaf: int = 8) -> np.ndarray:
    """Geometric nested-dissection order of a box grid.

    The box is split along its longest axis (ties: x, then y, then z) at the
    plane m = floor((lo + hi) / 2).  Elimination order is: left part, right
    part, then the separator plane (numbered x fastest).  Boxes with at most
    ``leaf`` vertices are numbered naturally.  Returns perm with
    perm[new] = old.
    """
    dims = tuple(int(d) for d in dims)
    while len(dims) < 3:
        dims = dims + (1,)
    nx, ny, nz = dims
    out: List[np.ndarray] = []

    def box_ids(lo, hi):
        xs = np.arange(lo[0], hi[0] + 1)
        ys = np.arange(lo[1], hi[1] + 1)
        zs = np.arange(lo[2], hi[2] + 1)
        z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")
        return (x + nx * (y + ny * z)).ravel()

    stack = [(tuple([0, 0, 0]), tuple([nx - 1, ny - 1, nz - 1]), 0)]
    # explicit stack to avoid recursion limits; state 0 = visit, 1 = emit sep
    while stack:
        lo, hi, state = stack.pop()
        if state == 1:
            out.append(box_ids(lo, hi))
            continue
        ext = [hi[a] - lo[a] + 1 for a in range(3)]
        if min(ext) <= 0:
            continue
        if ext[0] * ext[1] * ext[2] <= leaf:
            out.append(box_ids(lo, hi))
            continue
        a = int(np.argmax(ext))  # first maximum: x before y before z
        m = (lo[a] + hi[a]) // 2
        left_hi = list(hi); left_hi[a] = m - 1
        right_lo = list(lo); right_lo[a] = m + 1
        sep_lo = list(lo); sep_lo[a] = m
        sep_hi = list(hi); sep_hi[a] = m
        # pushed in reverse: left is processed first, then right, then sep
        stack.append((tuple(sep_lo), tuple(sep_hi), 1))
        stack.append((tuple(right_lo), tuple(hi), 0))
        stack.append((tuple(lo), tuple(left_hi), 0))
    perm = np.concatenate(out) if out else np.zeros(0, dtype=np.int64)
    assert perm.size == nx * ny * nz
    return perm.astype(np.int32)


# ---------------------------------------------------------------------------
# values
# ---------------------------------------------------------------------------

def laplacian_values(pat: SymPattern, rng: np.random.Generator) -> np.ndarray:
    """Grid-Laplacian value distribution (strictly diagonally dominant).

    Off-diagonals: -U(0.5, 1.5), drawn in storage order.  Diagonal: the sum of
    |off-diagonals| of the row (both triangles) plus U(0.01, 0.1), drawn in
    vertex order.
    """
    off = pat.offdiag_mask()
    vals = np.zeros(pat.nnz, dtype=np.float64)
    noff = int(off.sum())
    vals[off] = -rng.uniform(0.5, 1.5, size=noff)
    rowsum = np.zeros(pat.n, dtype=np.float64)
    np.add.at(rowsum, pat.rows[off], np.abs(vals[off]))
    np.add.at(rowsum, pat.cols[off], np.abs(vals[off]))
    shift = rng.uniform(0.01, 0.1, size=pat.n)
    vals[~off] = (rowsum + shift)[pat.rows[~off]]
    return vals


def rhs(n: int, nrhs: int, rng: np.random.Generator) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=(nrhs, n))


def trimesh_edges_weights(k: int, rng: np.random.Generator):
    """Jittered k x k triangle mesh and its clipped cotangent edge weights.

    Vertex (i, j) sits at (i, j) + U(-0.2, 0.2)^2; every quad is split along
    (i, j)-(i+1, j+1).  The weight of edge (a, b) is half the sum of the
    cotangents of the angles opposite to it, clipped to [0.05, 2].
    Vertex index: i + k*j.
    """
    n = k * k
    pos, tris = trimesh_geometry(k, rng)
    ea, eb, cot = [], [], []
    for c in range(3):
        a = tris[:, (c + 1) % 3]
        b = tris[:, (c + 2) % 3]
        u = pos[a] - pos[tris[:, c]]
        v = pos[b] - pos[tris[:, c]]
        dot = (u * v).sum(1)
        cross = np.abs(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0])
        ea.append(a); eb.append(b); cot.append(dot / cross)
    ea = np.concatenate(ea); eb = np.concatenate(eb); cot = np.concatenate(cot)
    lo = np.minimum(ea, eb); hi = np.maximum(ea, eb)
    key = lo.astype(np.int64) * n + hi
    uk, inv = np.unique(key, return_inverse=True)
    w = np.zeros(uk.size, dtype=np.float64)
    np.add.at(w, inv, 0.5 * cot)
    w = np.clip(w, 0.05, 2.0)
    edges = np.stack([uk // n, uk % n], 1)
    return n, edges, w, pos, tris


def trimesh_geometry(k: int, rng: np.random.Generator):
    """Vertex positions [k*k, 2] ((i, j) + U(-0.2, 0.2)^2, vertex i + k*j)
    and triangles [2 (k-1)^2, 3] of the jittered k x k mesh, every quad
    split along (i, j)-(i+1, j+1)."""
    n = k * k
    jit = rng.uniform(-0.2, 0.2, size=(n, 2))
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    pos = np.stack([ii.ravel(), jj.ravel()], 1).astype(np.float64) + jit
    q = np.arange(k - 1)
    qi, qj = np.meshgrid(q, q, indexing="xy")
    v00 = (qi + k * qj).ravel()
    v10 = v00 + 1
    v11 = v00 + 1 + k
    v01 = v00 + k
    tris = np.concatenate([np.stack([v00, v10, v11], 1),
                           np.stack([v00, v11, v01], 1)], 0)
    return pos, tris


def _stiffness_mass_values(pat: SymPattern, edges: np.ndarray, w: np.ndarray,
                           mass: np.ndarray, mass_scale: float) -> np.ndarray:
    n = pat.n
    # position of each edge (lo, hi) in storage: storage is sorted by (col,row)
    key_store = pat.cols.astype(np.int64) * n + pat.rows
    key_edge = edges[:, 0].astype(np.int64) * n + edges[:, 1]
    pos = np.searchsorted(key_store, key_edge)
    vals = np.zeros(pat.nnz, dtype=np.float64)
    vals[pos] = -w
    deg = np.zeros(n, dtype=np.float64)
    np.add.at(deg, edges[:, 0], w)
    np.add.at(deg, edges[:, 1], w)
    diag = ~pat.offdiag_mask()
    vals[diag] = (deg + mass_scale * mass)[pat.rows[diag]]
    return vals


# ---------------------------------------------------------------------------
# named configurations
# ---------------------------------------------------------------------------

def _streams(seed: int, k: int):
    return np.random.SeedSequence(seed).spawn(k)


def _grid_workload(name: str, dims, order: str, batch: int, nrhs: int,
                   seed: int, rng_vals=None, rng_rhs=None) -> Workload:
    n, e = grid_edges(dims)
    pat = lower_csc_from_edges(n, e)
    perm = grid_nd_perm(dims) if order == "nd" else None
    if rng_vals is None:
        ss = _streams(seed, 4)
        vss = ss[1].spawn(batch)
        rss = ss[2].spawn(batch)
        rng_vals = [np.random.Generator(np.random.PCG64(s)) for s in vss]
        rng_rhs = [np.random.Generator(np.random.PCG64(s)) for s in rss]
    vals = np.stack([laplacian_values(pat, rng_vals[s]) for s in range(batch)])
    b = np.stack([rhs(n, nrhs, rng_rhs[s]) for s in range(batch)])
    return Workload(name=name, pattern=pat, perm=perm, values=vals, b=b,
                    seed=seed, extra={"dims": tuple(dims), "order": order})


def config(idx: int, batch: Optional[int] = None) -> List[Workload] | Workload:
    """The five benchmark configurations (seed = 1000 + idx).

    0: 2D 5-point 32x32, natural order, 1 system, 1 RHS (FP64)
    1: 3D 7-point 64^3, nested dissection, 1 system, 1 RHS (FP64)
    2: jittered 512x512 triangle mesh, cotangent stiffness + 1e-3 * lumped
       mass, 64 value sets (weights re-jittered by U(0.9, 1.1)), 3 RHS each
    3: uneven batch: 2D 16^2, 32^2, 64^2, 128^2 and 3D 8^3, 12^3, 16^3, 24^3,
       32 value sets each (returns a list of 8 workloads)
    4: block vector Laplacian, 3 x 3 rotated SPD blocks on a 40^3 grid
       (n = 192000), 16 value sets, 1 RHS, targets x* ~ N(0, 1) in
       extra["xstar"] for the loss 0.5 ||x - x*||^2
    """
    seed = 1000 + idx
    if idx == 0:
        return _grid_workload("grid2d_32x32_natural", (32, 32), "natural",
                              batch or 1, 1, seed)
    if idx == 1:
        return _grid_workload("grid3d_64^3_nd", (64, 64, 64), "nd",
                              batch or 1, 1, seed)
    if idx == 2:
        return trimesh_workload(512, batch or 64, 3, seed)
    if idx == 3:
        shapes = [(16, 16), (32, 32), (64, 64), (128, 128),
                  (8, 8, 8), (12, 12, 12), (16, 16, 16), (24, 24, 24)]
        ss = _streams(seed, len(shapes))
        out = []
        nb = batch or 32
        for s, dims in enumerate(shapes):
            sub = ss[s].spawn(2)
            rv = [np.random.Generator(np.random.PCG64(c)) for c in sub[0].spawn(nb)]
            rr = [np.random.Generator(np.random.PCG64(c)) for c in sub[1].spawn(nb)]
            name = "grid%dd_%s_nd" % (len(dims), "x".join(map(str, dims)))
            out.append(_grid_workload(name, dims, "nd", nb, 1, seed,
                                      rng_vals=rv, rng_rhs=rr))
        return out
    if idx == 4:
        return block_vector_workload((40, 40, 40), batch or 16, 1, seed)
    raise ValueError("unknown configuration %r" % (idx,))


def trimesh_workload(k: int, batch: int, nrhs: int, seed: int,
                     mass_coeff: float = 1e-3) -> Workload:
    ss = _streams(seed, 4)
    geo = np.random.Generator(np.random.PCG64(ss[0]))
    n, edges, w, pos, tris = trimesh_edges_weights(k, geo)
    mass = geo.uniform(0.5, 1.5, size=n) / n
    pat = lower_csc_from_edges(n, edges)
    vss = ss[1].spawn(batch)
    rss = ss[2].spawn(batch)
    vals = []
    scales = np.empty((batch, w.size))
    for s in range(batch):
        r = np.random.Generator(np.random.PCG64(vss[s]))
        scales[s] = r.uniform(0.9, 1.1, size=w.size)
        ws = np.clip(w * scales[s], 0.05, 2.0)
        vals.append(_stiffness_mass_values(pat, edges, ws, mass, mass_coeff))
    b = np.stack([rhs(n, nrhs, np.random.Generator(np.random.PCG64(s)))
                  for s in rss])
    # the mesh itself, for assembling the values from the geometry: edge e
    # is the e-th stored off-diagonal entry (edges sorted by (lo, hi))
    mesh = {"pos": pos, "tris": tris.astype(np.int32), "mass": mass,
            "mass_coeff": mass_coeff, "edge_scale": scales, "clip": (0.05, 2.0)}
    return Workload(name="trimesh_%dx%d_nd" % (k, k), pattern=pat,
                    perm=grid_nd_perm((k, k)), values=np.stack(vals), b=b,
                    seed=seed, extra={"dims": (k, k), "order": "nd", "mesh": mesh})


def small_grid(dims, order="nd", batch=1, nrhs=1, seed=7) -> Workload:
    """Any grid with the Laplacian value rule; handy for tests."""
    return _grid_workload("grid_%s_%s" % ("x".join(map(str, dims)), order),
                          dims, order, batch, nrhs, seed)


def random_spd(n: int, density: float, seed: int, batch: int = 1,
               nrhs: int = 1, perm: bool = True) -> Workload:
    """Random symmetric pattern with the Laplacian value rule (SPD by strict
    diagonal dominance) and an optional random permutation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = int(round(density * n * (n - 1) / 2))
    if n > 1 and m > 0:
        a = rng.integers(0, n, size=4 * m + 8)
        b = rng.integers(0, n, size=4 * m + 8)
        keep = a != b
        lo = np.minimum(a[keep], b[keep]); hi = np.maximum(a[keep], b[keep])
        key = np.unique(lo.astype(np.int64) * n + hi)[:m]
        rng.shuffle(key)
        key = np.sort(key[:m])
        edges = np.stack([key // n, key % n], 1)
    else:
        edges = np.zeros((0, 2), dtype=np.int64)
    pat = lower_csc_from_edges(n, edges)
    vals = np.stack([laplacian_values(pat, rng) for _ in range(batch)])
    b = np.stack([rhs(n, nrhs, rng) for _ in range(batch)])
    p = rng.permutation(n).astype(np.int32) if perm else None
    return Workload(name="random_%d" % n, pattern=pat, perm=p, values=vals,
                    b=b, seed=seed)


def group_arrays(ws: Sequence[Workload]) -> Tuple[np.ndarray, np.ndarray]:
    """Value sets and right-hand sides of several workloads with the same
    batch and nrhs laid out as one block-diagonal group: set b is the
    concatenation of every pattern's set b, vector (b, r) the concatenation
    of every pattern's vector (b, r), in pattern order."""
    batch, nrhs = ws[0].batch, ws[0].nrhs
    if any(w.batch != batch or w.nrhs != nrhs for w in ws):
        raise ValueError("group members need the same batch and nrhs")
    vals = np.concatenate([w.values for w in ws], axis=1)
    b = np.concatenate([w.b for w in ws], axis=2)
    return np.ascontiguousarray(vals), np.ascontiguousarray(b)


def _rotations(rng: np.random.Generator, m: int) -> np.ndarray:
    """m rotation matrices, uniform on SO(3): normalized Gaussian quaternions."""
    q = rng.standard_normal((m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((m, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def block_vector_workload(dims, batch: int = 1, nrhs: int = 1, seed: int = 1004) -> Workload:
    """Block vector Laplacian: 3 unknowns per grid vertex, 7-point (3D) or
    5-point (2D) stencil of 3 x 3 blocks.

    For every edge (i, j) and value set: B_ij = R diag(U(0.5, 1.5)^3) R^T with
    R uniform on SO(3); the off-diagonal block is A_ij = -B_ij; the diagonal
    block's off-diagonal entries are sums over the neighbours of B's
    off-diagonal entries, negated; every scalar diagonal entry is the sum of
    the absolute off-diagonal entries of its row plus U(0.01, 0.1) (strict
    diagonal dominance, hence SPD).  Unknown 3 v + c belongs to vertex v;
    the permutation is the geometric nested dissection of the vertices with
    each vertex's three unknowns kept together.  extra["xstar"] holds
    targets N(0, 1) [batch, nrhs, n] for the loss 0.5 ||x - x*||^2."""
    nv, e = grid_edges(dims)
    n = 3 * nv
    ei, ej = e[:, 0], e[:, 1]  # ei < ej
    # pattern: lower triangle of every diagonal block and full off-diagonal blocks
    r3, c3 = np.tril_indices(3)
    drow = (3 * np.arange(nv)[:, None] + r3[None, :]).ravel()
    dcol = (3 * np.arange(nv)[:, None] + c3[None, :]).ravel()
    br, bc = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    orow = (3 * ej[:, None] + br.ravel()[None, :]).ravel()  # block row j > block column i
    ocol = (3 * ei[:, None] + bc.ravel()[None, :]).ravel()
    rows = np.concatenate([drow, orow]).astype(np.int64)
    cols = np.concatenate([dcol, ocol]).astype(np.int64)
    order = np.lexsort((rows, cols))
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)
    pat = SymPattern(n=n, colptr=colptr, rowind=rows[order].astype(np.int32),
                     rows=rows[order], cols=cols[order])
    inv = np.empty_like(order)
    inv[order] = np.arange(order.size)  # position in storage of each generated entry
    nd = drow.size
    ss = _streams(seed, 4)
    vss = ss[1].spawn(batch)
    rss = ss[2].spawn(batch)
    xss = ss[3].spawn(batch)
    vals = np.zeros((batch, pat.nnz))
    for s in range(batch):
        g = np.random.Generator(np.random.PCG64(vss[s]))
        R = _rotations(g, ei.size)
        dd = g.uniform(0.5, 1.5, size=(ei.size, 3))
        B = np.einsum("eab,eb,ecb->eac", R, dd, R)  # R diag(d) R^T per edge
        D = np.zeros((nv, 3, 3))
        np.add.at(D, ei, B)
        np.add.at(D, ej, B)
        # scalar row sums of |off-diagonal| entries (both triangles)
        rs = np.zeros(n)
        absB = np.abs(B)
        np.add.at(rs, (3 * ei[:, None] + np.arange(3)).ravel(), absB.sum(2).ravel())
        np.add.at(rs, (3 * ej[:, None] + np.arange(3)).ravel(), absB.sum(1).ravel())
        Dm = -D  # diagonal blocks: negated sums of the neighbours' blocks
        offd = np.abs(Dm) * (1 - np.eye(3))[None]
        rs += offd.sum(2).ravel()
        shift = g.uniform(0.01, 0.1, size=n)
        diag = rs + shift
        Dm[:, np.arange(3), np.arange(3)] = diag.reshape(nv, 3)
        v = np.empty(pat.nnz)
        v[inv[:nd]] = Dm[:, r3, c3].ravel()
        v[inv[nd:]] = (-B[:, br.ravel(), bc.ravel()]).ravel()
        vals[s] = v
    b = np.stack([rhs(n, nrhs, np.random.Generator(np.random.PCG64(q))) for q in rss])
    xstar = np.stack([np.random.Generator(np.random.PCG64(q)).standard_normal((nrhs, n))
                      for q in xss])
    vperm = grid_nd_perm(dims)
    perm = (3 * vperm.astype(np.int64)[:, None] + np.arange(3)[None, :]).ravel().astype(np.int32)
    name = "blockvec3_%s_nd" % "x".join(map(str, dims))
    return Workload(name=name, pattern=pat, perm=perm, values=vals, b=b, seed=seed,
                    extra={"dims": tuple(dims), "order": "nd", "xstar": xstar})
