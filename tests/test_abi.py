"""C-ABI checks that need no GPU: the library loads and exports every
function the header declares, input validation returns the documented
status codes, and the host symbolic pass (sc_analyze) matches the oracle's
elimination tree and pattern bit for bit and satisfies the supernode and
level invariants the GPU schedule relies on."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    """Every function declared by the headers under include/."""
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(sc_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_function():
    import paper_2110_12865_amd as S
    names = header_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(S.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    from paper_2110_12865_amd import mesh, products
    assert sorted(S.EXPORTS + mesh.EXPORTS + products.EXPORTS) == names


def test_status_strings():
    import paper_2110_12865_amd as S
    for st in range(-6, 1):
        assert S.status_string(st)


def _analyze_raw(n, colptr, rowind, perm=None):
    import paper_2110_12865_amd as S
    colptr = np.ascontiguousarray(colptr, np.int64)
    rowind = np.ascontiguousarray(rowind, np.int32)
    h = ctypes.c_void_p()
    p = None if perm is None else np.ascontiguousarray(perm, np.int32)
    st = S._lib.sc_analyze(n, S._ptr(colptr), S._ptr(rowind), S._ptr(p), None, ctypes.byref(h))
    if h:
        S._lib.sc_plan_destroy(h)
    return st


def test_malformed_patterns_are_rejected():
    import paper_2110_12865_amd as S
    w = W.small_grid((4, 3), "natural")
    cp, ri = w.pattern.colptr.copy(), w.pattern.rowind.copy()
    n = w.pattern.n
    assert _analyze_raw(n, cp, ri) == S.SC_OK
    # diagonal missing / not first
    bad = ri.copy(); bad[cp[2]] = bad[cp[2] + 1]
    assert _analyze_raw(n, cp, bad) == S.SC_EPATTERN
    # unsorted rows
    bad = ri.copy(); c = 1
    bad[cp[c] + 1], bad[cp[c] + 2] = bad[cp[c] + 2], bad[cp[c] + 1]
    assert _analyze_raw(n, cp, bad) == S.SC_EPATTERN
    # duplicate row
    bad = ri.copy(); bad[cp[1] + 2] = bad[cp[1] + 1]
    assert _analyze_raw(n, cp, bad) == S.SC_EPATTERN
    # row out of range
    bad = ri.copy(); bad[cp[n - 2] + 1] = n
    assert _analyze_raw(n, cp, bad) == S.SC_EPATTERN
    # an entry above the diagonal
    bad = ri.copy(); bad[cp[5] + 1] = 4
    assert _analyze_raw(n, cp, bad) == S.SC_EPATTERN
    # colptr not monotone / not starting at 0
    badc = cp.copy(); badc[3] = badc[2]
    assert _analyze_raw(n, badc, ri) == S.SC_EPATTERN
    badc = cp.copy(); badc[0] = 1
    assert _analyze_raw(n, badc, ri) == S.SC_EPATTERN
    # perm: duplicate and out-of-range entries
    perm = np.arange(n, dtype=np.int32); perm[3] = perm[4]
    assert _analyze_raw(n, cp, ri, perm) == S.SC_EPATTERN
    perm = np.arange(n, dtype=np.int32); perm[0] = n
    assert _analyze_raw(n, cp, ri, perm) == S.SC_EPATTERN
    # sizes and null pointers
    assert _analyze_raw(0, np.zeros(1, np.int64), np.zeros(0, np.int32)) == S.SC_EINVAL
    h = ctypes.c_void_p()
    assert S._lib.sc_analyze(n, None, S._ptr(ri), None, None, ctypes.byref(h)) == S.SC_EINVAL
    assert S._lib.sc_analyze(n, S._ptr(cp), S._ptr(ri), None, None, None) == S.SC_EINVAL


def symbolic_cases():
    out = [("cfg0", W.config(0)),
           ("grid3d_16_nd", W.small_grid((16, 16, 16), "nd")),
           ("grid2d_50x37_nd", W.small_grid((50, 37), "nd")),
           ("grid3d_7x9x5_natural", W.small_grid((7, 9, 5), "natural")),
           ("trimesh_40", W.trimesh_workload(40, 1, 1, seed=5))]
    for seed in range(6):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 400))
        out.append(("random_%d" % seed,
                    W.random_spd(n, float(rng.uniform(0.0, 0.05)), seed=900 + seed)))
    return out


@pytest.mark.parametrize("name,w", symbolic_cases(), ids=[c[0] for c in symbolic_cases()])
@pytest.mark.parametrize("relax", [1, 0])
def test_symbolic_bit_exact_and_invariants(name, w, relax):
    import paper_2110_12865_amd as S
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm, relax=relax)
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    perm, parent, Lcolptr, Lrowind = plan.export_symbolic()
    if w.perm is not None:
        assert np.array_equal(perm, w.perm)
    else:
        assert np.array_equal(perm, np.arange(p.n))
    assert np.array_equal(parent, sym.parent)
    assert np.array_equal(Lcolptr, sym.Lcolptr)
    assert np.array_equal(Lrowind, sym.Lrowind)
    inf = plan.info()
    assert inf["nnzL"] == sym.nnzL
    assert inf["flops"] == pytest.approx(sym.flops(), rel=1e-12)
    check_supernode_invariants(plan, sym)


def check_supernode_invariants(plan, sym):
    first, sparent, level, rowptr, rows = plan.export_supernodes()
    n = sym.n
    ns = len(sparent)
    assert first[0] == 0 and first[-1] == n and np.all(np.diff(first) > 0)
    col2sn = np.repeat(np.arange(ns), np.diff(first))
    for s in range(ns):
        R = rows[rowptr[s]:rowptr[s + 1]]
        w = first[s + 1] - first[s]
        assert np.array_equal(R[:w], np.arange(first[s], first[s + 1]))
        assert np.all(np.diff(R) > 0)
        # every exact column structure of the supernode lies inside R
        for j in (first[s], first[s + 1] - 1):
            ex = sym.Lrowind[sym.Lcolptr[j]:sym.Lcolptr[j + 1]]
            assert np.all(np.isin(ex, R))
        p = sparent[s]
        last = first[s + 1] - 1
        if sym.parent[last] < 0:
            assert p == -1 and len(R) == w
        else:
            assert p == col2sn[sym.parent[last]]
            assert level[p] > level[s]          # strictly lower level
            Rp = rows[rowptr[p]:rowptr[p + 1]]
            assert np.all(np.isin(R[w:], Rp))    # update rows land in the parent
        # every column but the last has its etree parent inside the
        # supernode (a chain for fundamental supernodes; amalgamation may
        # attach a child's last column anywhere inside its parent)
        for j in range(first[s], last):
            assert first[s] < sym.parent[j] <= last
    # levels: leaves at 0, every level non-empty
    assert level.min() == 0
    assert set(np.unique(level)) == set(range(level.max() + 1))


def test_workload_sizes_and_fill_match_oracle():
    """nnz(A) of the 32x32 grid and of the 512x512 mesh, and nnz(L) of both
    (the generator and the analysis agree with the independent oracle)."""
    import paper_2110_12865_amd as S
    for idx, nnzA in ((0, 3008), (2, 1046529)):
        w = W.config(idx, batch=1)
        p = w.pattern
        assert p.nnz == nnzA
        plan = S.analyze(p.colptr, p.rowind, w.perm)
        sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
        assert plan.info()["nnzL"] == sym.nnzL


def test_options_validation():
    import paper_2110_12865_amd as S
    w = W.small_grid((5, 5), "nd")
    p = w.pattern
    with pytest.raises(S.SpcholError):
        S.analyze(p.colptr, p.rowind, w.perm, relax_zeros=-1.0)
    with pytest.raises(S.SpcholError):
        S.analyze(p.colptr, p.rowind, w.perm, small_front=-3)


def test_cotan_create_rejects_bad_meshes():
    """sc_cotan_create validates the mesh against the pattern before any
    device work: a stored entry that is no mesh edge, a mesh edge that is
    not stored, an edge of three triangles, a vertex out of range and a
    degenerate triangle are SC_EPATTERN."""
    import paper_2110_12865_amd as S
    from paper_2110_12865_amd.mesh import CotanAssembly
    tris = np.array([[0, 1, 2], [1, 3, 2]], np.int32)
    edges = np.array([[0, 1], [0, 2], [1, 2], [1, 3], [2, 3]])
    pat = W.lower_csc_from_edges(4, edges)
    bad = {
        "extra_entry": (W.lower_csc_from_edges(4, np.vstack([edges, [[0, 3]]])), tris),
        "missing_edge": (W.lower_csc_from_edges(4, edges[:4]), tris),
        "three_triangles": (W.lower_csc_from_edges(5, np.vstack([edges, [[1, 4], [2, 4]]])),
                            np.array([[0, 1, 2], [1, 3, 2], [1, 2, 4]], np.int32)),
        "out_of_range": (pat, np.array([[0, 1, 2], [1, 4, 2]], np.int32)),
        "degenerate": (pat, np.array([[0, 1, 2], [1, 1, 2]], np.int32)),
    }
    # in the three-triangle case edge (1, 2) has the corners 0, 3 and 4
    for name, (p, t) in bad.items():
        with pytest.raises(S.SpcholError) as ei:
            CotanAssembly(p.n, p.colptr, p.rowind, t)
        assert ei.value.status == S.SC_EPATTERN, name


def _csr_random(rng, rows, cols, per_row):
    rp, ci = [0], []
    for _ in range(rows):
        ci.extend(np.sort(rng.choice(cols, size=min(per_row, cols), replace=False)).tolist())
        rp.append(len(ci))
    return np.array(rp, np.int64), np.array(ci, np.int32)


@pytest.mark.parametrize("transB,with_d", [(False, False), (True, False), (False, True),
                                           (True, True)])
def test_product_pattern_bit_exact(transB, with_d):
    """The host pass of sc_spprod_create: C's pattern equals the oracle's
    structural pattern of A B (A B^T) union D, entry for entry, and the term
    count equals the number of (k) pairs."""
    from paper_2110_12865_amd.products import SparseProduct
    rng = np.random.default_rng(40 + 2 * transB + with_d)
    m, p, n = 37, 29, 31
    A = _csr_random(rng, m, p, 5)
    B = _csr_random(rng, n, p, 4) if transB else _csr_random(rng, p, n, 4)
    D = _csr_random(rng, m, n, 3) if with_d else None
    pr = SparseProduct(m, p, n, A, B, transB, D)
    rp, ci = oracle.sparse_product_pattern(m, n, A[0], A[1], B[0], B[1], transB,
                                           *(D if with_d else (None, None)))
    assert np.array_equal(pr.rowptr, rp)
    assert np.array_equal(pr.colind, ci)
    Ad = np.zeros((m, p), int)
    for i in range(m):
        Ad[i, A[1][A[0][i]:A[0][i + 1]]] = 1
    Bd = np.zeros((n, p) if transB else (p, n), int)
    for i in range(Bd.shape[0]):
        Bd[i, B[1][B[0][i]:B[0][i + 1]]] = 1
    assert pr.nterms == int((Ad @ (Bd.T if transB else Bd)).sum())


def test_product_rejects_bad_patterns():
    import paper_2110_12865_amd as S
    from paper_2110_12865_amd.products import SparseProduct
    A = (np.array([0, 2, 3], np.int64), np.array([1, 0, 1], np.int32))   # row 0 unsorted
    B = (np.array([0, 1, 2], np.int64), np.array([0, 1], np.int32))
    with pytest.raises(S.SpcholError) as ei:
        SparseProduct(2, 2, 2, A, B)
    assert ei.value.status == S.SC_EPATTERN
    A = (np.array([0, 1, 2], np.int64), np.array([0, 2], np.int32))      # column out of range
    with pytest.raises(S.SpcholError) as ei:
        SparseProduct(2, 2, 2, A, B)
    assert ei.value.status == S.SC_EPATTERN


@pytest.mark.parametrize("name,w", [
    ("grid3d_12^3", W.small_grid((12, 12, 12), "nd", seed=61)),
    ("grid2d_40x30", W.small_grid((40, 30), "nd", seed=62)),
    ("trimesh_30", W.trimesh_workload(30, batch=1, nrhs=1, seed=63)),
    ("random_300", W.random_spd(300, 0.02, seed=64)),
    ("disconnected", W.random_spd(200, 0.0, seed=65)),
], ids=lambda x: x if isinstance(x, str) else "")
def test_builtin_nd_ordering_valid(name, w):
    """ordering = nd: the plan's permutation is a permutation of 0..n-1, the
    symbolic result equals the oracle's under that permutation bit for bit
    (parity unpinned for the ordering itself: it has no single right
    answer), and on grids its fill stays within 1.25x of the geometric
    nested dissection."""
    import paper_2110_12865_amd as S
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, None, ordering="nd")
    perm, parent, Lcolptr, Lrowind = plan.export_symbolic()
    assert np.array_equal(np.sort(perm), np.arange(p.n))
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, perm)
    assert np.array_equal(parent, sym.parent)
    assert np.array_equal(Lcolptr, sym.Lcolptr)
    assert np.array_equal(Lrowind, sym.Lrowind)
    if w.perm is not None:
        geo = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
        assert sym.nnzL <= 1.25 * geo.nnzL
    nat = oracle.symbolic(p.n, p.colptr, p.rowind, None)
    assert sym.nnzL <= nat.nnzL


def test_ordering_option_rules():
    """natural ignores nothing: it equals no permutation; a permutation
    together with natural or nd ordering is SC_EINVAL; group plans order
    every pattern on its own."""
    import paper_2110_12865_amd as S
    w = W.small_grid((9, 8), "nd", seed=66)
    p = w.pattern
    a = S.analyze(p.colptr, p.rowind, None, ordering="natural").export_symbolic()
    b = S.analyze(p.colptr, p.rowind, None).export_symbolic()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    for o in ("natural", "nd"):
        with pytest.raises(S.SpcholError) as ei:
            S.analyze(p.colptr, p.rowind, w.perm, ordering=o)
        assert ei.value.status == S.SC_EINVAL
    w2 = W.small_grid((5, 5, 5), "nd", seed=67)
    g = S.analyze_group([(p.colptr, p.rowind, None), (w2.pattern.colptr, w2.pattern.rowind, None)],
                        ordering="nd")
    gperm = g.export_symbolic()[0]
    one = S.analyze(p.colptr, p.rowind, None, ordering="nd").export_symbolic()[0]
    two = S.analyze(w2.pattern.colptr, w2.pattern.rowind, None, ordering="nd").export_symbolic()[0]
    assert np.array_equal(gperm, np.concatenate([one, two + p.n]))
