"""Pins for the CPU oracle, against results fixed by mathematics rather than
by the oracle itself: dense LAPACK Cholesky (numpy), closed forms of the 1D
Laplacian, exact results on diagonal matrices, brute-force dense boolean
elimination for the pattern, and the closed-form fill count of the natural
5-point grid.  None of these tests needs a GPU."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def brute_symbolic(n, colptr, rowind, perm=None):
    """Dense boolean elimination: eliminating k joins all its later
    neighbours into a clique (structural fill, nothing cancels)."""
    B = np.zeros((n, n), dtype=bool)
    for c in range(n):
        for p in range(colptr[c], colptr[c + 1]):
            r = int(rowind[p])
            B[r, c] = B[c, r] = True
    if perm is not None:
        perm = np.asarray(perm, np.int64)
        B = B[np.ix_(perm, perm)]
    for k in range(n):
        rows = np.nonzero(B[k + 1:, k])[0] + k + 1
        if rows.size:
            B[np.ix_(rows, rows)] = True
    parent = np.full(n, -1, dtype=np.int32)
    Lcolptr = [0]
    Lrowind = []
    for j in range(n):
        rows = np.nonzero(B[j:, j])[0] + j
        below = rows[rows > j]
        if below.size:
            parent[j] = below.min()
        Lrowind.extend(rows.tolist())
        Lcolptr.append(len(Lrowind))
    return parent, np.array(Lcolptr, np.int64), np.array(Lrowind, np.int32)


def path_laplacian(n):
    """tridiag(-1, 2, -1) in lower CSC."""
    e = np.stack([np.arange(n - 1), np.arange(1, n)], 1)
    pat = W.lower_csc_from_edges(n, e)
    vals = np.where(pat.rows == pat.cols, 2.0, -1.0)
    return pat, vals


def spd_cases():
    out = []
    for seed, (n, dens) in enumerate([(1, 0.0), (2, 1.0), (5, 0.5), (17, 0.2),
                                      (40, 0.08), (64, 0.05), (64, 0.3)]):
        out.append(W.random_spd(n, dens, seed=100 + seed, perm=True))
    out.append(W.small_grid((6, 5), order="natural", seed=3))
    out.append(W.small_grid((4, 4, 3), order="nd", seed=4))
    out.append(W.small_grid((7, 9), order="nd", seed=5))
    return out


@pytest.mark.parametrize("case", spd_cases(), ids=lambda w: "%s_n%d" % (w.name, w.pattern.n))
def test_symbolic_matches_brute_force(case):
    p = case.pattern
    s = oracle.symbolic(p.n, p.colptr, p.rowind, case.perm)
    parent, Lcolptr, Lrowind = brute_symbolic(p.n, p.colptr, p.rowind, case.perm)
    assert np.array_equal(s.parent, parent)
    assert np.array_equal(s.Lcolptr, Lcolptr)
    assert np.array_equal(s.Lrowind, Lrowind)


@pytest.mark.parametrize("seed", range(6))
def test_symbolic_random_patterns_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 120))
    w = W.random_spd(n, float(rng.uniform(0.01, 0.1)), seed=500 + seed, perm=True)
    p = w.pattern
    s = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    parent, Lcolptr, Lrowind = brute_symbolic(p.n, p.colptr, p.rowind, w.perm)
    assert np.array_equal(s.parent, parent)
    assert np.array_equal(s.Lcolptr, Lcolptr)
    assert np.array_equal(s.Lrowind, Lrowind)
    # column counts never grow by more than one up the tree
    c = s.counts
    for j in range(n):
        if s.parent[j] >= 0:
            assert c[j] <= c[s.parent[j]] + 1


def test_natural_grid_fill_closed_form():
    """Natural order k x k 5-point grid: the band fills completely, so
    nnz(L) = 1 + 2(k-1) + (n-k)(k+1) and the etree is a chain."""
    for k in (3, 8, 32):
        w = W.small_grid((k, k), order="natural")
        p = w.pattern
        s = oracle.symbolic(p.n, p.colptr, p.rowind, None)
        n = k * k
        assert s.nnzL == 1 + 2 * (k - 1) + (n - k) * (k + 1)
        assert np.array_equal(s.parent[:-1], np.arange(1, n))
        assert s.parent[-1] == -1
    w = W.config(0)
    s = oracle.symbolic(w.pattern.n, w.pattern.colptr, w.pattern.rowind, w.perm)
    assert s.nnzL == 32799


@pytest.mark.parametrize("case", spd_cases(), ids=lambda w: "%s_n%d" % (w.name, w.pattern.n))
def test_factor_matches_lapack(case):
    p = case.pattern
    s = oracle.symbolic(p.n, p.colptr, p.rowind, case.perm)
    Lx, info = oracle.factor(p.n, p.colptr, p.rowind, case.values[0], s)
    assert info == 0
    A = oracle.to_dense_permuted(p.n, p.colptr, p.rowind, case.values[0], case.perm)
    Lref = np.linalg.cholesky(A)
    L = oracle.L_dense(s, Lx)
    scale = np.abs(Lref).max()
    assert np.abs(L - Lref).max() <= 1e-13 * scale
    # the structural pattern holds every nonzero of the dense factor
    assert np.all(np.abs(Lref[L == 0]) <= 1e-13 * scale)


@pytest.mark.parametrize("n", [1, 2, 7, 100, 1000])
def test_path_laplacian_closed_form(n):
    """tridiag(-1,2,-1): L_kk = sqrt((k+1)/k), L_{k+1,k} = -sqrt(k/(k+1))
    (1-based), prod L_kk = sqrt(n+1); with b = 1, x_i = i(n+1-i)/2."""
    pat, vals = path_laplacian(n)
    s = oracle.symbolic(n, pat.colptr, pat.rowind, None)
    Lx, info = oracle.factor(n, pat.colptr, pat.rowind, vals, s)
    assert info == 0
    k = np.arange(1, n + 1, dtype=np.float64)
    diag = Lx[s.Lcolptr[:-1]]
    assert np.allclose(diag, np.sqrt((k + 1) / k), rtol=1e-14, atol=0)
    if n > 1:
        sub = Lx[s.Lcolptr[:-2] + 1]
        assert np.allclose(sub, -np.sqrt(k[:-1] / (k[:-1] + 1)), rtol=1e-14, atol=0)
    assert math.isclose(float(np.prod(diag)), math.sqrt(n + 1), rel_tol=1e-12)
    x = oracle.solve(s, Lx, np.ones(n))
    assert np.allclose(x, k * (n + 1 - k) / 2, rtol=1e-11, atol=0)


def test_path_laplacian_inverse_closed_form():
    """A^{-1}_ij = min(i,j)(n+1-max(i,j))/(n+1) (1-based)."""
    n = 12
    pat, vals = path_laplacian(n)
    s = oracle.symbolic(n, pat.colptr, pat.rowind, None)
    Lx, _ = oracle.factor(n, pat.colptr, pat.rowind, vals, s)
    Ainv = oracle.solve(s, Lx, np.eye(n))
    i = np.arange(1, n + 1)[:, None]
    j = np.arange(1, n + 1)[None, :]
    ref = np.minimum(i, j) * (n + 1 - np.maximum(i, j)) / (n + 1)
    assert np.abs(Ainv - ref).max() <= 1e-13


def test_diagonal_matrix_exact():
    n = 50
    rng = np.random.default_rng(1)
    pat = W.lower_csc_from_edges(n, np.zeros((0, 2)))
    d = rng.uniform(0.1, 10, n)
    perm = rng.permutation(n).astype(np.int32)
    s = oracle.symbolic(n, pat.colptr, pat.rowind, perm)
    assert np.all(s.parent == -1)
    Lx, info = oracle.factor(n, pat.colptr, pat.rowind, d, s)
    assert info == 0
    assert np.array_equal(Lx, np.array([math.sqrt(v) for v in d[perm]]))
    b = rng.uniform(-1, 1, n)
    x = oracle.solve(s, Lx, b)
    assert np.allclose(x, b / d, rtol=4e-16 * 4, atol=0)


def test_not_spd_reports_first_failed_step():
    n = 30
    pat, vals = path_laplacian(n)
    for p in (0, 1, 9, 29):
        v = vals.copy()
        v[pat.colptr[p]] = 0.4  # pivot p becomes 0.4 - p/(p+1) < 0 for p >= 1
        if p == 0:
            v[pat.colptr[p]] = -1.0
        s = oracle.symbolic(n, pat.colptr, pat.rowind, None)
        _, info = oracle.factor(n, pat.colptr, pat.rowind, v, s)
        assert info == p + 1
    # NaN on the diagonal fails the d > 0 test as well
    v = vals.copy(); v[pat.colptr[4]] = np.nan
    _, info = oracle.factor(n, pat.colptr, pat.rowind, v, s)
    assert info == 5
    # with a permutation the step is counted in elimination order
    perm = np.arange(n)[::-1].astype(np.int32)
    v = vals.copy(); v[pat.colptr[n - 1]] = -3.0  # vertex n-1 is eliminated first
    s = oracle.symbolic(n, pat.colptr, pat.rowind, perm)
    _, info = oracle.factor(n, pat.colptr, pat.rowind, v, s)
    assert info == 1


def test_disconnected_pattern_is_blockwise():
    a = W.small_grid((5, 4), order="nd", seed=11)
    b = W.small_grid((3, 3, 2), order="nd", seed=12)
    na, nb = a.pattern.n, b.pattern.n
    ea = np.stack([a.pattern.rows, a.pattern.cols], 1)[a.pattern.offdiag_mask()]
    eb = np.stack([b.pattern.rows, b.pattern.cols], 1)[b.pattern.offdiag_mask()] + na
    pat = W.lower_csc_from_edges(na + nb, np.concatenate([ea, eb]))
    # values: copy through (row, col) keys
    va = dict(zip(zip(a.pattern.rows.tolist(), a.pattern.cols.tolist()), a.values[0]))
    vb = dict(zip(zip((b.pattern.rows + na).tolist(), (b.pattern.cols + na).tolist()), b.values[0]))
    va.update(vb)
    vals = np.array([va[(r, c)] for r, c in zip(pat.rows.tolist(), pat.cols.tolist())])
    perm = np.concatenate([a.perm, b.perm + na]).astype(np.int32)
    s = oracle.symbolic(pat.n, pat.colptr, pat.rowind, perm)
    assert int(np.sum(s.parent == -1)) >= 2
    Lx, info = oracle.factor(pat.n, pat.colptr, pat.rowind, vals, s)
    assert info == 0
    sa = oracle.symbolic(na, a.pattern.colptr, a.pattern.rowind, a.perm)
    La, _ = oracle.factor(na, a.pattern.colptr, a.pattern.rowind, a.values[0], sa)
    sb = oracle.symbolic(nb, b.pattern.colptr, b.pattern.rowind, b.perm)
    Lb, _ = oracle.factor(nb, b.pattern.colptr, b.pattern.rowind, b.values[0], sb)
    assert np.array_equal(Lx, np.concatenate([La, Lb]))


def test_residual_and_reconstruction_invariants():
    w = W.config(0)
    p = w.pattern
    s = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[0], s)
    assert info == 0
    A = oracle.to_dense_permuted(p.n, p.colptr, p.rowind, w.values[0], w.perm)
    L = oracle.L_dense(s, Lx)
    cmax = int(s.counts.max())
    assert np.linalg.norm(A - L @ L.T) <= 1e-14 * math.sqrt(cmax) * np.linalg.norm(A)
    # strict diagonal dominance survives every Schur complement
    assert np.all(Lx[s.Lcolptr[:-1]] ** 2 >= 0.01)
    x = oracle.solve(s, Lx, w.b[0])
    relres, eta = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[0], x, w.b[0])
    assert relres[0] < 1e-13 and eta[0] < 1e-15
    # spmv against the dense product
    assert np.allclose(oracle.spmv(p.n, p.colptr, p.rowind, w.values[0], x[0]),
                       oracle.to_dense_permuted(p.n, p.colptr, p.rowind, w.values[0]) @ x[0],
                       rtol=0, atol=1e-12)


def test_solution_independent_of_permutation():
    w = W.small_grid((9, 8), order="natural", seed=21, nrhs=2)
    p = w.pattern
    xs = []
    for perm in (None, W.grid_nd_perm((9, 8)),
                 np.random.default_rng(0).permutation(p.n).astype(np.int32)):
        s = oracle.symbolic(p.n, p.colptr, p.rowind, perm)
        Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[0], s)
        assert info == 0
        xs.append(oracle.solve(s, Lx, w.b[0]))
    for x in xs[1:]:
        assert oracle.forward_error(x, xs[0]) < 1e-13


def test_leading_block_is_cholesky_of_leading_submatrix():
    """Rows < m of L are the factor of the leading m x m block of P A P^T."""
    w = W.small_grid((6, 6, 2), order="nd", seed=31)
    p = w.pattern
    A = oracle.to_dense_permuted(p.n, p.colptr, p.rowind, w.values[0], w.perm)
    for m in (1, 17, 40, p.n):
        s = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm, nrows=m)
        Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[0], s)
        assert info == 0
        L = oracle.L_dense(s, Lx)
        Lref = np.linalg.cholesky(A[:m, :m])
        assert np.abs(L[:m, :m] - Lref).max() <= 1e-13 * np.abs(Lref).max()
        assert np.all(L[m:, :] == 0)


def test_multiple_rhs_columns_are_independent():
    w = W.small_grid((5, 5, 3), order="nd", seed=41, nrhs=3)
    p = w.pattern
    s = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    Lx, _ = oracle.factor(p.n, p.colptr, p.rowind, w.values[0], s)
    X = oracle.solve(s, Lx, w.b[0])
    for r in range(3):
        assert np.array_equal(X[r], oracle.solve(s, Lx, w.b[0][r]))
    A = oracle.to_dense_permuted(p.n, p.colptr, p.rowind, w.values[0])
    assert np.allclose(np.linalg.solve(A, w.b[0].T).T, X, rtol=0, atol=1e-12)


def test_golden_fixture_reproduces():
    """tests/golden/grid2d_4x4_nd.txt was written by make_golden.py, which
    calls only the oracle; a change of the oracle's arithmetic shows here."""
    import os
    from tests.golden.make_golden import case_grid2d_4x4, read_fixture
    path = os.path.join(os.path.dirname(__file__), "golden", "grid2d_4x4_nd.txt")
    fx = read_fixture(path)
    w = case_grid2d_4x4()
    p = w.pattern
    s = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    Lx, _ = oracle.factor(p.n, p.colptr, p.rowind, w.values[0], s)
    x = oracle.solve(s, Lx, w.b[0])
    assert np.array_equal(s.Lcolptr, fx["Lcolptr"])
    assert np.array_equal(s.Lrowind, fx["Lrowind"])
    assert np.array_equal(Lx, fx["Lx"])
    assert np.array_equal(x.ravel(), fx["x"])


# ---------------------------------------------------------------------------
# gradients through the solve (loss 0.5 ||x - x*||^2)


def _loss_and_grad(p, perm, vals, b, xstar):
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, perm)
    Lx, info = oracle.factor(p.n, p.colptr, p.rowind, vals, sym)
    assert info == 0
    x = oracle.solve(sym, Lx, b)
    loss = 0.5 * float(np.sum((x - xstar) ** 2))
    gv, gb = oracle.solve_gradients(p.n, p.colptr, p.rowind, vals, sym, Lx, x, x - xstar)
    return loss, gv, gb


def test_gradients_match_central_differences():
    """Pin: central differences of the loss, h = 1e-6 max(1, |v|), on 40
    value entries (diagonal and off-diagonal) and on every entry of b."""
    w = W.block_vector_workload((3, 3, 2), batch=1, nrhs=2, seed=71)
    p = w.pattern
    xs = w.extra["xstar"][0]
    v0, b0 = w.values[0], w.b[0]
    loss, gv, gb = _loss_and_grad(p, w.perm, v0, b0, xs)
    rng = np.random.default_rng(3)
    ks = rng.choice(p.nnz, size=40, replace=False)
    for k in ks:
        h = 1e-6 * max(1.0, abs(v0[k]))
        vp, vm = v0.copy(), v0.copy()
        vp[k] += h
        vm[k] -= h
        fd = (_loss_and_grad(p, w.perm, vp, b0, xs)[0] - _loss_and_grad(p, w.perm, vm, b0, xs)[0]) / (2 * h)
        assert abs(fd - gv[k]) <= 1e-6 * max(1.0, abs(gv[k]))
    for r in range(b0.shape[0]):
        for i in range(0, p.n, 5):
            bp, bm = b0.copy(), b0.copy()
            bp[r, i] += 1e-6
            bm[r, i] -= 1e-6
            fd = (_loss_and_grad(p, w.perm, v0, bp, xs)[0] - _loss_and_grad(p, w.perm, v0, bm, xs)[0]) / 2e-6
            assert abs(fd - gb[r, i]) <= 1e-6 * max(1.0, abs(gb[r, i]))


def test_gradients_1d_laplacian_closed_form():
    """Pin: for A = tridiag(-1, 2, -1) the inverse is known in closed form,
    A^{-1}_ij = min(i, j) (n + 1 - max(i, j)) / (n + 1) (1-based), so
    x = A^{-1} b, lambda = A^{-1} g and the value gradients -lambda_i x_j -
    lambda_j x_i (off-diagonal), -lambda_i x_i (diagonal) follow without any
    factorization."""
    n = 9
    e = np.stack([np.arange(n - 1), np.arange(1, n)], 1)
    p = W.lower_csc_from_edges(n, e)
    vals = np.where(p.rows == p.cols, 2.0, -1.0)
    rng = np.random.default_rng(4)
    b = rng.uniform(-1, 1, size=(1, n))
    g = rng.uniform(-1, 1, size=(1, n))
    i1 = np.arange(1, n + 1)
    Ainv = np.minimum.outer(i1, i1) * (n + 1 - np.maximum.outer(i1, i1)) / (n + 1)
    x = b @ Ainv
    lam = g @ Ainv
    sym = oracle.symbolic(n, p.colptr, p.rowind, None)
    Lx, info = oracle.factor(n, p.colptr, p.rowind, vals, sym)
    gv, gb = oracle.solve_gradients(n, p.colptr, p.rowind, vals, sym, Lx, x, g)
    assert np.allclose(gb, lam, rtol=0, atol=1e-13)
    ref = np.where(p.rows == p.cols, -lam[0, p.rows] * x[0, p.cols],
                   -(lam[0, p.rows] * x[0, p.cols] + lam[0, p.cols] * x[0, p.rows]))
    assert np.allclose(gv, ref, rtol=0, atol=1e-13)


def test_block_vector_generator_is_spd_and_dominant():
    """The block-vector systems are symmetric, strictly diagonally dominant
    (hence SPD), with 3 x 3 blocks; the 40^3 size has nnz(A) = 2,068,800."""
    w = W.block_vector_workload((3, 3, 3), batch=2, nrhs=1, seed=72)
    p = w.pattern
    A = np.zeros((p.n, p.n))
    A[p.rows, p.cols] = w.values[1]
    A[p.cols, p.rows] = w.values[1]
    off = np.abs(A).sum(1) - np.abs(np.diag(A))
    assert np.all(np.diag(A) - off >= 0.01 - 1e-12)
    assert np.linalg.eigvalsh(A).min() > 0
    assert p.nnz == 27 * 6 + 3 * 3 * 3 * 2 * 9  # 6 per diagonal block, 9 per edge
    nv, e = W.grid_edges((40, 40, 40))
    assert 6 * nv + 9 * len(e) == 2068800


# --- error measures, norms and the stop rule: hand-computed cases ----------

def _lower_csc(dense):
    """Lower CSC (diagonal first, rows ascending) of a small symmetric matrix,
    every lower entry stored (explicit zeros included)."""
    n = dense.shape[0]
    colptr, rowind, vals = [0], [], []
    for c in range(n):
        for r in range(c, n):
            rowind.append(r)
            vals.append(dense[r, c])
        colptr.append(len(rowind))
    return (np.array(colptr, np.int64), np.array(rowind, np.int32),
            np.array(vals, np.float64))


def test_norm_inf_sym_hand():
    # |2| + |-3| = 5 in row 0; |-3| + |1| = 4 in row 1.  Reading only the
    # stored lower triangle would give row 0 = 2 and ||A|| = 4.
    cp, ri, v = _lower_csc(np.array([[2.0, -3.0], [-3.0, 1.0]]))
    assert oracle.norm_inf_sym(2, cp, ri, v) == 5.0
    A = np.array([[4.0, 1.0, 0.0], [1.0, 3.0, -1.0], [0.0, -1.0, 2.0]])
    cp, ri, v = _lower_csc(A)
    assert oracle.norm_inf_sym(3, cp, ri, v) == 5.0
    # a 4x4 whose largest row is the last one (an index slip shows)
    B = np.array([[1.0, 0.0, 0.0, -2.0], [0.0, 1.0, 0.5, 0.0],
                  [0.0, 0.5, 1.0, 3.0], [-2.0, 0.0, 3.0, -4.0]])
    cp, ri, v = _lower_csc(B)
    assert oracle.norm_inf_sym(4, cp, ri, v) == 9.0


def test_residual_measures_hand():
    # A x = [5, 3, 1] for x = 1; b = [6, 3, 1] leaves r = [1, 0, 0].
    A = np.array([[4.0, 1.0, 0.0], [1.0, 3.0, -1.0], [0.0, -1.0, 2.0]])
    cp, ri, v = _lower_csc(A)
    x = np.ones(3)
    b = np.array([6.0, 3.0, 1.0])
    relres, eta = oracle.residual_measures(3, cp, ri, v, x, b)
    assert relres[0] == pytest.approx(1.0 / math.sqrt(46.0), rel=1e-15)
    # ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) = 1 / (5 + 6)
    assert eta[0] == pytest.approx(1.0 / 11.0, rel=1e-15)
    # two right-hand sides at once, the second exact
    relres, eta = oracle.residual_measures(3, cp, ri, v, np.stack([x, x]),
                                           np.stack([b, A @ x]))
    assert relres[1] == 0.0 and eta[1] == 0.0
    assert relres[0] == pytest.approx(1.0 / math.sqrt(46.0), rel=1e-15)


def test_forward_error_hand():
    assert oracle.forward_error([1.0, 2.0, 3.0], [1.0, 2.0, 4.0]) == 0.25
    # normalized by the reference (4), not by the tested vector (3)
    assert oracle.forward_error([-3.0, 1.0], [-4.0, 1.0]) == 0.25
    assert oracle.forward_error(np.zeros(4), np.zeros(4)) == 0.0


def test_factor_error_hand():
    # columns of 3, 1 and 2 entries; per column the largest deviation over
    # the reference column's largest magnitude
    Lcolptr = np.array([0, 3, 4, 6], np.int64)
    ref = np.array([2.0, -1.0, 0.5, 4.0, 5.0, -10.0])
    got = np.array([3.0, -1.0, 0.5, 4.0, 5.0, -10.0])      # column 0: 1 / 2
    assert oracle.factor_error(Lcolptr, got, ref) == 0.5
    got = np.array([2.0, -1.0, 0.5, 4.0, 5.0, -12.0])      # last column: 2 / 10
    assert oracle.factor_error(Lcolptr, got, ref) == pytest.approx(0.2, rel=1e-15)
    got = np.array([2.0, -1.0, 0.5, 4.5, 5.0, -10.0])      # middle column: 0.5 / 4
    assert oracle.factor_error(Lcolptr, got, ref) == 0.125
    assert oracle.factor_error(Lcolptr, ref, ref) == 0.0


def test_stop_clause_hand():
    A = np.array([[4.0, 1.0, 0.0], [1.0, 3.0, -1.0], [0.0, -1.0, 2.0]])
    cp, ri, v = _lower_csc(A)
    x = np.ones(3)
    b = np.array([6.0, 3.0, 1.0])           # ||r||_2 = 1, ||b||_2 = sqrt(46)
    assert oracle.stop_clause(3, cp, ri, v, x, b, 0.2)[0] == 1      # 1 <= 0.2 * 6.78
    assert oracle.stop_clause(3, cp, ri, v, x, b, 0.1)[0] == 0      # 1 > 0.678
    # the floor clause: r = b - A x of size ~ u ||A|| ||x||
    u = 2.0 ** -53
    eps_b = A @ x + np.array([8.0 * u, 0.0, 0.0])
    # ||r||_2 = 8u (to rounding) <= 2 u * 5 * sqrt(3) = 17.3 u, relres ~ 1.4e-16 > 1e-20
    assert oracle.stop_clause(3, cp, ri, v, x, eps_b, 1e-20)[0] == 2
    big = A @ x + np.array([64.0 * u, 0.0, 0.0])
    assert oracle.stop_clause(3, cp, ri, v, x, big, 1e-20)[0] == 0


# --- the condition estimate ---------------------------------------------

@pytest.mark.parametrize("case", spd_cases()[:7] + [W.random_spd(50, 0.9, seed=900),
                                                     W.random_spd(64, 0.15, seed=901)],
                         ids=lambda w: "%s_n%d" % (w.name, w.pattern.n))
def test_kappa1_against_numpy_dense(case):
    """Hager's estimate is a lower bound of ||A^{-1}||_1 that is exact on
    almost every small matrix; numpy's cond(A, 1) forms the exact value
    from the dense inverse."""
    p = case.pattern
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, case.perm)
    Lx, info = oracle.factor(p.n, p.colptr, p.rowind, case.values[0], sym)
    assert info == 0
    est = oracle.kappa1_estimate(p.n, p.colptr, p.rowind, case.values[0], sym, Lx)
    A = oracle.to_dense_permuted(p.n, p.colptr, p.rowind, case.values[0])
    exact = np.linalg.cond(A, 1)
    assert est <= exact * (1 + 1e-10)
    assert est >= exact / 3.0
    assert est == pytest.approx(exact, rel=1e-10)


def test_kappa1_indefinite_sign_inverse():
    """A matrix whose inverse has mixed signs (positive off-diagonals), so
    the first ascent vector is not optimal: still within numpy's value."""
    rng = np.random.default_rng(77)
    n = 30
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n) * 0.05
    cp, ri, v = _lower_csc(A)
    sym = oracle.symbolic(n, cp, ri)
    Lx, info = oracle.factor(n, cp, ri, v, sym)
    assert info == 0
    est = oracle.kappa1_estimate(n, cp, ri, v, sym, Lx)
    exact = np.linalg.cond(A, 1)
    assert exact / 3.0 <= est <= exact * (1 + 1e-10)


@pytest.mark.parametrize("n", [1, 2, 3, 10, 101, 2000])
def test_kappa1_1d_laplacian_closed_form(n):
    """tridiag(-1, 2, -1): (A^{-1})_ij = min(i,j)(n+1-max(i,j))/(n+1) > 0, so
    column j sums to j(n+1-j)/2 (1-based) and ||A^{-1}||_1 is its maximum,
    at j = floor((n+1)/2); ||A||_1 = 4 for n >= 3 (2, 3 for n = 1, 2)."""
    pat, vals = path_laplacian(n)
    sym = oracle.symbolic(n, pat.colptr, pat.rowind)
    Lx, info = oracle.factor(n, pat.colptr, pat.rowind, vals, sym)
    j = (n + 1) // 2
    inv1 = j * (n + 1 - j) / 2.0
    # the solves carry a relative error of about kappa_2 u ~ (4 n^2 / pi^2) u
    rel = max(1e-14, 10.0 * n * n * 2.0 ** -53)
    assert oracle.inv_norm1_estimate(sym, Lx) == pytest.approx(inv1, rel=rel)
    anorm = {1: 2.0, 2: 3.0}.get(n, 4.0)
    k = oracle.kappa1_estimate(n, pat.colptr, pat.rowind, vals, sym, Lx)
    assert k == pytest.approx(anorm * inv1, rel=rel)


def test_within_conditioning_rule():
    assert oracle.within_conditioning(1e-11, 1e-10, 1e20)
    assert not oracle.within_conditioning(1e-6, 1e-10, 1e6)       # 10 k u = 1.1e-9
    assert oracle.within_conditioning(1e-6, 1e-10, 1e10)          # 10 k u = 1.1e-5


# --- cotangent assembly ---------------------------------------------------

def _mesh_pattern(nv, tris):
    e = np.concatenate([np.asarray(tris)[:, [0, 1]], np.asarray(tris)[:, [1, 2]],
                        np.asarray(tris)[:, [2, 0]]])
    e = np.unique(np.sort(e, 1), axis=0)
    return W.lower_csc_from_edges(nv, e)


def _regular_grid(k):
    pos, tris = W.trimesh_geometry(k, np.random.default_rng(0))
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    pos = np.stack([ii.ravel(), jj.ravel()], 1).astype(np.float64)   # no jitter
    return pos, tris


def test_cotan_regular_grid_closed_form():
    """Unjittered grid split along (i,j)-(i+1,j+1): an axis edge sees two
    45-degree angles (cot 1) inside the mesh and one on the boundary; a
    diagonal edge sees two right angles (cot 0), clipped up to clip_lo;
    the diagonal is the sum of the weights plus c m."""
    k = 6
    pos, tris = _regular_grid(k)
    n = k * k
    pat = _mesh_pattern(n, tris)
    m = np.linspace(1.0, 2.0, n)
    v = oracle.cotan_values(n, pat.colptr, pat.rowind, pos, tris, m, 0.25, 0.05, 2.0)[0]
    rows, cols = pat.rows, pat.cols
    for q in range(pat.nnz):
        a, b = int(rows[q]), int(cols[q])
        if a == b:
            continue
        ia, ja, ib, jb = a % k, a // k, b % k, b // k
        if abs(ia - ib) + abs(ja - jb) == 2:          # diagonal edge
            assert v[q] == -0.05
        elif (ia == ib and ia in (0, k - 1)) or (ja == jb and ja in (0, k - 1)):
            assert v[q] == -0.5                        # boundary axis edge
        else:
            assert v[q] == -1.0                        # interior axis edge
    A = oracle.to_dense_permuted(n, pat.colptr, pat.rowind, v)
    off = A - np.diag(np.diag(A))
    assert np.allclose(np.diag(A), -off.sum(1) + 0.25 * m, rtol=0, atol=1e-15)


def test_cotan_equilateral_triangle():
    """One equilateral triangle: every angle is 60 degrees, cot = 1/sqrt(3),
    so each edge weighs 1/(2 sqrt(3))."""
    pos = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, math.sqrt(3.0) / 2]])
    tris = np.array([[0, 1, 2]])
    pat = _mesh_pattern(3, tris)
    v = oracle.cotan_values(3, pat.colptr, pat.rowind, pos, tris, np.zeros(3), 0.0,
                            -10.0, 10.0)[0]
    off = pat.rows != pat.cols
    assert np.allclose(v[off], -1.0 / (2.0 * math.sqrt(3.0)), rtol=1e-15, atol=0)
    assert np.allclose(v[~off], 1.0 / math.sqrt(3.0), rtol=1e-15, atol=0)


def test_cotan_against_angles():
    """A jittered mesh against cot(theta) = 1/tan(theta) of the corner angle
    theta = atan2(|u x v|, u . v) computed per corner in plain Python."""
    k = 7
    rng = np.random.default_rng(3)
    pos, tris = W.trimesh_geometry(k, rng)
    n = k * k
    pat = _mesh_pattern(n, tris)
    m = rng.uniform(0.5, 1.5, n)
    v = oracle.cotan_values(n, pat.colptr, pat.rowind, pos, tris, m, 1e-3, -100.0, 100.0)[0]
    w = {}
    for t in tris:
        for c in range(3):
            o, a, b = int(t[c]), int(t[(c + 1) % 3]), int(t[(c + 2) % 3])
            ux, uy = pos[a] - pos[o]
            vx, vy = pos[b] - pos[o]
            th = math.atan2(abs(ux * vy - uy * vx), ux * vx + uy * vy)
            key = (min(a, b), max(a, b))
            w[key] = w.get(key, 0.0) + 0.5 / math.tan(th)
    deg = np.zeros(n)
    for q in range(pat.nnz):
        a, b = int(pat.rows[q]), int(pat.cols[q])
        if a != b:
            ref = w[(b, a)]
            assert v[q] == pytest.approx(-ref, rel=1e-12, abs=1e-14)
            deg[a] += ref
            deg[b] += ref
    for q in range(pat.nnz):
        a = int(pat.rows[q])
        if a == int(pat.cols[q]):
            assert v[q] == pytest.approx(deg[a] + 1e-3 * m[a], rel=1e-12)


def test_cotan_edge_scale_and_clip():
    """Per-set scales multiply the clipped weights and are clipped again;
    positions per value set give independent systems."""
    k = 5
    pos, tris = _regular_grid(k)
    n = k * k
    pat = _mesh_pattern(n, tris)
    nedge = int(np.sum(pat.rows != pat.cols))
    sc = np.stack([np.full(nedge, 2.0), np.full(nedge, 0.5)])
    v = oracle.cotan_values(n, pat.colptr, pat.rowind, pos, tris, np.ones(n), 0.0, 0.05, 1.5,
                            edge_scale=sc)
    base = oracle.cotan_values(n, pat.colptr, pat.rowind, pos, tris, np.ones(n), 0.0, 0.05, 1.5)[0]
    off = pat.rows != pat.cols
    assert np.array_equal(v[0][off], np.maximum(-1.5, 2.0 * base[off]))   # 2 x 1 -> 1.5
    assert np.array_equal(v[1][off], np.minimum(-0.05, 0.5 * base[off]))  # 0.05/2 -> 0.05
    # a second position set (scaled mesh: cotangents are scale invariant)
    v2 = oracle.cotan_values(n, pat.colptr, pat.rowind, np.stack([pos, 3.0 * pos]), tris,
                             np.ones(n), 0.0, 0.05, 1.5)
    assert np.array_equal(v2[0], v2[1])


# --- sparse products ------------------------------------------------------

def _rand_csr(rng, m, n, per_row):
    rowptr = [0]
    cols = []
    for i in range(m):
        c = np.sort(rng.choice(n, size=min(per_row, n), replace=False))
        cols.extend(c.tolist())
        rowptr.append(len(cols))
    return (np.array(rowptr, np.int64), np.array(cols, np.int32),
            rng.uniform(-1, 1, size=len(cols)))


def _dense(csr, m, n):
    r, c, v = csr
    out = np.zeros((m, n))
    for i in range(m):
        for q in range(r[i], r[i + 1]):
            out[i, c[q]] += v[q]
    return out


@pytest.mark.parametrize("transB", [False, True])
@pytest.mark.parametrize("with_d", [False, True])
def test_sparse_product_against_dense(transB, with_d):
    """Against numpy's dense product (brute force on small matrices), the
    pattern against a plain loop over the rows."""
    rng = np.random.default_rng(11 + 2 * transB + with_d)
    m, p, n = 23, 17, 19
    A = _rand_csr(rng, m, p, 4)
    B = _rand_csr(rng, n, p, 5) if transB else _rand_csr(rng, p, n, 5)
    D = _rand_csr(rng, m, n, 3) if with_d else None
    C = oracle.sparse_product(m, n, A, B, transB, D)
    Bd = _dense(B, n, p).T if transB else _dense(B, p, n)
    ref = _dense(A, m, p) @ Bd + (_dense(D, m, n) if with_d else 0.0)
    assert np.allclose(C.toarray(), ref, rtol=1e-14, atol=1e-14)
    rp, ci = oracle.sparse_product_pattern(m, n, A[0], A[1], B[0], B[1], transB,
                                           D[0] if with_d else None, D[1] if with_d else None)
    # every structural entry is listed (values may cancel to zero)
    S = np.zeros((m, n), bool)
    for i in range(m):
        S[i, ci[rp[i]:rp[i + 1]]] = True
    Ad = _dense(A, m, p) != 0
    Bs = (_dense(B, n, p).T if transB else _dense(B, p, n)) != 0
    ref_s = (Ad.astype(int) @ Bs.astype(int)) > 0
    if with_d:
        ref_s |= _dense(D, m, n) != 0
    assert np.array_equal(S, ref_s)


def test_sparse_power_of_laplacian_annihilates_constants():
    """K 1 = 0 for the cotangent stiffness (zero row sums), so K^2 1 = K^3 1
    = 0 up to rounding, and (K M K^T + D) 1 = D 1."""
    import scipy.sparse as sp
    k = 12
    w = W.trimesh_workload(k, batch=1, nrhs=1, seed=13)
    m = w.extra["mesh"]
    p = w.pattern
    v = oracle.cotan_values(p.n, p.colptr, p.rowind, m["pos"], m["tris"], m["mass"], 0.0,
                            *m["clip"])[0]
    K = sp.csc_matrix((v, p.rowind, p.colptr), shape=(p.n, p.n))
    K = (K + sp.tril(K, -1).T).tocsr()
    Kt = (K.indptr, K.indices, K.data)
    K2 = oracle.sparse_product(p.n, p.n, Kt, Kt)
    K3 = oracle.sparse_product(p.n, p.n, (K2.indptr, K2.indices, K2.data), Kt)
    one = np.ones(p.n)
    scale = np.abs(K3).sum(1).max()
    assert np.abs(K2 @ one).max() <= 1e-13 * np.abs(K2).sum(1).max()
    assert np.abs(K3 @ one).max() <= 1e-13 * scale
    Mdiag = (np.arange(p.n + 1, dtype=np.int64), np.arange(p.n, dtype=np.int32), m["mass"])
    T = oracle.sparse_product(p.n, p.n, Kt, Mdiag)
    rng = np.random.default_rng(5)
    D = _rand_csr(rng, p.n, p.n, 6)
    R = oracle.sparse_product(p.n, p.n, (T.indptr, T.indices, T.data), Kt, True, D)
    assert np.allclose(R @ one, _dense(D, p.n, p.n) @ one, rtol=0, atol=1e-12)
