"""GPU parity: the HIP factor and solves against the CPU oracle.

Tolerances (FP64 path): per-column normwise factor error
max_j ||L[:, j] - L_o[:, j]||_inf / ||L_o[:, j]||_inf <= 1e-12 and solution
forward error ||x - x_o||_inf / ||x_o||_inf <= 1e-12.  The two sides sum in
different orders (multifrontal assembly versus up-looking rows), so
bit-equality is not expected; both are backward stable and these systems are
well conditioned (strict diagonal dominance, kappa <= ~2e3), so the
difference stays near kappa * u ~ 1e-13.  Exact results: the elimination
tree and pattern (bit-exact), diagonal matrices (sqrt is correctly rounded
on both sides), breakdown steps, and batch/repeat reproducibility
(bit-identical)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import all_columns, log, oracle_run, run_library

pytestmark = pytest.mark.gpu

TOL_L = 1e-12
TOL_X = 1e-12


def _cases():
    return [
        ("cfg0_grid2d_32x32_natural", lambda: W.config(0), {}),
        ("grid2d_64x64_nd", lambda: W.small_grid((64, 64), "nd", seed=11), {}),
        ("grid3d_12^3_nd", lambda: W.small_grid((12, 12, 12), "nd", seed=12), {}),
        ("grid3d_16x15x14_nd", lambda: W.small_grid((16, 15, 14), "nd", seed=13), {}),
        ("random_300_dense_fill", lambda: W.random_spd(300, 0.05, seed=14), {}),
        ("random_200_nearly_dense", lambda: W.random_spd(200, 0.5, seed=15), {}),
        ("random_130_ragged", lambda: W.random_spd(130, 0.9, seed=16), {}),
        # every front through the tiled kernels (assembly/potrf/trsm/mfma)
        ("grid3d_10^3_tiled_only", lambda: W.small_grid((10, 10, 10), "nd", seed=17),
         {"small_front": 1}),
        ("grid2d_40x40_tiled_only", lambda: W.small_grid((40, 40), "natural", seed=18),
         {"small_front": 1}),
        # bigger fronts in the one-workgroup LDS kernel (packed triangle)
        ("grid3d_12^3_lds_big", lambda: W.small_grid((12, 12, 12), "nd", seed=19),
         {"small_front": 100}),
        ("random_200_lds_whole", lambda: W.random_spd(200, 0.5, seed=23), {"small_front": 200}),
        ("grid3d_16x15x14_lds_192", lambda: W.small_grid((16, 15, 14), "nd", seed=24),
         {"small_front": 192}),
        # one 700-column front: the trailing update of its first 256-column
        # block is split between the two streams (lookahead)
        ("random_700_lookahead", lambda: W.random_spd(700, 0.9, seed=25), {"small_front": 1}),
        # fundamental supernodes only
        ("grid3d_9^3_norelax", lambda: W.small_grid((9, 9, 9), "nd", seed=20), {"relax": 0}),
        ("n1", lambda: W.random_spd(1, 0.0, seed=21), {}),
        ("n2", lambda: W.random_spd(2, 1.0, seed=22), {}),
    ]


@pytest.mark.parametrize("name,make,opts", _cases(), ids=[c[0] for c in _cases()])
def test_factor_solve_parity(name, make, opts):
    w = make()
    p = w.pattern
    log("case %s n=%d nnz=%d opts=%s" % (name, p.n, p.nnz, opts))
    plan, num, info, x = run_library(w, "f64", opts=opts)
    assert info[0] == 0
    # symbolic bit-exact
    sym, Lx, oinfo, xo = oracle_run(w)
    assert oinfo == 0
    perm, parent, Lcolptr, Lrowind = plan.export_symbolic()
    assert np.array_equal(parent, sym.parent)
    assert np.array_equal(Lcolptr, sym.Lcolptr)
    assert np.array_equal(Lrowind, sym.Lrowind)
    # factor and solution
    Lg = num.get_columns(0, all_columns(p.n))
    assert np.all(np.isfinite(Lg))
    ferr = oracle.factor_error(sym.Lcolptr, Lg, Lx)
    xerr = oracle.forward_error(x[0], xo)
    relres, eta = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[0], x[0], w.b[0])
    # the oracle's own residual bounds what FP64 elimination attains on the
    # system (the dense 700 case: 7.9e-13)
    orel, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[0], xo, w.b[0])
    log("  factor err %.2e  x err %.2e  relres %.2e (oracle %.2e)"
        % (ferr, xerr, relres.max(), orel.max()))
    assert ferr <= TOL_L
    assert xerr <= TOL_X
    assert relres.max() <= max(1e-13, 2.0 * orel.max())


def test_golden_fixture():
    """The stored oracle output for the 4x4 grid (tests/golden)."""
    import os
    from tests.golden.make_golden import case_grid2d_4x4, read_fixture
    fx = read_fixture(os.path.join(os.path.dirname(__file__), "golden", "grid2d_4x4_nd.txt"))
    w = case_grid2d_4x4()
    plan, num, info, x = run_library(w, "f64")
    assert info[0] == 0
    Lg = num.get_columns(0, all_columns(w.pattern.n))
    assert oracle.factor_error(fx["Lcolptr"], Lg, fx["Lx"]) <= 1e-14
    assert oracle.forward_error(x[0, 0], fx["x"]) <= 1e-14


def test_diagonal_matrix_bit_exact():
    n = 1000
    rng = np.random.default_rng(3)
    pat = W.lower_csc_from_edges(n, np.zeros((0, 2)))
    d = rng.uniform(0.1, 10.0, n)
    perm = rng.permutation(n).astype(np.int32)
    w = W.Workload("diag", pat, perm, d[None, :], rng.uniform(-1, 1, (1, 1, n)), 3)
    plan, num, info, x = run_library(w, "f64")
    Lg = num.get_columns(0, all_columns(n))
    assert np.array_equal(Lg, np.sqrt(d[perm]))
    assert np.allclose(x[0, 0], w.b[0, 0] / d, rtol=2e-16 * 4, atol=0)


@pytest.mark.parametrize("dims,opts", [((20, 20), {}), ((20, 20), {"small_front": 1}),
                                       ((11, 11, 11), {"small_front": 180})],
                         ids=["registers", "tiled", "workgroup"])
def test_not_spd_info_matches_oracle(dims, opts):
    w = W.small_grid(dims, "nd", seed=31)
    p = w.pattern
    vals = w.values.copy()
    # break two pivots; the smallest failing elimination step must be reported
    pinv = np.empty(p.n, np.int64)
    pinv[w.perm] = np.arange(p.n)
    for old in (37, 250):
        vals[0, p.colptr[old]] = -1.0
    w2 = W.Workload("bad", p, w.perm, vals, w.b, 0)
    _, _, oinfo, _ = oracle_run(w2)
    assert oinfo > 0
    plan, num, info, x = run_library(w2, "f64", opts=opts)
    log("oracle info %d gpu info %d" % (oinfo, info[0]))
    assert info[0] == oinfo


def test_batch_element_equals_single_run_bitwise():
    w = W.small_grid((14, 13, 12), "nd", seed=41, batch=4, nrhs=2)
    import paper_2110_12865_amd as S
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm)
    _, numb, info, xb = run_library(w, "f64", plan=plan)
    assert np.all(info == 0)
    for s in (0, 3):
        _, num1, info1, x1 = run_library(w, "f64", values=w.values[s:s + 1], b=w.b[s:s + 1],
                                         plan=plan)
        assert np.array_equal(numb.get_columns(s, all_columns(p.n)),
                              num1.get_columns(0, all_columns(p.n)))
        assert np.array_equal(xb[s], x1[0])


def test_batch_isolates_breakdown():
    w = W.small_grid((16, 16), "nd", seed=42, batch=3)
    vals = w.values.copy()
    vals[1, w.pattern.colptr[100]] = -5.0
    w2 = W.Workload("b", w.pattern, w.perm, vals, w.b, 0)
    plan, num, info, x = run_library(w2, "f64")
    assert info[0] == 0 and info[2] == 0 and info[1] > 0
    for s in (0, 2):
        assert np.all(np.isfinite(x[s]))
        relres, _ = oracle.residual_measures(w.pattern.n, w.pattern.colptr, w.pattern.rowind,
                                             vals[s], x[s], w.b[s])
        assert relres.max() <= 1e-13


def test_repeat_factor_is_reproducible():
    """factor A, then B, then A again on the same numeric object."""
    import torch
    import paper_2110_12865_amd as S
    w = W.small_grid((11, 11, 11), "nd", seed=43, batch=2)
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm)
    num = plan.numeric(1, "f64")
    outs = []
    for s in (0, 1, 0):
        num.factor(torch.from_numpy(w.values[s:s + 1].copy()).cuda())
        outs.append(num.get_columns(0, all_columns(p.n)))
    assert np.array_equal(outs[0], outs[2])
    assert not np.array_equal(outs[0], outs[1])


def test_multiple_rhs():
    w = W.small_grid((10, 9, 8), "nd", seed=44, nrhs=3)
    plan, num, info, x = run_library(w, "f64")
    sym, Lx, _, xo = oracle_run(w)
    for r in range(3):
        assert oracle.forward_error(x[0, r], xo[r]) <= TOL_X


@pytest.mark.parametrize("opts", [{}, {"small_front": 192}], ids=["default", "workgroup"])
def test_fp32_factor_accuracy(opts):
    """FP32 factor (FP32 accumulation) and FP32 solve: the factor and the
    solution match the oracle to FP32 accuracy (no parity claim at FP64
    level)."""
    w = W.small_grid((16, 16, 16), "nd", seed=45)
    plan, num, info, x = run_library(w, "f32", opts=opts)
    sym, Lx, _, xo = oracle_run(w)
    Lg = num.get_columns(0, all_columns(w.pattern.n))
    ferr = oracle.factor_error(sym.Lcolptr, Lg, Lx)
    xerr = oracle.forward_error(x[0], xo)
    log("fp32 factor err %.2e x err %.2e" % (ferr, xerr))
    assert ferr <= 2e-5
    assert xerr <= 1e-4


def _sampled_llt_check(plan, num, w, rows_sel):
    """(L L^T)_ij against (P A P^T)_ij for every pair of the selected rows
    (permuted numbering), within the componentwise backward-error bound of
    Cholesky: |L L^T - P A P^T| <= gamma_{c+1} |L| |L|^T with c the longest
    column (Higham, Accuracy and Stability of Numerical Algorithms, Thm 10.3),
    gamma_k = k u / (1 - k u).  Returns the largest ratio error / bound."""
    import scipy.sparse as sp
    p = w.pattern
    n = p.n
    _, _, Lcolptr, Lrowind = plan.export_symbolic()
    Lx = num.get_columns(0, all_columns(n))
    L = sp.csc_matrix((Lx, Lrowind, Lcolptr), shape=(n, n))
    LR = L[rows_sel, :].tocsr()
    G = (LR @ LR.T).toarray()
    absLR = abs(LR)
    B = (absLR @ absLR.T).toarray()
    # (P A P^T)_ij = A_{perm i, perm j} from the lower CSC pattern
    perm = np.asarray(w.perm, np.int64)
    A = sp.csc_matrix((w.values[0], p.rowind, p.colptr), shape=(n, n))
    A = (A + sp.tril(A, -1).T).tocsr()
    orig = perm[rows_sel]
    Asub = A[orig, :][:, orig].toarray()
    c = int(np.max(np.diff(Lcolptr)))
    u = 2.0 ** -53
    gamma = (c + 1) * u / (1 - (c + 1) * u)
    err = np.abs(G - Asub)
    return float(np.max(err / (gamma * B + 1e-300))), float(np.max(err))


def test_full_size_grid3d_64_nd():
    """The 64^3 7-point system (n = 262144) in the benchmark's launch
    configuration: the leading 32768 x 32768 block of L against the oracle
    (rows < m of L are the factor of the leading m x m block of P A P^T),
    the residual of the full solve, and, for 48 rows of the top separators
    (the 4096-column root front and the separators below it, where the
    tiled MFMA kernels and the lookahead run), every entry (L L^T)_ij
    against (P A P^T)_ij within Cholesky's componentwise backward-error
    bound."""
    w = W.config(1)
    p = w.pattern
    log("full-size 64^3: factor + solve")
    plan, num, info, x = run_library(w, "f64")
    assert info[0] == 0
    relres, eta = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[0], x[0], w.b[0])
    log("  relres %.2e eta %.2e" % (relres.max(), eta.max()))
    assert relres.max() <= 1e-12
    m = 32768
    sym, Lx, oinfo, _ = oracle_run(w, nrows=m)
    assert oinfo == 0
    cols = np.arange(m, dtype=np.int32)
    Lg = num.get_columns(0, cols)
    _, _, Lcolptr, Lrowind = plan.export_symbolic()
    # keep, per column, the rows below m (they come first, rows ascend)
    keep = np.zeros(Lcolptr[m], bool)
    keep[:] = Lrowind[:Lcolptr[m]] < m
    Lg_lead = Lg[keep]
    assert Lg_lead.size == sym.nnzL
    ferr = oracle.factor_error(sym.Lcolptr[:m + 1], Lg_lead, Lx[:sym.Lcolptr[m]])
    log("  leading-block factor err %.2e" % ferr)
    assert ferr <= TOL_L
    del Lg, keep, Lg_lead, sym, Lx
    rng = np.random.default_rng(201)
    rows_sel = np.sort(np.concatenate([
        rng.choice(np.arange(p.n - 4096, p.n), 32, replace=False),       # root front
        rng.choice(np.arange(p.n - 12288, p.n - 4096), 16, replace=False)]))  # next separators
    ratio, emax = _sampled_llt_check(plan, num, w, rows_sel)
    log("  sampled L L^T: max |error| %.2e, max error / bound %.3f" % (emax, ratio))
    assert ratio <= 1.0


@pytest.mark.parametrize("name,make", [
    ("grid3d_16x15x14_nd", lambda: W.small_grid((16, 15, 14), "nd", batch=3, nrhs=6, seed=46)),
    ("random_200_nearly_dense", lambda: W.random_spd(200, 0.5, seed=47, batch=3, nrhs=6)),
], ids=["grid3d_panels", "dense_panels"])
def test_many_rhs_padded_ldb(name, make):
    """Six right-hand sides (two blocks of the per-launch right-hand-side
    count) in a buffer with a padded leading dimension, batch of three:
    every solution column against the oracle, the padding untouched."""
    import torch
    import paper_2110_12865_amd as S
    w = make()
    p = w.pattern
    log("case %s n=%d batch=%d nrhs=%d" % (name, p.n, w.batch, w.nrhs))
    plan = S.analyze(p.colptr, p.rowind, w.perm)
    num = plan.numeric(w.batch, "f64")
    num.factor(torch.from_numpy(np.ascontiguousarray(w.values)).cuda())
    assert np.all(num.info() == 0)
    ldb = p.n + 7
    host = np.full((w.batch, w.nrhs, ldb), 123.25)
    host[:, :, :p.n] = w.b
    db = torch.from_numpy(host).cuda()
    num.solve(db)  # leading dimension = db.shape[2] = n + 7
    out = db.cpu().numpy()
    assert np.all(out[:, :, p.n:] == 123.25)
    for s in range(w.batch):
        sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
        Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
        xo = oracle.solve(sym, Lx, w.b[s])
        for r in range(w.nrhs):
            assert oracle.forward_error(out[s, r, :p.n], xo[r]) <= TOL_X


def _solve_with(w, dtype, **opts):
    import torch
    import paper_2110_12865_amd as S
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm, **opts)
    num = plan.numeric(w.batch, dtype)
    num.factor(torch.from_numpy(np.ascontiguousarray(w.values)).cuda())
    assert np.all(num.info() == 0)
    db = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    num.solve(db)
    return db.cpu().numpy()


@pytest.mark.parametrize("seg_max", [-1, 0, 1 << 30], ids=["lanes-per-matrix", "default", "lanes-per-row"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,make", [
    ("grid3d_20x18x16_nd", lambda: W.small_grid((20, 18, 16), "nd", batch=40, nrhs=3, seed=48)),
    ("trimesh_48", lambda: W.trimesh_workload(48, batch=70, nrhs=2, seed=49)),
    ("random_180_dense", lambda: W.random_spd(180, 0.4, seed=50, batch=33, nrhs=5)),
], ids=["grid3d", "trimesh", "dense"])
def test_interleaved_layout_bitwise_equal_rowmajor(name, make, dtype, seg_max):
    """Batches of at least 32 matrices solve in the batch-interleaved layout
    (one matrix per lane); levels with few supernodes may instead put one
    lane on each row (soa_seg_max: never, the default split, every level).
    All kernels perform the same operations in the same order on every
    entry, so the solutions are bit-identical to the row-major layout's; a
    batch that is not a multiple of 64 exercises the partial lane group; the
    FP64 result also matches the oracle."""
    w = make()
    log("case %s batch=%d nrhs=%d %s seg_max=%d" % (name, w.batch, w.nrhs, dtype, seg_max))
    x_soa = _solve_with(w, dtype, soa_min_batch=32, soa_seg_max=seg_max)  # interleaved
    x_row = _solve_with(w, dtype, soa_min_batch=-1)                        # row-major segments
    assert np.array_equal(x_soa, x_row)
    if dtype == "f64":
        # the mesh (no Dirichlet rows, kappa ~ 1e6 at this size) may differ
        # from the oracle by more than 1e-10 between two correct FP64
        # solvers: there the bound is 10 kappa_1 u (kappa_1 estimated from
        # oracle solves)
        p = w.pattern
        for s in (0, w.batch - 1):
            sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
            Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
            xo = oracle.solve(sym, Lx, w.b[s])
            kap = oracle.kappa1_estimate(p.n, p.colptr, p.rowind, w.values[s], sym, Lx)
            for r in range(w.nrhs):
                err = oracle.forward_error(x_soa[s, r], xo[r])
                log("  set %d rhs %d: x err %.2e (kappa_1 ~ %.2e)" % (s, r, err, kap))
                assert oracle.within_conditioning(err, 1e-10, kap)


@pytest.mark.parametrize("sub_min", [1, 24, 400], ids=["all-levels", "some-levels", "few-levels"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,make", [
    ("grid3d_20x18x16_nd", lambda: W.small_grid((20, 18, 16), "nd", batch=70, nrhs=3, seed=53)),
    ("trimesh_48", lambda: W.trimesh_workload(48, batch=40, nrhs=2, seed=54)),
    ("random_180_dense", lambda: W.random_spd(180, 0.4, seed=55, batch=33, nrhs=5)),
], ids=["grid3d", "trimesh", "dense"])
def test_interleaved_subtrees_bitwise_equal_rowmajor(name, make, dtype, sub_min):
    """The lowest levels of the interleaved solve run as whole subtrees, one
    wave per (subtree, group of matrices), up to the highest level with at
    least `sub_min` such waves.  Every supernode goes through the same
    operations in the same order as in the level kernels, so the solutions
    are bit-identical to the row-major layout's for every cut."""
    w = make()
    log("case %s batch=%d nrhs=%d %s subtree_min=%d" % (name, w.batch, w.nrhs, dtype, sub_min))
    x_sub = _solve_with(w, dtype, soa_min_batch=32, soa_subtree_min=sub_min)
    x_lvl = _solve_with(w, dtype, soa_min_batch=32, soa_subtree_min=-1)
    x_row = _solve_with(w, dtype, soa_min_batch=-1)
    assert np.array_equal(x_lvl, x_row)
    assert np.array_equal(x_sub, x_row)


def test_interleaved_copy_refreshed_after_refactor():
    """The interleaved copy of L is rebuilt after every factorization: value
    set A, then B, on one numeric object gives B's fresh solution."""
    import torch
    import paper_2110_12865_amd as S
    wa = W.small_grid((14, 13, 12), "nd", batch=36, nrhs=2, seed=51)
    wb = W.small_grid((14, 13, 12), "nd", batch=36, nrhs=2, seed=52)
    p = wa.pattern
    plan = S.analyze(p.colptr, p.rowind, wa.perm, soa_min_batch=32)
    num = plan.numeric(wa.batch, "f64")
    db = torch.from_numpy(np.ascontiguousarray(wa.b)).cuda()
    num.factor(torch.from_numpy(np.ascontiguousarray(wa.values)).cuda())
    num.solve(db)
    num.factor(torch.from_numpy(np.ascontiguousarray(wb.values)).cuda())
    db = torch.from_numpy(np.ascontiguousarray(wb.b)).cuda()
    num.solve(db)
    assert np.array_equal(db.cpu().numpy(), _solve_with(wb, "f64", soa_min_batch=32))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("soa", [-1, 1], ids=["rowmajor", "interleaved"])
def test_panel_workgroup_path_bitwise_equal(dtype, soa):
    """Batches of 16 or more solve each panel supernode (w > 64 or c > 512)
    with one workgroup per (supernode, matrix); smaller batches use one
    launch per panel over many workgroups.  Both perform the same operations
    in the same order, so matrices 0..14 of a 16-matrix batch solve to the
    same bits as the same 15 matrices alone (whole-block inverses off: they
    apply to batches of 16 or more only)."""
    import dataclasses
    import paper_2110_12865_amd as S
    w16 = W.small_grid((24, 22, 20), "nd", batch=16, nrhs=5, seed=53)
    w15 = dataclasses.replace(w16, values=w16.values[:15], b=w16.b[:15])
    p = w16.pattern
    plan = S.analyze(p.colptr, p.rowind, w16.perm, soa_min_batch=soa)
    first, parent, level, rowptr, rows = plan.export_supernodes()
    wd, c = np.diff(first), np.diff(rowptr)
    npan = int(np.sum((wd > 64) | (c > 512)))
    log("case grid 24x22x20 %s soa=%d: %d panel supernodes (max w %d, max c %d)"
        % (dtype, soa, npan, wd.max(), c.max()))
    assert npan > 0
    x16 = _solve_with(w16, dtype, soa_min_batch=soa, panel_inverse=-1)
    x15 = _solve_with(w15, dtype, soa_min_batch=soa, panel_inverse=-1)
    assert np.array_equal(x16[:15], x15)
    if dtype == "f64":
        sym = oracle.symbolic(p.n, p.colptr, p.rowind, w16.perm)
        Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w16.values[15], sym)
        xo = oracle.solve(sym, Lx, w16.b[15])
        for r in range(w16.nrhs):
            assert oracle.forward_error(x16[15, r], xo[r]) <= 1e-10


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,make", [
    ("grid3d_24x22x20_nd", lambda: W.small_grid((24, 22, 20), "nd", batch=16, nrhs=5, seed=56)),
    ("trimesh_128", lambda: W.trimesh_workload(128, batch=20, nrhs=3, seed=57)),
], ids=["grid3d", "trimesh"])
def test_panel_inverse_solve(name, make, dtype):
    """Batches of 16 or more may solve the panel-solved supernodes with the
    whole-block inverse X = L11^{-1} of each diagonal block (formed after the
    factorization): y = X v1, u = v2 - L21 y forward, x1 = X^T (y - L21^T x2)
    backward.  The result agrees with panel-by-panel substitution to the
    precision of the factor (not bit for bit), the FP64 result matches the
    oracle, and the interleaved and row-major layouts give the same bits."""
    import paper_2110_12865_amd as S
    w = make()
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm)
    first, parent, level, rowptr, rows = plan.export_supernodes()
    wd, c = np.diff(first), np.diff(rowptr)
    pan = (wd > 64) | (c > 512)
    log("case %s %s batch=%d: %d panel supernodes (max w %d)" % (name, dtype, w.batch,
        int(pan.sum()), int(wd[pan].max()) if pan.any() else 0))
    assert pan.any() and wd[pan].max() <= 1024
    x_sub = _solve_with(w, dtype, soa_min_batch=-1, panel_inverse=-1)
    x_inv = _solve_with(w, dtype, soa_min_batch=-1, panel_inverse=1)
    x_soa = _solve_with(w, dtype, soa_min_batch=16, panel_inverse=1)
    assert np.array_equal(x_soa, x_inv)
    assert not np.array_equal(x_inv, x_sub)  # the inverse path was taken
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    for s in (0, w.batch - 1):
        Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
        xo = oracle.solve(sym, Lx, w.b[s])
        kap = oracle.kappa1_estimate(p.n, p.colptr, p.rowind, w.values[s], sym, Lx)
        for r in range(w.nrhs):
            e_inv = oracle.forward_error(x_inv[s, r], xo[r])
            e_sub = oracle.forward_error(x_sub[s, r], xo[r])
            log("  set %d rhs %d: x err %.2e (substitution %.2e, kappa_1 ~ %.2e)"
                % (s, r, e_inv, e_sub, kap))
            if dtype == "f64":
                assert oracle.within_conditioning(e_inv, 1e-10, kap)
            else:
                # FP32 factor and solve: both paths within the FP32 bound
                assert e_inv <= max(1e-4, 10.0 * kap * 2.0 ** -24)
                assert e_inv <= 10.0 * max(e_sub, 1e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,make,opts", [
    ("grid3d_14^3_relaxed", lambda: W.small_grid((14, 14, 14), "nd", seed=210),
     {"relax_cols": 16, "relax_zeros": 0.3}),
    ("trimesh_60_relaxed_tiled", lambda: W.trimesh_workload(60, batch=2, nrhs=1, seed=211),
     {"relax_cols": 16, "relax_zeros": 0.3, "small_front": 1}),
    ("random_400_relaxed_lds", lambda: W.random_spd(400, 0.02, seed=212),
     {"relax_cols": 32, "relax_zeros": 0.5, "small_front": 200}),
], ids=["registers", "tiled", "workgroup"])
def test_padded_entries_exactly_zero(name, make, opts, dtype):
    """Amalgamation stores entries outside the exact pattern of L; every
    product that reaches such an entry has a stored-zero factor, so each
    comes out exactly 0.0 (reading 4 of the oracle's conventions), in every
    front kernel family, while the exact entries match the oracle."""
    w = make()
    p = w.pattern
    log("case %s %s opts=%s" % (name, dtype, opts))
    plan, num, info, x = run_library(w, dtype, opts=opts)
    assert np.all(info == 0)
    first, _, _, rowptr, rows = plan.export_supernodes()
    _, _, Lcolptr, Lrowind = plan.export_symbolic()
    npad = 0
    for s in range(len(first) - 1):
        blk = num.get_block(0, s)
        R = rows[rowptr[s]:rowptr[s + 1]]
        for t in range(first[s + 1] - first[s]):
            j = first[s] + t
            exact = set(Lrowind[Lcolptr[j]:Lcolptr[j + 1]].tolist())
            for i in range(t, len(R)):
                if int(R[i]) not in exact:
                    npad += 1
                    assert blk[t, i] == 0.0, (s, t, i)
    log("  %d padded entries, all 0.0" % npad)
    assert npad > 0
    if dtype == "f64":
        # the mesh case is ill-conditioned (kappa_1 ~ 5e7): two correct FP64
        # factorizations that sum in different orders agree in L only to the
        # conditioning limit (first-order perturbation of the Cholesky factor,
        # ||dL|| / ||L|| <~ kappa(A) ||dA|| / ||A||), the same rule as for x
        sym, Lx, _, _ = oracle_run(w)
        ferr = oracle.factor_error(sym.Lcolptr, num.get_columns(0, all_columns(p.n)), Lx)
        kap = oracle.kappa1_estimate(p.n, p.colptr, p.rowind, w.values[0], sym, Lx)
        log("  factor err %.2e (kappa_1 %.2e)" % (ferr, kap))
        assert oracle.within_conditioning(ferr, TOL_L, kap)
