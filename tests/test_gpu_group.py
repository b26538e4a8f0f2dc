"""GPU parity of group plans (an uneven batch: several patterns factored and
solved in the same launches) against the oracle run on every pattern alone.

Same tolerances as the single-pattern parity tests: per-column normwise
factor error <= 1e-12, forward error of x <= 1e-12 (FP64); breakdown steps
exact and reported per block; refinement held to the stop rule per
(matrix, right-hand side, block)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def _members(batch=3, nrhs=2):
    return [W.small_grid((6, 6), "nd", batch=batch, nrhs=nrhs, seed=81),
            W.small_grid((40, 40), "nd", batch=batch, nrhs=nrhs, seed=82),
            W.small_grid((9, 7), "natural", batch=batch, nrhs=nrhs, seed=83),
            W.small_grid((14, 14, 14), "nd", batch=batch, nrhs=nrhs, seed=84),
            W.small_grid((4, 4, 4), "nd", batch=batch, nrhs=nrhs, seed=85)]


def _group_plan(ws, **opts):
    import paper_2110_12865_amd as S
    return S.analyze_group([(w.pattern.colptr, w.pattern.rowind, w.perm) for w in ws], **opts)


@pytest.mark.parametrize("opts", [{}, {"small_front": 1}], ids=["lds", "tiled"])
def test_group_factor_solve_matches_oracle_per_pattern(opts):
    ws = _members()
    plan = _group_plan(ws, **opts)
    col0, _ = plan.export_blocks()
    vals, b = W.group_arrays(ws)
    num = plan.numeric(vals.shape[0], "f64")
    num.factor(torch.from_numpy(vals).cuda())
    info = num.info()
    assert info.shape == (vals.shape[0], len(ws)) and np.all(info == 0)
    db = torch.from_numpy(b).cuda()
    num.solve(db)
    x = db.cpu().numpy()
    for k, w in enumerate(ws):
        p = w.pattern
        sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
        for s in range(w.batch):
            Lx, inf = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
            assert inf == 0
            xo = oracle.solve(sym, Lx, w.b[s])
            cols = np.arange(col0[k], col0[k + 1], dtype=np.int32)
            Lg = num.get_columns(s, cols)
            ferr = oracle.factor_error(sym.Lcolptr, Lg, Lx)
            xerr = max(oracle.forward_error(x[s, r, col0[k]:col0[k + 1]], xo[r])
                       for r in range(w.nrhs))
            log("%s set %d: factor err %.2e, x err %.2e" % (w.name, s, ferr, xerr))
            assert ferr <= 1e-12
            assert xerr <= 1e-12


def test_group_breakdown_reported_per_block():
    """A non-positive pivot in one pattern of one batch element is reported
    at that (element, block) with the oracle's step; every other system of
    the group is unaffected."""
    ws = _members(batch=3, nrhs=1)
    k_bad, s_bad = 3, 1
    w = ws[k_bad]
    p = w.pattern
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    # lower the diagonal of an original column so that its pivot fails
    j = int(w.perm[p.n // 2]) if w.perm is not None else p.n // 2
    w.values[s_bad, p.colptr[j]] = -1.0
    _, step = oracle.factor(p.n, p.colptr, p.rowind, w.values[s_bad], sym)
    assert step > 0
    plan = _group_plan(ws)
    col0, _ = plan.export_blocks()
    vals, b = W.group_arrays(ws)
    num = plan.numeric(vals.shape[0], "f64")
    num.factor(torch.from_numpy(vals).cuda())
    info = num.info()
    log("info per (set, block):\n%s; oracle step %d" % (info, step))
    expect = np.zeros_like(info)
    expect[s_bad, k_bad] = step
    assert np.array_equal(info, expect)
    db = torch.from_numpy(b).cuda()
    num.solve(db)
    x = db.cpu().numpy()
    for k, wk in enumerate(ws):
        pk = wk.pattern
        symk = oracle.symbolic(pk.n, pk.colptr, pk.rowind, wk.perm)
        for s in range(wk.batch):
            if (k, s) == (k_bad, s_bad):
                continue
            Lx, _ = oracle.factor(pk.n, pk.colptr, pk.rowind, wk.values[s], symk)
            xo = oracle.solve(symk, Lx, wk.b[s])
            assert oracle.forward_error(x[s, 0, col0[k]:col0[k + 1]], xo[0]) <= 1e-12


@pytest.mark.parametrize("method", ["classical", "pcg"])
def test_group_refinement_per_system(method):
    """FP32 factor + FP64 refinement on a group: every (set, rhs, block)
    meets the stop rule on its own rows, its reported relres matches the
    oracle's residual of that block, and x agrees with the FP64 oracle."""
    import paper_2110_12865_amd as S
    ws = _members(batch=2, nrhs=2)
    plan = _group_plan(ws)
    col0, _ = plan.export_blocks()
    vals, b = W.group_arrays(ws)
    num = plan.numeric(vals.shape[0], "f32")
    dv = torch.from_numpy(vals).cuda()
    num.factor(dv)
    assert np.all(num.info() == 0)
    db = torch.from_numpy(b).cuda()
    dx = torch.empty_like(db)
    rc, stats = num.refine_solve(dv, db, dx, tol=1e-10, maxit=10, method=method)
    assert rc == S.SC_OK
    x = dx.cpu().numpy()
    nb = len(ws)
    assert len(stats) == 2 * 2 * nb
    for k, w in enumerate(ws):
        p = w.pattern
        sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
        for s in range(w.batch):
            Lx, _ = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
            xo = oracle.solve(sym, Lx, w.b[s])
            xs = x[s, :, col0[k]:col0[k + 1]]
            relres, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[s], xs,
                                                 w.b[s])
            for r in range(w.nrhs):
                st = stats[(s * w.nrhs + r) * nb + k]
                err = oracle.forward_error(xs[r], xo[r])
                log("%s %s set %d rhs %d: iters %d clause %d relres %.2e (oracle %.2e) "
                    "err %.2e" % (method, w.name, s, r, st["iters"], st["clause"],
                                  st["relres"], relres[r], err))
                assert st["clause"] in (1, 2)
                assert relres[r] <= 1e-10
                # the two residuals differ by the rounding of b - A x in another
                # summation order, about u ||A|| ||x|| / ||b|| <= 1e-14 here
                assert abs(st["relres"] - relres[r]) <= 1e-3 * relres[r] + 1e-14
                assert err <= 1e-10


def test_group_matches_separate_plans():
    """The group's solution of each pattern equals the pattern's own plan's
    solution to rounding (the launches group different work, the arithmetic
    of every front is the same algorithm)."""
    ws = _members(batch=2, nrhs=1)
    plan = _group_plan(ws)
    col0, _ = plan.export_blocks()
    vals, b = W.group_arrays(ws)
    num = plan.numeric(2, "f64")
    num.factor(torch.from_numpy(vals).cuda())
    db = torch.from_numpy(b).cuda()
    num.solve(db)
    xg = db.cpu().numpy()
    import paper_2110_12865_amd as S
    for k, w in enumerate(ws):
        p = w.pattern
        pl = S.analyze(p.colptr, p.rowind, w.perm)
        nm = pl.numeric(2, "f64")
        nm.factor(torch.from_numpy(np.ascontiguousarray(w.values)).cuda())
        d1 = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
        nm.solve(d1)
        x1 = d1.cpu().numpy()
        for s in range(2):
            assert oracle.forward_error(xg[s, 0, col0[k]:col0[k + 1]], x1[s, 0]) <= 1e-13


def test_autotuner_picks_a_measured_candidate():
    """The autotuner measures every candidate on the caller's data and
    returns the one with the smallest score (parity unpinned: there is no
    single right choice; the checks are validity and that the chosen plan
    solves correctly)."""
    import torch
    import paper_2110_12865_amd as S
    import oracle
    w = W.small_grid((12, 11, 10), "nd", seed=68, batch=20, nrhs=2)
    p = w.pattern
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    best, table = S.autotune(p.colptr, p.rowind, w.perm, vals, b, "f32", solves_per_factor=3.0)
    assert len(table) == 16  # 4 thresholds x 2 widths x 2 layouts (batch >= 16)
    assert all(t["factor_ms"] > 0 and t["solve_ms"] > 0 for t in table)
    scores = [t["score"] for t in table]
    k = int(np.argmin(scores))
    for key in ("small_front", "relax_cols", "soa_min_batch"):
        assert best[key] == table[k][key]
    assert np.array_equal(b.cpu().numpy(), w.b)  # the caller's right-hand sides are untouched
    plan = S.analyze(p.colptr, p.rowind, w.perm, **best)
    num = plan.numeric(w.batch, "f64")
    num.factor(vals)
    x = b.clone()
    num.solve(x)
    x = x.cpu().numpy()
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[3], sym)
    xo = oracle.solve(sym, Lx, w.b[3])
    assert oracle.forward_error(x[3, 1], xo[1]) <= 1e-12


def test_full_uneven_batch_against_oracle():
    """The whole uneven batch in the benchmark's launch configuration: 8
    patterns (2D 16^2 .. 128^2, 3D 8^3 .. 24^3, geometric nested
    dissection) x 32 value sets in one group plan.  FP64: for value sets 0
    and 31 of every pattern, the factor (per-column error <= 1e-12) and x
    (<= 1e-12) against the oracle run on that pattern alone.  FP32 factor +
    refinement to the stop rule: x of the same systems within 1e-10 of the
    oracle."""
    import paper_2110_12865_amd as S
    ws = W.config(3)
    plan = _group_plan(ws)
    col0, _ = plan.export_blocks()
    vals, b = W.group_arrays(ws)
    log("uneven batch: %d patterns x %d sets, n = %d" % (len(ws), vals.shape[0], b.shape[2]))
    dv = torch.from_numpy(vals).cuda()
    num = plan.numeric(vals.shape[0], "f64")
    num.factor(dv)
    assert np.all(num.info() == 0)
    db = torch.from_numpy(b).cuda()
    num.solve(db)
    x64 = db.cpu().numpy()
    n32 = plan.numeric(vals.shape[0], "f32")
    n32.factor(dv)
    assert np.all(n32.info() == 0)
    db = torch.from_numpy(b).cuda()
    x32 = torch.empty_like(db)
    rc, st = n32.refine_solve(dv, db, x32, tol=1e-10, maxit=10, method="classical")
    assert rc == S.SC_OK
    x32 = x32.cpu().numpy()
    for k, w in enumerate(ws):
        p = w.pattern
        sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
        cols = np.arange(col0[k], col0[k + 1], dtype=np.int32)
        for s in (0, w.batch - 1):
            Lx, inf = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
            assert inf == 0
            xo = oracle.solve(sym, Lx, w.b[s])
            ferr = oracle.factor_error(sym.Lcolptr, num.get_columns(s, cols), Lx)
            e64 = oracle.forward_error(x64[s, 0, col0[k]:col0[k + 1]], xo[0])
            e32 = oracle.forward_error(x32[s, 0, col0[k]:col0[k + 1]], xo[0])
            log("  %s set %d: factor err %.2e, x err f64 %.2e, f32+refinement %.2e"
                % (w.name, s, ferr, e64, e32))
            assert ferr <= 1e-12
            assert e64 <= 1e-12
            assert e32 <= 1e-10


def test_group_autotune_choice_is_valid():
    """sc_autotune_group times every candidate on the group plan and returns
    the one with the smallest score; the chosen options build a group plan
    whose solutions match the oracle (the choice itself has no single right
    answer: parity unpinned, validity checked)."""
    import paper_2110_12865_amd as S
    ws = _members(batch=3, nrhs=1)
    vals, b = W.group_arrays(ws)
    dv = torch.from_numpy(vals).cuda()
    db = torch.from_numpy(b).cuda()
    pats = [(w.pattern.colptr, w.pattern.rowind, w.perm) for w in ws]
    best, table = S.autotune_group(pats, dv, db, "f64", solves_per_factor=2.0)
    log("group autotune: %d candidates, best %s" % (len(table), best))
    assert len(table) == 8
    assert min(r["score"] for r in table) == pytest.approx(
        [r for r in table if all(r[k] == best[k] for k in ("small_front", "relax_cols",
                                                           "soa_min_batch"))][0]["score"])
    assert torch.equal(db, torch.from_numpy(b).cuda())      # b not modified
    opts = {k: best[k] for k in ("small_front", "relax_cols", "soa_min_batch")}
    plan = _group_plan(ws, **opts)
    col0, _ = plan.export_blocks()
    num = plan.numeric(vals.shape[0], "f64")
    num.factor(dv)
    assert np.all(num.info() == 0)
    num.solve(db)
    x = db.cpu().numpy()
    for k, w in enumerate(ws):
        p = w.pattern
        sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
        for s in range(w.batch):
            Lx, _ = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
            xo = oracle.solve(sym, Lx, w.b[s])
            assert oracle.forward_error(x[s, 0, col0[k]:col0[k + 1]], xo[0]) <= 1e-12
