"""GPU iterative refinement: FP32 factor with FP64 residual and update, and
the FP64 factor under the same stop rule, against the FP64 oracle.

Stop rule per (matrix, rhs): relres = ||b - A x||_2 / ||b||_2 <= tol, or
||r||_2 <= 2 u ||A||_inf ||x||_2 (the FP64 evaluation floor).  After
refinement the solution must agree with the oracle's FP64 solution to
1e-10 (forward error, infinity norm) on the well-conditioned grid systems."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_helpers import log, oracle_run

pytestmark = pytest.mark.gpu


def _refine(w, dtype, tol=1e-10, maxit=10, method="classical", **opts):
    import paper_2110_12865_amd as S
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm, **opts)
    num = plan.numeric(w.batch, dtype)
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    num.factor(vals)
    assert np.all(num.info() == 0)
    b = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    x = torch.empty_like(b)
    rc, stats = num.refine_solve(vals, b, x, tol=tol, maxit=maxit, method=method)
    return rc, stats, x.cpu().numpy()


@pytest.mark.parametrize("method", ["classical", "pcg"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_refine_matches_fp64_oracle(dtype, method):
    import paper_2110_12865_amd as S
    w = W.small_grid((14, 14, 14), "nd", seed=61, batch=3, nrhs=2)
    rc, stats, x = _refine(w, dtype, method=method)
    assert rc == S.SC_OK
    p = w.pattern
    for s in range(w.batch):
        sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
        Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
        xo = oracle.solve(sym, Lx, w.b[s])
        relres, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[s], x[s], w.b[s])
        for r in range(w.nrhs):
            st = stats[s * w.nrhs + r]
            err = oracle.forward_error(x[s, r], xo[r])
            log("%s set %d rhs %d: iters %d clause %d relres %.2e (oracle %.2e) err %.2e" % (
                dtype, s, r, st["iters"], st["clause"], st["relres"], relres[r], err))
            assert st["clause"] in (1, 2)
            assert relres[r] <= 1e-10
            # the two residuals differ by the rounding of b - A x in another
            # summation order, about u ||A|| ||x|| / ||b|| <= 1e-14 here
            assert abs(st["relres"] - relres[r]) <= 1e-3 * relres[r] + 1e-14
            assert err <= 1e-10
            if dtype == "f64":
                assert st["iters"] == 0
            else:
                assert 1 <= st["iters"] <= 4


def test_refine_reports_no_convergence():
    import paper_2110_12865_amd as S
    w = W.small_grid((12, 12, 12), "nd", seed=62)
    rc, stats, x = _refine(w, "f32", tol=1e-10, maxit=0)
    assert rc == S.SC_ENOCONV
    assert stats[0]["clause"] == 0 and stats[0]["iters"] == 0
    assert 1e-10 < stats[0]["relres"] < 1e-4


@pytest.mark.parametrize("method", ["classical", "pcg"])
def test_refine_ill_conditioned_mesh_reaches_floor(method):
    """Cotangent stiffness + 1e-3 lumped mass (the 512^2 mesh construction at
    64^2): kappa ~ 1e7-1e8.  Every system must stop by one of the two
    clauses, within a few corrections."""
    import paper_2110_12865_amd as S
    w = W.trimesh_workload(64, 4, 3, seed=63)
    rc, stats, x = _refine(w, "f32", maxit=20, method=method)
    for st in stats:
        log("mesh: iters %d clause %d relres %.2e" % (st["iters"], st["clause"], st["relres"]))
    assert rc == S.SC_OK
    assert all(st["clause"] in (1, 2) for st in stats)
    p = w.pattern
    sym, Lx, _, xo = oracle_run(w, 0)
    relres_o, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[0], xo, w.b[0])
    relres_g, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[0], x[0], w.b[0])
    # the refined FP32 result is as good as the direct FP64 solve, up to 10x
    assert np.all(relres_g <= np.maximum(10 * relres_o, 1e-10))


@pytest.mark.parametrize("method", ["classical", "pcg"])
def test_refine_six_rhs_floor_clause_against_host_norm(method):
    """Six right-hand sides (two passes of the residual product, 4 + 2) on
    the ill-conditioned 64^2 mesh: every system stops; a system stopped by
    the floor clause satisfies ||r||_2 <= 2 u ||A||_inf ||x||_2 with its own
    recorded norms and ||A||_inf computed on the host (the device takes
    ||A||_inf from the first residual pass); a system stopped by the first
    clause has relres <= tol; each refined x is as good as the direct FP64
    solve."""
    import paper_2110_12865_amd as S
    w = W.trimesh_workload(64, 2, 6, seed=69)
    tol = 1e-10
    rc, stats, x = _refine(w, "f32", tol=tol, maxit=20, method=method)
    assert rc == S.SC_OK
    p = w.pattern
    u = np.finfo(np.float64).eps / 2
    nfloor = 0
    for s in range(w.batch):
        anorm = oracle.norm_inf_sym(p.n, p.colptr, p.rowind, w.values[s])
        sym, Lx, _, xo = oracle_run(w, s)
        relres_o, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[s], xo, w.b[s])
        relres_g, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[s], x[s], w.b[s])
        for r in range(w.nrhs):
            st = stats[s * w.nrhs + r]
            log("%s set %d rhs %d: iters %d clause %d relres %.2e rnorm %.3e xnorm %.3e ||A|| %.6e"
                % (method, s, r, st["iters"], st["clause"], st["relres"], st["rnorm"],
                   st["xnorm"], anorm))
            assert st["clause"] in (1, 2)
            if st["clause"] == 1:
                assert st["relres"] <= tol
            else:
                nfloor += 1
                assert st["rnorm"] <= 2 * u * anorm * st["xnorm"] * (1 + 1e-12)
            assert relres_g[r] <= max(10 * relres_o[r], tol)
    log("%s: %d of %d systems stopped on the floor clause" % (method, nfloor, len(stats)))


def test_refine_batch_matches_single_bitwise():
    w = W.small_grid((10, 10, 10), "nd", seed=64, batch=3, nrhs=1)
    rc, stats, xb = _refine(w, "f32")
    w1 = W.Workload("one", w.pattern, w.perm, w.values[1:2].copy(), w.b[1:2].copy(), 0)
    rc1, stats1, x1 = _refine(w1, "f32")
    assert np.array_equal(xb[1], x1[0])
    assert stats[1]["iters"] == stats1[0]["iters"]


def test_pcg_converges_where_classical_stalls():
    """The 512^2 mesh construction at 256^2 keeps kappa ~ 2.5e9 (the mass
    term scales as 1/n), so kappa * u_32 >> 1: classical refinement with the
    FP32 factor stalls, preconditioned CG reaches the stop rule."""
    import paper_2110_12865_amd as S
    w = W.trimesh_workload(256, 2, 1, seed=65)
    rc_c, st_c, _ = _refine(w, "f32", maxit=15, method="classical")
    rc_p, st_p, x = _refine(w, "f32", maxit=40, method="pcg")
    for a, b in zip(st_c, st_p):
        log("256^2 mesh: classical relres %.2e clause %d | pcg iters %d relres %.2e clause %d"
            % (a["relres"], a["clause"], b["iters"], b["relres"], b["clause"]))
    assert rc_p == S.SC_OK
    assert all(s["clause"] in (1, 2) for s in st_p)
    p = w.pattern
    for s in range(w.batch):
        sym, Lx, _, xo = oracle_run(w, s)
        relres_o, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[s], xo, w.b[s])
        relres_g, _ = oracle.residual_measures(p.n, p.colptr, p.rowind, w.values[s], x[s], w.b[s])
        log("  set %d: direct FP64 relres %.2e, pcg relres %.2e" % (s, relres_o[0], relres_g[0]))
        assert relres_g[0] <= max(10 * relres_o[0], 1e-10)


@pytest.mark.parametrize("method", ["classical", "pcg"])
def test_refine_interleaved_batch_matches_single_bitwise(method):
    """A batch of 40 refines in the batch-interleaved layout; element 17 is
    bit-identical to the same system refined alone (row-major layout), with
    the same iteration count (whole-block inverses off: they apply to
    batches of 16 or more only)."""
    w = W.small_grid((12, 11, 10), "nd", seed=65, batch=40, nrhs=2)
    rc, stats, xb = _refine(w, "f32", method=method, soa_min_batch=32, panel_inverse=-1)
    w1 = W.Workload("one", w.pattern, w.perm, w.values[17:18].copy(), w.b[17:18].copy(), 0)
    rc1, stats1, x1 = _refine(w1, "f32", method=method, panel_inverse=-1)
    assert np.array_equal(xb[17], x1[0])
    for r in range(2):
        assert stats[17 * 2 + r]["iters"] == stats1[r]["iters"]


@pytest.mark.parametrize("batch,soa", [(4, -1), (64, 64)], ids=["rowmajor", "interleaved"])
@pytest.mark.parametrize("method", ["classical", "pcg"])
def test_step_graph_replays_match_eager(method, batch, soa):
    """The captured factor + refinement step, replayed three times with
    unrelated eager work and synchronizations in between, reproduces the
    eager sc_refine_solve result bit for bit on every replay (the output is
    cleared before each replay), with the same per-system statistics."""
    import paper_2110_12865_amd as S
    w = W.small_grid((11, 10, 9), "nd", seed=66, batch=batch, nrhs=2)
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm, soa_min_batch=soa)
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    # eager reference
    ne = plan.numeric(w.batch, "f32")
    ne.factor(vals)
    xe = torch.empty_like(b)
    rc_e, st_e = ne.refine_solve(vals, b, xe, tol=1e-10, maxit=4, method=method)
    xe = xe.cpu().numpy()
    # captured step on its own numeric object
    ng = plan.numeric(w.batch, "f32")
    xg = torch.empty_like(b)
    g = ng.step_graph(vals, b, xg, tol=1e-10, iters=4, method=method)
    other = W.small_grid((7, 6, 5), "nd", seed=67, batch=2, nrhs=1)
    for rep in range(3):
        xg.zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        rc_g, st_g = g.stats()
        assert rc_g == rc_e
        assert np.array_equal(xg.cpu().numpy(), xe), "replay %d" % rep
        for a, e in zip(st_g, st_e):
            assert a["iters"] == e["iters"] and a["clause"] == e["clause"]
            assert a["relres"] == e["relres"]
        # unrelated eager work between replays
        from tests.gpu_helpers import run_library
        run_library(other, "f64")
        torch.cuda.synchronize()


def test_step_graph_blocks_workspace_growth():
    """A captured graph holds the numeric object's workspace addresses: while
    it exists, calls on the same object that would need larger workspaces
    (more right-hand sides, a larger leading dimension) are refused with
    SC_EINVAL instead of reallocating under the graph.  The graph is not
    replayed after a refused call; once it is destroyed the same calls run
    and agree with a fresh numeric object."""
    import paper_2110_12865_amd as S
    w = W.small_grid((9, 8, 7), "nd", seed=68, batch=2, nrhs=3)
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm)
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    b1 = torch.from_numpy(np.ascontiguousarray(w.b[:, :1])).cuda()
    x1 = torch.empty_like(b1)
    num = plan.numeric(w.batch, "f32")
    g = num.step_graph(vals, b1, x1, tol=1e-10, iters=3, method="pcg")
    g.launch()
    torch.cuda.synchronize()
    rc, _ = g.stats()
    assert rc == S.SC_OK
    b3 = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    x3 = torch.empty_like(b3)
    with pytest.raises(S.SpcholError) as ei:
        num.solve(b3.clone())                      # 3 right-hand sides > 1
    assert ei.value.status == S.SC_EINVAL
    with pytest.raises(S.SpcholError) as ei:
        num.refine_solve(vals, b3, x3, tol=1e-10, maxit=3, method="pcg")
    assert ei.value.status == S.SC_EINVAL
    wide = torch.zeros((w.batch, 1, p.n + 5), dtype=torch.float64, device="cuda")
    wide[:, :, :p.n] = b1
    with pytest.raises(S.SpcholError) as ei:       # larger leading dimension
        num.refine_solve(vals, wide, torch.empty_like(wide), tol=1e-10, maxit=3)
    assert ei.value.status == S.SC_EINVAL
    # a solve that fits the existing workspaces is still allowed
    xs = b1.clone()
    num.solve(xs)
    g.destroy()
    del g
    torch.cuda.synchronize()
    xb = b3.clone()
    num.solve(xb)                                   # grows now
    fresh = plan.numeric(w.batch, "f32")
    fresh.factor(vals)
    xf = b3.clone()
    fresh.solve(xf)
    assert torch.equal(xb, xf)


def test_full_size_mesh_refined_against_oracle():
    """The 512^2 mesh in the benchmark's launch configuration (64 value
    sets, 3 right-hand sides, FP32 factor, PCG refinement to the stop rule):
    x of value sets 0 and 63 against the FP64 oracle, accepted at 1e-10 or,
    as the system's conditioning demands (kappa_1 ~ 1e9..1e10), within
    10 kappa_1 u with kappa_1 estimated from oracle solves; every system's
    stop clause re-evaluated by the oracle on the host."""
    import paper_2110_12865_amd as S
    w = W.config(2)
    p = w.pattern
    log("mesh 512^2: batch %d, %d rhs" % (w.batch, w.nrhs))
    plan = S.analyze(p.colptr, p.rowind, w.perm)
    num = plan.numeric(w.batch, "f32")
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    num.factor(vals)
    assert np.all(num.info() == 0)
    b = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    x = torch.empty_like(b)
    rc, stats = num.refine_solve(vals, b, x, tol=1e-10, maxit=30, method="pcg")
    assert rc == S.SC_OK
    x = x.cpu().numpy()
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    for s in (0, w.batch - 1):
        Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
        assert info == 0
        xo = oracle.solve(sym, Lx, w.b[s])
        kap = oracle.kappa1_estimate(p.n, p.colptr, p.rowind, w.values[s], sym, Lx)
        cl = oracle.stop_clause(p.n, p.colptr, p.rowind, w.values[s], x[s], w.b[s], 1e-10)
        for r in range(w.nrhs):
            err = oracle.forward_error(x[s, r], xo[r])
            log("  set %d rhs %d: x err %.2e, kappa_1 ~ %.2e, clause %d (GPU %d)"
                % (s, r, err, kap, cl[r], stats[s * w.nrhs + r]["clause"]))
            assert oracle.within_conditioning(err, 1e-10, kap)
            assert cl[r] in (1, 2)
