"""Benchmark: sparse Cholesky factor + solve on one MI355X.

A step is one pass of the whole hot path over one batch of value sets:
numeric factorization (value scatter, assembly, dense front kernels) and
the solves with iterative refinement to the stop rule, from values and
right-hand sides already resident in HBM to the solution in HBM.  The
timed steps replay one captured HIP graph of the step (its refinement
budget is the step count an eager run needed; systems that have met the
stop rule are skipped on the device); the per-kernel table comes from one
extra eager step with per-launch events.
The symbolic analysis and the plan upload are one-time costs and are
excluded, as the paper excludes preprocessing.

Workloads (--workload):
  trimesh512 (default)  jittered 512 x 512 triangle mesh, cotangent stiffness
                        + 1e-3 * lumped mass, n = 262144, 64 value sets x 3
                        right-hand sides; FP32 factor + FP64 refinement, and
                        the FP64 factor, both to the same stop rule
                        (relres <= 1e-10 or the FP64 evaluation floor)
  grid3d64              3D 7-point 64^3 (n = 262144), nested dissection,
                        one value set, one right-hand side, FP64
  grid2d32              2D 5-point 32 x 32, natural order, FP64
  uneven8               uneven batch: 2D 16^2, 32^2, 64^2, 128^2 and 3D 8^3,
                        12^3, 16^3, 24^3, 32 value sets each (256 systems),
                        one group plan; FP32 + refinement versus FP64
  blockvec40            3 x 3 block vector Laplacian on a 40^3 grid
                        (n = 192000), 16 value sets, FP64: factor, solve and
                        the gradient of 0.5 ||x - x*||^2 in the values and b
                        (one more solve plus the value-gradient pass)

    python bench.py [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  Only the cpu_baseline leg calls the CPU oracle.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, GB/s
PEAK_MFMA_TFLOPS = {"f64": 78.6, "f32": 157.3}   # dense MFMA peaks
METRIC = "factor+solve per sec (batched FP32+refine vs FP64) at residual ≤1e-10; HBM GB/s"
TOL = 1e-10


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    import workloads as W
    if name == "trimesh512":
        return W.config(2), "trimesh_512x512_cotan_mass_nd_batch64_rhs3", "mixed"
    if name == "grid3d64":
        return W.config(1), "grid3d_7pt_64^3_nd", "f64"
    if name == "grid2d32":
        return W.config(0), "grid2d_5pt_32x32_natural", "f64"
    if name == "uneven8":
        return W.config(3), "uneven_8_patterns_x32_grid2d_grid3d_nd", "mixed"
    if name == "blockvec40":
        return W.config(4), "blockvec3_40^3_nd_batch16_adjoint", "adjoint"
    raise SystemExit("unknown workload %r" % name)


def relres_host(pat, values, x, b):
    """||b - A x||_2 / ||b||_2 with A from its lower triangle (scipy)."""
    import scipy.sparse as sp
    n = pat.n
    A = sp.csc_matrix((values, pat.rowind, pat.colptr), shape=(n, n))
    A = A + sp.tril(A, -1).T
    r = b - A @ x
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def leading_block(w, s, m):
    """Lower CSC of the leading m x m block of P A P^T for value set s."""
    p = w.pattern
    n = p.n
    perm = w.perm if w.perm is not None else np.arange(n, dtype=np.int32)
    pinv = np.empty(n, np.int64)
    pinv[perm] = np.arange(n)
    i = pinv[p.rows]
    j = pinv[p.cols]
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    keep = hi < m
    lo, hi, v = lo[keep], hi[keep], w.values[s][keep]
    order = np.lexsort((hi, lo))
    lo, hi, v = lo[order], hi[order], v[order]
    colptr = np.zeros(m + 1, np.int64)
    np.add.at(colptr, lo + 1, 1)
    colptr = np.cumsum(colptr)
    return colptr, hi.astype(np.int32), v, w.b[s][:, perm[:m]]


def cpu_baseline(w, flops_full, nnzL_full, budget_flops=5.0e10):
    """The CPU oracle (serial FP64) on a bounded sample of the workload.

    Whole systems are used when one costs at most the flop budget (as many
    value sets as fit, each factored and solved for all its right-hand
    sides); otherwise the leading block of P A P^T whose factor fits the
    budget, with factor and solve times scaled to the full system by the
    flop and nnz(L) ratios."""
    import oracle
    p = w.pattern
    n = p.n
    if flops_full <= budget_flops:
        sets = max(1, min(w.batch, int(budget_flops // max(flops_full, 1.0))))
        sets = min(sets, 24)
        t0 = time.perf_counter()
        sym = oracle.symbolic(n, p.colptr, p.rowind, w.perm)
        t1 = time.perf_counter()
        for s in range(sets):
            Lx, info = oracle.factor(n, p.colptr, p.rowind, w.values[s], sym)
            oracle.solve(sym, Lx, w.b[s])
        t2 = time.perf_counter()
        per = (t2 - t1) / sets
        return {"value": 1.0 / per, "unit": "factor+solve/s", "cores": 1, "kind": "oracle",
                "sample": "%d whole value set(s) of the workload, factor + solve of all %d "
                          "right-hand sides each, FP64 direct (no refinement needed); "
                          "%.2f s measured" % (sets, w.nrhs, t2 - t1),
                "oracle_gflops": flops_full * sets / (t2 - t1) / 1e9}
    m = n
    # largest leading block within the budget (flops grow fast near the top)
    for frac in (0.5, 0.375, 0.25, 0.1875, 0.125, 0.0625):
        mm = int(n * frac)
        sym = oracle.symbolic(n, p.colptr, p.rowind, w.perm, nrows=mm)
        if sym.flops() <= budget_flops:
            m = mm
            break
    colptr, rowind, v, b = leading_block(w, 0, m)
    sym = oracle.symbolic(m, colptr, rowind, None)
    t1 = time.perf_counter()
    Lx, info = oracle.factor(m, colptr, rowind, v, sym)
    t2 = time.perf_counter()
    oracle.solve(sym, Lx, b)
    t3 = time.perf_counter()
    tf = (t2 - t1) * flops_full / sym.flops()
    ts = (t3 - t2) * nnzL_full / sym.nnzL
    return {
        "value": 1.0 / (tf + ts),
        "unit": "factor+solve/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("leading %dx%d block of P A P^T (%.3g flops, nnz(L) %d); measured "
                   "factor %.2f s, solve %.3f s; scaled by flop and nnz(L) ratios to the "
                   "full system" % (m, m, sym.flops(), sym.nnzL, t2 - t1, t3 - t2)),
        "projected_factor_s": tf,
        "projected_solve_s": ts,
        "oracle_gflops": sym.flops() / (t2 - t1) / 1e9,
    }


def cpu_baseline_group(ws, budget_s=12.0):
    """The CPU oracle on whole value sets of every pattern of a group (one
    set of all patterns after another, until the time budget is spent)."""
    import oracle
    syms = [oracle.symbolic(w.pattern.n, w.pattern.colptr, w.pattern.rowind, w.perm)
            for w in ws]
    t0 = time.perf_counter()
    sets = 0
    while sets < ws[0].batch:
        for w, sym in zip(ws, syms):
            p = w.pattern
            Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[sets], sym)
            oracle.solve(sym, Lx, w.b[sets])
        sets += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    flops = sum(s.flops() for s in syms) * sets
    return {"value": sets * len(ws) / dt, "unit": "factor+solve/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d value set(s) of each of the %d patterns, factor + solve, FP64 "
                      "direct; %.2f s measured" % (sets, len(ws), dt),
            "oracle_gflops": flops / dt / 1e9}


def kernel_table(prof, steps):
    kern = {}
    total_bytes = 0.0
    for name, st in prof.items():
        kern[name] = {"launches_per_step": st["launches"] / steps,
                      "ms_per_step": st["ms"] / steps,
                      "gflop_s": st["flops"] / max(st["ms"], 1e-9) / 1e6,
                      "gb_s": st["bytes"] / max(st["ms"], 1e-9) / 1e6}
        total_bytes += st["bytes"]
    return kern, total_bytes


# kernel kinds of the library's per-launch records and the HIP kernels they
# time (kinds that bracket more than one kernel family are not candidates
# for the roofline line)
HIP_KERNEL = {
    "front_small": "k_front_reg|k_front_wg", "assemble": "k_assemble_cols", "potrf": "k_potrf",
    "trsm": "k_trsm", "syrk_mfma": "k_syrk", "diag_inverse": "k_dinv",
    "solve_fwd": "k_fwd_soa_diag|k_fwd_seg", "solve_bwd": "k_bwd_soa_diag|k_bwd_seg",
    "solve_fwd_rows": "k_fwd_soa_rows", "solve_bwd_rows": "k_bwd_soa_rows",
    "solve_fwd_panel": "k_pan_gather|k_fwd_panel|k_fwd_sn",
    "solve_bwd_panel": "k_bwd_pan_part|k_bwd_pan_fin|k_bwd_sn",
    "solve_gather": "k_gather", "spmv_residual": "k_apply|k_apply2",
    "solve_copy_interleaved": "k_to_soa",
}


def source_digest():
    """sha256 of the library sources: HBM counters taken on other sources
    are stale."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2110_12865_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(workload, kind):
    """HBM bytes per launch of `kind` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a copy kernel of known
    size), or None when there is none for this workload and kernel or the
    sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    e = t.get(workload, {})
    if e.get("kernel") != kind or e.get("source_sha256") != source_digest():
        return None
    return e.get("bytes_per_launch")


def roofline(prof, dtype, workload):
    cand = {k: v for k, v in prof.items() if k in HIP_KERNEL}
    name, st = max(cand.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = st["ms"] / st["launches"]
    if name == "syrk_mfma":
        ach = st["flops"] / st["launches"] / (avg_ms * 1e-3) / 1e12
        roof = {"kernel": name, "bound": "mfma", "achieved": ach,
                "peak": PEAK_MFMA_TFLOPS[dtype], "unit": "TFLOP/s"}
    else:
        ach = st["bytes"] / st["launches"] / (avg_ms * 1e-3) / 1e9
        roof = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(workload, name)
    roof["hip_kernel"] = HIP_KERNEL[name]
    roof["avg_launch_ms"] = avg_ms
    roof["launches"] = st["launches"]
    roof["algorithmic_bytes_per_launch"] = st["bytes"] / st["launches"]
    return roof


def run_form(S, plan, w, dtype, steps, warmup, profile):
    """Time `steps` steps of one form: factor of the whole batch plus the
    refined solve to the stop rule, replayed as one captured HIP graph whose
    refinement budget is the step count an eager run needed (systems that
    have met the rule are skipped on the device).  Returns (seconds,
    per-system stats of the last replay, x, per-kernel profile of one eager
    step, refinement steps)."""
    import torch
    num = plan.numeric(w.batch, dtype)
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    b0 = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    x = torch.empty_like(b0)
    method = "pcg"
    # eager step: the refinement budget and a factorization check
    num.factor(vals)
    bad = num.info()
    if np.any(bad):
        raise SystemExit("factorization failed (%s): info=%s" % (dtype, bad[bad != 0][:8]))
    rc, st0 = num.refine_solve(vals, b0, x, tol=TOL, maxit=30, method=method)
    iters = max(s["iters"] for s in st0)
    g = num.step_graph(vals, b0, x, tol=TOL, iters=iters, method=method)
    for _ in range(warmup):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, stats = g.stats()
    out = x.cpu().numpy()
    prof = {}
    if profile:
        # one eager step with per-launch events, for the kernel table
        num.profile(True)
        num.factor(vals)
        num.refine_solve(vals, b0, x, tol=TOL, maxit=iters, method=method)
        torch.cuda.synchronize()
        num.profile(False)
        prof = num.profile_read()
    del g
    del num
    torch.cuda.empty_cache()
    return t1 - t0, stats, out, prof, iters

def run_adjoint(S, plan, w, steps, warmup, profile):
    """Time `steps` steps of factor + solve + adjoint (the gradient of
    0.5 ||x - x*||^2 in the values and in b) over the batch."""
    import torch
    num = plan.numeric(w.batch, "f64")
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    b0 = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    xs = torch.from_numpy(np.ascontiguousarray(w.extra["xstar"])).cuda()
    x = torch.empty_like(b0)
    gx = torch.empty_like(b0)

    def step():
        num.factor(vals)
        x.copy_(b0)
        num.solve(x)
        torch.sub(x, xs, out=gx)
        return num.adjoint(x, gx)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    bad = num.info()
    if np.any(bad):
        raise SystemExit("factorization failed: info=%s" % bad[bad != 0][:8])
    t0 = time.perf_counter()
    for _ in range(steps):
        gv, gb = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {}
    if profile:
        num.profile(True)
        step()
        torch.cuda.synchronize()
        num.profile(False)
        prof = num.profile_read()
    return t1 - t0, x.cpu().numpy(), gv.cpu().numpy(), gb.cpu().numpy(), prof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="trimesh512")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="no per-launch events")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only copy this many MiB device to device once (calibration of "
                         "the HBM byte counters) and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default options instead of the autotuner's choice")
    ap.add_argument("--soa-min-batch", type=int, default=None,
                    help="batch size from which solves use the batch-interleaved layout "
                         "(library default when omitted, negative: never)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    if args.calib_copy_mib > 0:
        import torch
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nbytes}), flush=True)
        return 0

    import paper_2110_12865_amd as S

    import workloads as W
    w, wname, form = make_workload(args.workload)
    members = None
    if isinstance(w, list):
        # uneven batch: one group plan over all patterns
        members = w
        vals, b = W.group_arrays(members)
        w = W.Workload(wname, None, None, vals, b, members[0].seed)
        nnz = sum(m.pattern.nnz for m in members)
        n = sum(m.pattern.n for m in members)
    else:
        n, nnz = w.pattern.n, w.pattern.nnz
    p = w.pattern
    log("workload %s n=%d nnzA=%d batch=%d nrhs=%d" % (wname, n, nnz, w.batch, w.nrhs))
    t = time.perf_counter()
    opts = {} if args.soa_min_batch is None else {"soa_min_batch": args.soa_min_batch}
    tuned = None
    if members is None and not args.no_tune and args.soa_min_batch is None:
        # one-time tuning of thresholds, amalgamation and solve layout on this
        # workload (like the analysis, outside the timed steps)
        import torch
        tt = time.perf_counter()
        tv = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
        tb = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
        best, table = S.autotune(p.colptr, p.rowind, w.perm, tv, tb,
                                 "f32" if form == "mixed" else "f64",
                                 solves_per_factor={"mixed": 4.0, "adjoint": 2.0}.get(form, 1.0))
        del tv, tb
        torch.cuda.empty_cache()
        opts = {k: best[k] for k in ("small_front", "relax_cols", "soa_min_batch")}
        tuned = {"options": opts, "seconds": time.perf_counter() - tt,
                 "candidates": [{k: round(r[k], 4) if isinstance(r[k], float) else r[k]
                                 for k in ("small_front", "relax_cols", "soa_min_batch",
                                           "factor_ms", "solve_ms", "score")} for r in table]}
        log("autotune %.1f s: %s" % (tuned["seconds"], opts))
    t = time.perf_counter()
    if members is not None:
        plan = S.analyze_group([(m.pattern.colptr, m.pattern.rowind, m.perm) for m in members],
                               **opts)
    else:
        plan = S.analyze(p.colptr, p.rowind, w.perm, **opts)
    info = plan.info()
    nblk = info["nblocks"]
    log("analyze %.2f s: nnzL=%d supernodes=%d levels=%d flops=%.3e" % (
        time.perf_counter() - t, info["nnzL"], info["nsuper"], info["nlevels"], info["flops"]))
    prof_on = not args.no_profile
    out = {"metric": METRIC, "unit": "factor+solve/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic"}
    cfg = {"workload": wname, "n": n, "nnzA": nnz, "nnzL": info["nnzL"],
           "batch": w.batch, "nrhs": w.nrhs,
           "ordering": ("geometric nested dissection"
                        if members is not None or w.perm is not None else "natural"),
           "flops_sum_c2_per_system": info["flops"], "supernodes": info["nsuper"],
           "levels": info["nlevels"]}
    if tuned is not None:
        cfg["autotuned"] = tuned
    if members is not None:
        cfg["patterns"] = [m.name for m in members]
        cfg["matrices_per_step"] = w.batch * nblk
        cfg["flops_sum_c2_per_system"] = info["flops"] / nblk
    if form == "mixed":
        # FP64 form first (reference of the comparison), then the headline form
        t64, st64, x64, _, it64 = run_form(S, plan, w, "f64", args.steps, args.warmup, False)
        log("fp64 form: %.3f ms/step" % (t64 * 1e3 / args.steps))
        t32, st32, x32, prof, it32 = run_form(S, plan, w, "f32", args.steps, args.warmup,
                                              prof_on)
        log("fp32+refinement form: %.3f ms/step" % (t32 * 1e3 / args.steps))
        ms = t32 * 1e3 / args.steps
        nmat = w.batch * nblk
        out.update({"value": nmat / (t32 / args.steps), "ms_per_step": ms,
                    "dtype": "f32 factor, f64 residual/update"})
        iters = [s["iters"] for s in st32]
        clauses = [s["clause"] for s in st32]
        out["fp64_form"] = {"value": nmat / (t64 / args.steps),
                            "ms_per_step": t64 * 1e3 / args.steps,
                            "refinement_budget": it64,
                            "iters_max": max(s["iters"] for s in st64),
                            "relres_max": max(s["relres"] for s in st64),
                            "clauses": sorted(set(s["clause"] for s in st64))}
        out["speedup_vs_fp64_form"] = out["value"] / out["fp64_form"]["value"]
        out["refinement"] = {"method": "pcg", "budget": it32, "iters_max": max(iters),
                             "iters_mean": float(np.mean(iters)),
                             "relres_max": max(s["relres"] for s in st32),
                             "clause_counts": {str(c): clauses.count(c)
                                               for c in sorted(set(clauses))},
                             "fwd_err_vs_fp64_form_max": float(max(
                                 np.abs(x32[s] - x64[s]).max() / np.abs(x64[s]).max()
                                 for s in range(w.batch)))}
        if 0 in clauses or 0 in set(s["clause"] for s in st64):
            raise SystemExit("a system did not meet the stop rule")
        # independent residual check on the first and last value sets
        if members is None:
            rr = max(relres_host(p, w.values[s], x32[s, r], w.b[s, r])
                     for s in (0, w.batch - 1) for r in range(w.nrhs))
        else:
            col0, val0 = plan.export_blocks()
            rr = max(relres_host(m.pattern, w.values[s, val0[k]:val0[k + 1]],
                                 x32[s, r, col0[k]:col0[k + 1]], w.b[s, r, col0[k]:col0[k + 1]])
                     for k, m in enumerate(members) for s in (0, w.batch - 1)
                     for r in range(w.nrhs))
        out["relres_check_host"] = rr
        pdtype = "f32"
    elif form == "adjoint":
        t, x, gv, gb, prof = run_adjoint(S, plan, w, args.steps, args.warmup, prof_on)
        ms = t * 1e3 / args.steps
        out.update({"value": w.batch / (t / args.steps), "ms_per_step": ms, "dtype": "f64",
                    "unit": "factor+solve+gradient/s"})
        # the gradient of value set 0 against the closed form at sampled entries
        lam = gb[0, 0]
        xs = x[0, 0]
        ks = np.random.default_rng(0).choice(p.nnz, size=1000, replace=False)
        ref = np.where(p.rows[ks] == p.cols[ks], -lam[p.rows[ks]] * xs[p.cols[ks]],
                       -(lam[p.rows[ks]] * xs[p.cols[ks]] + lam[p.cols[ks]] * xs[p.rows[ks]]))
        out["gradient_check_max_rel"] = float(np.max(np.abs(gv[0, ks] - ref) /
                                                     np.maximum(np.abs(ref), 1e-300)))
        out["relres"] = max(relres_host(p, w.values[s], x[s, r], w.b[s, r])
                            for s in (0, w.batch - 1) for r in range(w.nrhs))
        pdtype = "f64"
    else:
        t64, st64, x, prof, it64 = run_form(S, plan, w, "f64", args.steps, args.warmup, prof_on)
        ms = t64 * 1e3 / args.steps
        out.update({"value": w.batch / (t64 / args.steps), "ms_per_step": ms, "dtype": "f64",
                    "refinement_budget": it64})
        if 0 in set(s["clause"] for s in st64):
            raise SystemExit("a system did not meet the stop rule")
        out["relres"] = max(relres_host(p, w.values[s], x[s, r], w.b[s, r])
                            for s in range(w.batch) for r in range(w.nrhs))
        pdtype = "f64"
    out["config"] = cfg
    log("timed %d steps: %.3f ms/step" % (args.steps, ms))
    if prof:
        kern, total_bytes = kernel_table(prof, 1)  # one eager profiled step
        out["kernels"] = kern
        out["hbm_gb_s_step"] = total_bytes / (ms * 1e-3) / 1e9
        out["roofline"] = roofline(prof, pdtype, wname)
    if not args.no_cpu:
        log("cpu baseline (oracle on a bounded sample)...")
        if members is not None:
            out["cpu_baseline"] = cpu_baseline_group(members)
        else:
            out["cpu_baseline"] = cpu_baseline(w, info["flops"], info["nnzL"])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
