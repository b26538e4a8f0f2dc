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


def host_info():
    """The host CPU as lscpu reports it (model, sockets, cores, threads)."""
    import subprocess
    keys = {"Model name": "model", "CPU(s)": "cpus", "Thread(s) per core": "threads_per_core",
            "Core(s) per socket": "cores_per_socket", "Socket(s)": "sockets"}
    out = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:
        return out
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keys:
            out[keys[k.strip()]] = v.strip()
    return out


def cpu_threads():
    """Threads for the N-thread oracle run: the CPUs this process may use,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(w, flops_full, nnzL_full, budget_flops=5.0e10, x_gpu=None):
    """The CPU oracle (serial FP64) on a bounded sample of the workload.

    Whole systems are used when one costs at most the flop budget (as many
    value sets as fit, each factored and solved for all its right-hand
    sides); otherwise the leading block of P A P^T whose factor fits the
    budget, with factor and solve times scaled to the full system by the
    flop and nnz(L) ratios.  With whole systems, the oracle's solutions are
    also compared with the GPU's (x_gpu: {form: x[batch, nrhs, n]}): forward
    error ||x - x_o||_inf / ||x_o||_inf per system, accepted at 1e-10 or,
    beyond that, within 10 kappa_1 u (kappa_1 estimated from oracle solves);
    that comparison is outside the timed factor and solve calls."""
    import oracle
    p = w.pattern
    n = p.n
    if flops_full <= budget_flops:
        sets = max(1, min(w.batch, int(budget_flops // max(flops_full, 1.0))))
        sets = min(sets, 24)
        sym = oracle.symbolic(n, p.colptr, p.rowind, w.perm)
        t_meas = 0.0
        worst = {}
        kappas = []
        for s in range(sets):
            t1 = time.perf_counter()
            Lx, info = oracle.factor(n, p.colptr, p.rowind, w.values[s], sym)
            xo = oracle.solve(sym, Lx, w.b[s])
            t_meas += time.perf_counter() - t1
            if not x_gpu:
                continue
            kap = oracle.kappa1_estimate(n, p.colptr, p.rowind, w.values[s], sym, Lx)
            kappas.append(kap)
            for form, xg in x_gpu.items():
                wf = worst.setdefault(form, {"fwd_err_max": 0.0, "systems": 0, "accepted": 0,
                                             "within_1e-10": 0})
                for r in range(w.nrhs):
                    e = oracle.forward_error(xg[s, r], xo[r])
                    wf["fwd_err_max"] = max(wf["fwd_err_max"], e)
                    wf["systems"] += 1
                    wf["within_1e-10"] += int(e <= TOL)
                    wf["accepted"] += int(oracle.within_conditioning(e, TOL, kap))
        res = {"value": sets / t_meas, "unit": "factor+solve/s", "cores": 1, "kind": "oracle",
               "sample": "%d whole value set(s) of the workload, factor + solve of all %d "
                         "right-hand sides each, FP64 direct (no refinement needed); "
                         "%.2f s measured" % (sets, w.nrhs, t_meas),
               "oracle_gflops": flops_full * sets / t_meas / 1e9}
        res["threads"] = cpu_baseline_threads(w, sym)
        res["host"] = host_info()
        if x_gpu:
            res["vs_oracle"] = {"value_sets": sets, "kappa1_est_max": max(kappas),
                                "rule": "fwd err <= 1e-10, else <= 10 kappa_1 u",
                                "forms": worst}
        return res
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
        "host": host_info(),
    }


def cpu_baseline_threads(w, sym):
    """The same serial oracle on N threads, each factoring and solving its own
    value sets (independent systems; the C calls release the interpreter
    lock): throughput in systems per second over about two sets per
    thread."""
    import concurrent.futures
    import oracle
    p = w.pattern
    nt = cpu_threads()
    sets = min(w.batch, 2 * nt)

    def one(s):
        Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
        oracle.solve(sym, Lx, w.b[s])
        return info

    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=nt) as ex:
        list(ex.map(one, range(sets)))
    dt = time.perf_counter() - t0
    return {"value": sets / dt, "unit": "factor+solve/s", "cores": nt,
            "sample": "%d value sets on %d threads of the serial oracle, %.2f s wall"
                      % (sets, nt, dt)}


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
    """Per kernel family: launches, time, and rates of the algorithmic work
    (flops; the survey's algorithmic bytes: A read plus L written for the
    factor, L read once per sweep for the solves, A read for the residual
    products) and of the library's own byte model of what each launch moves
    (front and update blocks, vectors, indices).  A model rate above the HBM
    peak means that family's working set is served from cache, so it is not
    an HBM figure."""
    kern = {}
    total_alg = 0.0
    for name, st in prof.items():
        ms = max(st["ms"], 1e-9)
        e = {"launches_per_step": st["launches"] / steps, "ms_per_step": st["ms"] / steps,
             "gflop_s": st["flops"] / ms / 1e6,
             "alg_gb_s": st["alg_bytes"] / ms / 1e6,
             "model_gb_s": st["bytes"] / ms / 1e6}
        if e["model_gb_s"] > PEAK_HBM_GBS:
            e["note"] = "model bytes above the HBM peak: cache-resident, not HBM traffic"
        kern[name] = e
        total_alg += st["alg_bytes"]
    return kern, total_alg


# kernel kinds of the library's per-launch records and the HIP kernels they
# time
HIP_KERNEL = {
    "front_small": "k_front_reg|k_front_wg", "assemble": "k_assemble_cols", "potrf": "k_potrf",
    "trsm": "k_trsm", "syrk_mfma": "k_syrk", "diag_inverse": "k_dinv",
    "solve_fwd": "k_fwd_soa_diag|k_fwd_seg", "solve_bwd": "k_bwd_soa_diag|k_bwd_seg",
    "solve_fwd_rows": "k_fwd_soa_rows", "solve_bwd_rows": "k_bwd_soa_rows",
    "solve_fwd_panel": "k_pan_gather|k_fwd_panel|k_fwd_sn",
    "solve_bwd_panel": "k_bwd_pan_part|k_bwd_pan_fin|k_bwd_sn",
    "solve_gather": "k_gather", "spmv_residual": "k_apply|k_apply2",
    "solve_copy_interleaved": "k_to_soa", "refine_vector": "refinement vector kernels",
    "solve_permute": "k_perm_in|k_perm_out",
}
# families whose work is a dense contraction on the matrix cores
MFMA_FAMILIES = {"syrk_mfma", "trsm"}


# sources that define each kernel family (HBM counters taken on other
# versions of them are stale)
FAMILY_SOURCES = {
    "factor": ("factor.hip",),
    "solve": ("solve.hip",),
    "refine": ("refine.hip",),
}
FACTOR_FAMILIES = {"front_small", "assemble", "potrf", "trsm", "syrk_mfma"}
REFINE_FAMILIES = {"spmv_residual", "refine_vector"}


def source_digest(kind):
    """sha256 of the library sources that define kernel family `kind`."""
    import hashlib
    group = ("factor" if kind in FACTOR_FAMILIES else
             "refine" if kind in REFINE_FAMILIES else "solve")
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2110_12865_amd", "csrc")
    for f in FAMILY_SOURCES[group]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(workload, kind):
    """HBM bytes per launch of `kind` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a copy kernel of known
    size), or None when there is none for this workload and kernel or the
    sources of that kernel family changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    e = t.get(workload, {})
    if e.get("kernel") != kind or e.get("source_sha256") != source_digest(kind):
        return None
    return e.get("bytes_per_launch")


def roofline(prof, dtype, workload):
    """Roofline line of the dominant kernel family (most time per step):
    achieved = algorithmic work per launch / mean launch time (HIP events on
    the stream each launch runs on).  HBM-bound families use the survey's
    algorithmic bytes; MFMA families their flops at the dtype's peak."""
    cand = {k: v for k, v in prof.items() if k in HIP_KERNEL}
    name, st = max(cand.items(), key=lambda kv: kv[1]["ms"])
    nl = st["launches"]
    avg_ms = st["ms"] / nl
    if name in MFMA_FAMILIES:
        ach = st["flops"] / nl / (avg_ms * 1e-3) / 1e12
        roof = {"kernel": name, "bound": "mfma", "achieved": ach,
                "peak": PEAK_MFMA_TFLOPS[dtype], "unit": "TFLOP/s"}
    else:
        ach = st["alg_bytes"] / nl / (avg_ms * 1e-3) / 1e9
        roof = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(workload, name)
    roof["hip_kernel"] = HIP_KERNEL[name]
    roof["avg_launch_ms"] = avg_ms
    roof["launches"] = nl
    roof["algorithmic_bytes_per_launch"] = st["alg_bytes"] / nl
    roof["algorithmic_flops_per_launch"] = st["flops"] / nl
    roof["model_bytes_per_launch"] = st["bytes"] / nl
    return roof


def floor_clause_host(pat, values, x, b, tol=TOL):
    """Which clause of the stop rule holds, re-evaluated on the host with
    scipy for every (set, right-hand side): 1 relres <= tol, 2 ||r||_2 <=
    2 u ||A||_inf ||x||_2, 0 neither.  values [batch, nnz], x and b
    [batch, nrhs, n]."""
    import scipy.sparse as sp
    n = pat.n
    u = 2.0 ** -53
    out = np.zeros(x.shape[:2], np.int32)
    for s in range(x.shape[0]):
        A = sp.csc_matrix((values[s], pat.rowind, pat.colptr), shape=(n, n))
        A = (A + sp.tril(A, -1).T).tocsr()
        anorm = float(np.abs(A).sum(axis=1).max())
        for r in range(x.shape[1]):
            rn = np.linalg.norm(b[s, r] - A @ x[s, r])
            if rn <= tol * np.linalg.norm(b[s, r]):
                out[s, r] = 1
            elif rn <= 2.0 * u * anorm * np.linalg.norm(x[s, r]):
                out[s, r] = 2
    return out


def run_form(S, plan, w, dtype, steps, warmup, profile, assemble=None):
    """Time `steps` steps of one form: factor of the whole batch plus the
    refined solve to the stop rule, replayed as one captured HIP graph whose
    refinement budget is the step count an eager run needed (systems that
    have met the rule are skipped on the device).  With `assemble` (a
    callable writing the values tensor it is given on the device), every
    step first assembles the values, then replays the graph, which reads
    them.  Returns (seconds, per-system stats of the last replay, x,
    per-kernel profile of one eager step, refinement steps)."""
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
    if assemble is not None:
        vals.fill_(float("nan"))   # the steps must see assembled values only

    def step():
        if assemble is not None:
            assemble(vals)
        g.launch()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if assemble is not None and not np.array_equal(vals.cpu().numpy(), w.values):
        raise SystemExit("assembled values differ from the generator's")
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


def prepare(name):
    """(workload, name, form, group members or None); a group is merged into
    one block-diagonal workload."""
    import workloads as W
    w, wname, form = make_workload(name)
    members = None
    if isinstance(w, list):
        members = w
        vals, b = W.group_arrays(members)
        w = W.Workload(wname, None, None, vals, b, members[0].seed)
    return w, wname, form, members


def run_workload(name, args, headline):
    """Analyze (once, untimed), then time args.steps steps of the workload's
    form after args.warmup untimed ones.  Returns the result dict; the
    headline also carries the per-kernel table and the CPU baseline."""
    import paper_2110_12865_amd as S
    w, wname, form, members = prepare(name)
    if members is not None:
        nnz = sum(m.pattern.nnz for m in members)
        n = sum(m.pattern.n for m in members)
    else:
        n, nnz = w.pattern.n, w.pattern.nnz
    p = w.pattern
    log("workload %s n=%d nnzA=%d batch=%d nrhs=%d" % (wname, n, nnz, w.batch, w.nrhs))
    opts = {} if args.soa_min_batch is None else {"soa_min_batch": args.soa_min_batch}
    # options given for the workload named by --workload: no tuning
    fixed = args.options is not None and headline
    if fixed:
        opts.update(args.options)
    tuned = None
    if fixed:
        tuned = {"options": dict(opts), "seconds": 0.0, "candidates": [], "given": True}
    if members is not None and not args.no_tune and args.soa_min_batch is None and not fixed:
        # the uneven batch: the group autotuner on the group plan
        import torch
        tt = time.perf_counter()
        tv = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
        tb = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
        best, table = S.autotune_group([(m.pattern.colptr, m.pattern.rowind, m.perm)
                                        for m in members], tv, tb, "f32",
                                       solves_per_factor=2.0)
        del tv, tb
        torch.cuda.empty_cache()
        opts = {k: best[k] for k in ("small_front", "relax_cols", "soa_min_batch")}
        tuned = {"options": opts, "seconds": time.perf_counter() - tt,
                 "candidates": [{k: round(r[k], 4) if isinstance(r[k], float) else r[k]
                                 for k in ("small_front", "relax_cols", "soa_min_batch",
                                           "factor_ms", "solve_ms", "score")} for r in table]}
        log("group autotune %.1f s: %s" % (tuned["seconds"], opts))
    if headline and members is None and not args.no_tune and args.soa_min_batch is None and not fixed:
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
    x_gpu = None
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
        # the stop rule re-evaluated on the host (scipy), every system
        if members is None:
            hc = {f: floor_clause_host(p, w.values, xf, w.b) for f, xf in (("f32", x32),
                                                                             ("f64", x64))}
            rr = max(relres_host(p, w.values[s], x32[s, r], w.b[s, r])
                     for s in (0, w.batch - 1) for r in range(w.nrhs))
            x_gpu = {"f32_refined": x32, "f64": x64}
        else:
            col0, val0 = plan.export_blocks()
            hc = {}
            for f, xf in (("f32", x32), ("f64", x64)):
                hc[f] = np.concatenate([floor_clause_host(
                    m.pattern, w.values[:, val0[k]:val0[k + 1]], xf[:, :, col0[k]:col0[k + 1]],
                    w.b[:, :, col0[k]:col0[k + 1]]).ravel() for k, m in enumerate(members)])
            rr = max(relres_host(m.pattern, w.values[s, val0[k]:val0[k + 1]],
                                 x32[s, r, col0[k]:col0[k + 1]], w.b[s, r, col0[k]:col0[k + 1]])
                     for k, m in enumerate(members) for s in (0, w.batch - 1)
                     for r in range(w.nrhs))
        if members is None and headline and "mesh" in (w.extra or {}):
            out["assembled_step"] = assembled_step(S, plan, w, args)
        out["stop_rule_host"] = {f: {"clause_counts": {str(c): int(np.sum(v == c))
                                                       for c in (1, 2, 0)},
                                     "all_met": bool(np.all(v > 0))} for f, v in hc.items()}
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
        kern, total_alg = kernel_table(prof, 1)  # one eager profiled step
        if headline:
            out["kernels"] = kern
        else:
            top = sorted(kern.items(), key=lambda kv: -kv[1]["ms_per_step"])[:4]
            out["kernels_top"] = {k: round(v["ms_per_step"], 4) for k, v in top}
        out["alg_hbm_gb_s_step"] = total_alg / (ms * 1e-3) / 1e9
        out["roofline"] = roofline(prof, pdtype, wname)
    if headline and not args.no_cpu:
        log("cpu baseline (oracle on a bounded sample)...")
        if members is not None:
            out["cpu_baseline"] = cpu_baseline_group(members)
        else:
            cb = cpu_baseline(w, info["flops"], info["nnzL"], x_gpu=x_gpu)
            if "vs_oracle" in cb:
                out["vs_oracle"] = cb.pop("vs_oracle")
            out["cpu_baseline"] = cb
    del plan
    return out


def assembled_step(S, plan, w, args):
    """The mesh step with the values assembled on the device from the
    geometry (cotangent weights, per-set scales, mass) right before the
    captured factor + refined solve of every step, and the assembly alone
    (HIP events over args.steps launches)."""
    import torch
    from paper_2110_12865_amd.mesh import CotanAssembly
    p = w.pattern
    m = w.extra["mesh"]
    A = CotanAssembly(p.n, p.colptr, p.rowind, m["tris"])
    pos = torch.from_numpy(np.ascontiguousarray(m["pos"])).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(m["mass"])).cuda()
    scale = torch.from_numpy(np.ascontiguousarray(m["edge_scale"])).cuda()

    def assemble(vals):
        A.assemble(pos, mass, vals, edge_scale=scale, mass_coeff=m["mass_coeff"], clip=m["clip"])

    vals = torch.empty((w.batch, p.nnz), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        assemble(vals)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        assemble(vals)
    e1.record()
    torch.cuda.synchronize()
    asm_ms = e0.elapsed_time(e1) / args.steps
    bit_exact = bool(np.array_equal(vals.cpu().numpy(), w.values))
    del vals
    t, stats, _, _, iters = run_form(S, plan, w, "f32", args.steps, args.warmup, False,
                                     assemble=assemble)
    ms = t * 1e3 / args.steps
    nedge = A.nedge
    # algorithmic bytes per set: per-edge scale read and value written, per
    # vertex diagonal written and mass read (positions are shared)
    abytes = w.batch * (16.0 * nedge + 8.0 * p.n) + 8.0 * p.n + 16.0 * p.n
    return {"value": w.batch / (t / args.steps), "unit": "assemble+factor+solve/s",
            "ms_per_step": ms, "assembly_ms": asm_ms,
            "assembly_alg_gb_s": abytes / (asm_ms * 1e-3) / 1e9,
            "values_bit_exact_vs_generator": bit_exact, "refinement_budget": iters,
            "all_met": all(s["clause"] > 0 for s in stats)}


def sparse_products(args):
    """The paper's structured sparse products (Table tab:Lpow): A^2, A^3,
    A^4 of a 50k-vertex mesh Laplacian and L M L^T + K at 500k, FP32 as in
    the paper, each timed over args.steps launches with HIP events."""
    import scipy.sparse as sp
    import torch
    import workloads as W
    from paper_2110_12865_amd.products import lmlt_plus_k, power_chain

    def laplacian(k, seed):
        w = W.trimesh_workload(k, batch=1, nrhs=1, seed=seed)
        p = w.pattern
        A = sp.csc_matrix((w.values[0], p.rowind, p.colptr), shape=(p.n, p.n))
        A = (A + sp.tril(A, -1).T).tocsr()
        A.sort_indices()
        return A, w.extra["mesh"]["mass"]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    f32 = torch.float32
    out = {"dtype": "f32", "paper_vega20_ms": {"A^2": 0.17, "A^3": 0.49, "A^4": 0.98,
                                                "LMLT+K": 3.89}}
    A, _ = laplacian(224, 93)
    n = A.shape[0]
    plans = power_chain(n, (A.indptr.astype(np.int64), A.indices.astype(np.int32)), 4)
    a = torch.from_numpy(A.data[None].astype(np.float32)).cuda()
    bufs = [torch.empty((1, pr.nnz), dtype=f32, device="cuda") for pr in plans]
    chain_ms = 0.0
    for k, pr in enumerate(plans, start=2):
        src = a if k == 2 else bufs[k - 3]
        ms = timed(lambda: pr.run(src, a, bufs[k - 2]))
        chain_ms += ms
        # algorithmic bytes: both operands read and the result written once
        # (4 B per value), plus the 8 B position pair of every term
        alg = 4.0 * (src.shape[1] + a.shape[1] + pr.nnz)
        out["A^%d" % k] = {"ms_product": ms, "ms_chain": chain_ms, "n": n, "nnz": pr.nnz,
                           "terms": pr.nterms, "alg_gb_s": alg / (ms * 1e-3) / 1e9,
                           "with_tables_gb_s": (alg + 8.0 * pr.nterms) / (ms * 1e-3) / 1e9}
    L, mass = laplacian(708, 94)
    n = L.shape[0]
    rng = np.random.default_rng(95)
    kr, kc = [0], []
    for _ in range(n):
        kc.extend(np.sort(rng.choice(n, 6, replace=False)).tolist())
        kr.append(len(kc))
    K = (np.array(kr, np.int64), np.array(kc, np.int32))
    t, r = lmlt_plus_k(n, (L.indptr.astype(np.int64), L.indices.astype(np.int32)), K)
    lv = torch.from_numpy(L.data[None].astype(np.float32)).cuda()
    mv = torch.from_numpy(mass[None].astype(np.float32)).cuda()
    kv = torch.from_numpy(rng.uniform(-1, 1, (1, K[1].size)).astype(np.float32)).cuda()
    T = torch.empty((1, t.nnz), dtype=f32, device="cuda")
    R = torch.empty((1, r.nnz), dtype=f32, device="cuda")

    def lmlt():
        t.run(lv, mv, T)
        r.run(T, lv, R, kv)

    ms = timed(lmlt)
    alg = 4.0 * (2 * lv.shape[1] + n + t.nnz + kv.shape[1] + r.nnz)
    out["LMLT+K"] = {"ms": ms, "n": n, "nnz": r.nnz, "terms": t.nterms + r.nterms,
                     "alg_gb_s": alg / (ms * 1e-3) / 1e9,
                     "with_tables_gb_s": (alg + 8.0 * (t.nterms + r.nterms)) / (ms * 1e-3) / 1e9}
    return out


# the other configurations, timed in the same run after the headline
EXTRAS = ("grid2d32", "grid3d64", "uneven8", "blockvec40")


def compact(r):
    keys = ("value", "unit", "ms_per_step", "dtype", "speedup_vs_fp64_form", "fp64_form",
            "refinement", "relres", "relres_check_host", "stop_rule_host",
            "gradient_check_max_rel", "roofline", "kernels_top", "config")
    out = {k: r[k] for k in keys if k in r}
    if "fp64_form" in out:
        out["fp64_form"] = {k: out["fp64_form"][k] for k in ("value", "ms_per_step")}
    if "refinement" in out:
        out["refinement"] = {k: out["refinement"][k] for k in ("method", "budget", "iters_max")}
    return out


def _parse_options(text):
    out = {}
    for item in text.split(","):
        k, v = item.split("=")
        k = k.strip()
        if k not in ("small_front", "relax_cols", "soa_min_batch", "soa_seg_max", "relax"):
            raise argparse.ArgumentTypeError("unknown option %r" % k)
        out[k] = int(v)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="trimesh512")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only --workload, not the other configurations")
    ap.add_argument("--no-profile", action="store_true", help="no per-launch events")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only copy this many MiB device to device once (calibration of "
                         "the HBM byte counters) and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default options instead of the autotuner's choice")
    ap.add_argument("--options", type=_parse_options, default=None,
                    help="fixed plan options instead of the autotuner's choice, e.g. "
                         "small_front=128,relax_cols=16,soa_min_batch=1 (the autotuner's "
                         "choice on the default workload; used by the profiling commands so "
                         "that a profile holds no tuning candidates)")
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

    out = run_workload(args.workload, args, headline=True)
    if not args.no_extras and args.workload == "trimesh512":
        import torch
        other = {}
        for name in EXTRAS:
            torch.cuda.empty_cache()
            other[name] = compact(run_workload(name, args, headline=False))
        out["other_workloads"] = other
        torch.cuda.empty_cache()
        out["sparse_products"] = sparse_products(args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
