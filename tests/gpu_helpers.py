"""Shared helpers of the GPU tests: run a workload through the library (C
ABI via the Python binding) and through the oracle, and compare."""
import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_library(w, dtype="f64", values=None, b=None, plan=None, opts=None):
    import torch
    import paper_2110_12865_amd as S
    p = w.pattern
    if plan is None:
        plan = S.analyze(p.colptr, p.rowind, w.perm, **(opts or {}))
    vals = w.values if values is None else values
    rhs = w.b if b is None else b
    batch = vals.shape[0]
    num = plan.numeric(batch, dtype)
    dv = torch.from_numpy(np.ascontiguousarray(vals)).cuda()
    num.factor(dv)
    info = num.info()
    db = torch.from_numpy(np.ascontiguousarray(rhs)).cuda()
    num.solve(db)
    x = db.cpu().numpy()
    torch.cuda.synchronize()
    return plan, num, info, x


def oracle_run(w, s=0, nrows=None):
    p = w.pattern
    sym = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm, nrows=nrows)
    Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[s], sym)
    x = oracle.solve(sym, Lx, w.b[s]) if info == 0 and nrows is None else None
    return sym, Lx, info, x


def all_columns(n):
    return np.arange(n, dtype=np.int32)
