"""sc_solve_noalloc: the solve with its vectors in the library's static
scratch array (no device allocation) against sc_solve on the same numeric
object, through the C ABI.  The kernels are the same, so the solutions
must be equal bit for bit; two calls in a row, the second on a smaller
input, so the second runs on the first one's leftovers in the array."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_helpers import log, oracle_run

pytestmark = pytest.mark.gpu


def _solve_both(w, dtype, **opts):
    import paper_2110_12865_amd as S
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm, **opts)
    num = plan.numeric(w.batch, dtype)
    num.factor(torch.from_numpy(np.ascontiguousarray(w.values)).cuda())
    assert np.all(num.info() == 0)
    b = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    x_ref = num.solve(b.clone())
    x_na = num.solve_noalloc(b.clone())
    torch.cuda.synchronize()
    return x_ref.cpu().numpy(), x_na.cpu().numpy()


def test_noalloc_equals_solve_two_calls():
    # first call: 64 matrices in the batch-interleaved layout, 3 right-hand
    # sides, FP32 factor; second call: a smaller single FP64 system
    cases = [
        ("grid 20x20 nd, batch 64, 3 rhs, f32 (interleaved)",
         W.small_grid((20, 20), "nd", batch=64, nrhs=3, seed=71), "f32", {}),
        ("grid 6x6x6 nd, batch 1, 1 rhs, f64",
         W.small_grid((6, 6, 6), "nd", batch=1, nrhs=1, seed=72), "f64", {}),
    ]
    for name, w, dtype, opts in cases:
        log("no-alloc solve: %s (n=%d)" % (name, w.pattern.n))
        x_ref, x_na = _solve_both(w, dtype, **opts)
        assert np.array_equal(x_ref, x_na), name
        if dtype == "f64":
            _, _, info, xo = oracle_run(w, 0)
            assert info == 0
            assert oracle.forward_error(x_na[0, 0], xo[0]) <= 1e-12


def test_noalloc_row_major_batch_after_larger_call():
    # a row-major batch (below the interleaving threshold) with panel-solved
    # top fronts, after the larger interleaved call of the test above
    w = W.small_grid((12, 12, 12), "nd", batch=4, nrhs=2, seed=73)
    log("no-alloc solve: grid 12^3 nd, batch 4, 2 rhs, f64 (n=%d)" % w.pattern.n)
    x_ref, x_na = _solve_both(w, "f64")
    assert np.array_equal(x_ref, x_na)


def test_noalloc_rejects_workspace_beyond_scratch():
    import paper_2110_12865_amd as S
    w = W.small_grid((128, 128), "nd", batch=64, nrhs=3, seed=74)
    p = w.pattern
    plan = S.analyze(p.colptr, p.rowind, w.perm)
    num = plan.numeric(w.batch, "f32")
    num.factor(torch.from_numpy(np.ascontiguousarray(w.values)).cuda())
    b = torch.from_numpy(np.ascontiguousarray(w.b)).cuda()
    b0 = b.clone()
    with pytest.raises(S.SpcholError) as ei:
        num.solve_noalloc(b)
    assert ei.value.status == S.SC_ESCRATCH
    torch.cuda.synchronize()
    assert torch.equal(b, b0)  # nothing was launched
