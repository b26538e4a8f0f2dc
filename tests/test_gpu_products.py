"""Sparse products on fixed patterns (sc_spprod_*) against the oracle
(scipy's FP64 sparse product): every entry within the componentwise error
bound of a sum of t products, |C - C_o| <= gamma_{t+1} (|A||B| + |D|),
gamma_k = k u / (1 - k u) with u the unit roundoff of the arithmetic (FP64
or FP32; the FP32 inputs are the FP64 values rounded, whose own error is
covered by one more u per product), and the paper's chains at their sizes:
A^2, A^3, A^4 of a 50k-vertex mesh Laplacian and L M L^T + K at 500k."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _csr_random(rng, rows, cols, per_row):
    rp, ci = [0], []
    for _ in range(rows):
        ci.extend(np.sort(rng.choice(cols, size=min(per_row, cols), replace=False)).tolist())
        rp.append(len(ci))
    rp, ci = np.array(rp, np.int64), np.array(ci, np.int32)
    return rp, ci, rng.uniform(-1, 1, size=ci.size)


def _check(C_gpu, m, n, A, B, transB, D, dtype):
    """Compare with the oracle within the componentwise bound."""
    import scipy.sparse as sp
    ref = oracle.sparse_product(m, n, A, B, transB, D)
    absA = (A[0], A[1], np.abs(A[2]))
    absB = (B[0], B[1], np.abs(B[2]))
    absD = None if D is None else (D[0], D[1], np.abs(D[2]))
    bnd = oracle.sparse_product(m, n, absA, absB, transB, absD)
    # terms per entry: the product of the patterns with unit values
    ones = lambda M: (M[0], M[1], np.ones(M[1].size))
    cnt = oracle.sparse_product(m, n, ones(A), ones(B), transB, None)
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    return ref, bnd, cnt, u


def _compare(pr, Cg, ref, bnd, cnt, u, extra_u=0):
    import scipy.sparse as sp
    Cg_m = sp.csr_matrix((Cg, pr.colind, pr.rowptr), shape=ref.shape)
    diff = abs(Cg_m - ref)
    t = cnt.copy()
    t.data = (t.data + 1 + extra_u)
    gam = t.copy()
    gam.data = t.data * u / (1 - t.data * u)
    lim = bnd.multiply(gam)
    ok = diff - lim
    ok.eliminate_zeros()
    return float(ok.max()) if ok.nnz else -1.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("transB,with_d", [(False, False), (True, False), (True, True)])
def test_random_products_against_oracle(dtype, transB, with_d):
    from paper_2110_12865_amd.products import SparseProduct
    rng = np.random.default_rng(300 + 2 * transB + with_d)
    m, p, n = 700, 513, 650
    A = _csr_random(rng, m, p, 6)
    B = _csr_random(rng, n, p, 6) if transB else _csr_random(rng, p, n, 6)
    D = _csr_random(rng, m, n, 6) if with_d else None
    log("product %dx%dx%d transB=%d D=%d %s" % (m, p, n, transB, with_d, dtype))
    pr = SparseProduct(m, p, n, A[:2], B[:2], transB, None if D is None else D[:2])
    tdt = torch.float64 if dtype == "f64" else torch.float32
    batch = 3
    vals = lambda M: np.stack([M[2] * (1 + 0.1 * s) for s in range(batch)])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", tdt)
    Ca = torch.empty((batch, pr.nnz), dtype=tdt, device="cuda")
    pr.run(dev(vals(A)), dev(vals(B)), Ca, None if D is None else dev(vals(D)))
    Cg = Ca.double().cpu().numpy()
    for s in range(batch):
        As = (A[0], A[1], vals(A)[s].astype(np.float32).astype(np.float64)
              if dtype == "f32" else vals(A)[s])
        Bs = (B[0], B[1], vals(B)[s].astype(np.float32).astype(np.float64)
              if dtype == "f32" else vals(B)[s])
        Ds = None if D is None else (D[0], D[1], vals(D)[s].astype(np.float32).astype(np.float64)
                                     if dtype == "f32" else vals(D)[s])
        ref, bnd, cnt, u = _check(None, m, n, As, Bs, transB, Ds, dtype)
        assert _compare(pr, Cg[s], ref, bnd, cnt, u) <= 0.0


def _mesh_laplacian(k, seed):
    """Symmetric CSR of the cotangent stiffness (+ 1e-3 mass) of a jittered
    k x k mesh, and its lumped mass vector."""
    import scipy.sparse as sp
    w = W.trimesh_workload(k, batch=1, nrhs=1, seed=seed)
    p = w.pattern
    A = sp.csc_matrix((w.values[0], p.rowind, p.colptr), shape=(p.n, p.n))
    A = (A + sp.tril(A, -1).T).tocsr()
    A.sort_indices()
    return A, w.extra["mesh"]["mass"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_laplacian_powers_50k(dtype):
    """A^2, A^3, A^4 of a 224 x 224 mesh Laplacian (n = 50176), the chain
    evaluated on the device (each power stored and read by the next
    product) against the oracle's chain: normwise per entry, |C - C_o| <=
    4 k u max|C_o| for the k-th power (FP64), 1e-5 max|C_o| (FP32)."""
    from paper_2110_12865_amd.products import power_chain
    A, _ = _mesh_laplacian(224, 93)
    n = A.shape[0]
    log("powers of a mesh Laplacian n=%d nnz=%d %s" % (n, A.nnz, dtype))
    plans = power_chain(n, (A.indptr.astype(np.int64), A.indices.astype(np.int32)), 4)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    cur = torch.from_numpy(A.data[None].copy()).to("cuda", tdt)
    a_dev = cur
    refA = (A.indptr, A.indices, A.data.astype(np.float32).astype(np.float64)
            if dtype == "f32" else A.data)
    ref = refA
    for k, pr in enumerate(plans, start=2):
        out = torch.empty((1, pr.nnz), dtype=tdt, device="cuda")
        pr.run(cur, a_dev, out)
        cur = out
        R = oracle.sparse_product(n, n, ref, refA)
        ref = (R.indptr, R.indices, R.data)
        assert np.array_equal(pr.rowptr, R.indptr) or pr.nnz >= R.nnz
        import scipy.sparse as sp
        G = sp.csr_matrix((out.double().cpu().numpy()[0], pr.colind, pr.rowptr), shape=(n, n))
        err = abs(G - R).max()
        scale = abs(R).max()
        tol = 4 * k * 2.0 ** -53 if dtype == "f64" else 1e-5
        log("  A^%d: nnz %d terms %d, max err %.2e (max |C| %.2e)"
            % (k, pr.nnz, pr.nterms, err, scale))
        assert err <= tol * scale


def test_lmlt_plus_k_500k():
    """L M L^T + K with L the Laplacian of a 708 x 708 mesh (n = 501264), M
    its lumped mass (diagonal) and K six random entries per row, FP64:
    against the oracle's product, per entry within 1e-14 max|C|."""
    import scipy.sparse as sp
    from paper_2110_12865_amd.products import lmlt_plus_k
    L, mass = _mesh_laplacian(708, 94)
    n = L.shape[0]
    rng = np.random.default_rng(95)
    K = _csr_random(rng, n, n, 6)
    log("L M L^T + K n=%d nnz(L)=%d" % (n, L.nnz))
    Lp = (L.indptr.astype(np.int64), L.indices.astype(np.int32))
    t, r = lmlt_plus_k(n, Lp, K[:2])
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)[None]).cuda()
    T = torch.empty((1, t.nnz), dtype=torch.float64, device="cuda")
    t.run(dv(L.data), dv(mass), T)
    R = torch.empty((1, r.nnz), dtype=torch.float64, device="cuda")
    r.run(T, dv(L.data), R, dv(K[2]))
    diag = (np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), mass)
    To = oracle.sparse_product(n, n, (L.indptr, L.indices, L.data), diag)
    Ro = oracle.sparse_product(n, n, (To.indptr, To.indices, To.data),
                               (L.indptr, L.indices, L.data), True, K)
    G = sp.csr_matrix((R.cpu().numpy()[0], r.colind, r.rowptr), shape=(n, n))
    err = abs(G - Ro).max()
    log("  nnz %d terms %d, max err %.2e (max |C| %.2e)" % (r.nnz, r.nterms, err, abs(Ro).max()))
    assert err <= 1e-14 * abs(Ro).max()
