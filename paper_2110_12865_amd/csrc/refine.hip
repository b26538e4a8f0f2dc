// Iterative refinement on the GPU: the factor (FP32 or FP64) gives the
// corrections, the residual b - A x, the norms, the stop test and the update
// x += d run in FP64.
//
//   x_0 = solve(b)
//   loop: r = b - A x;  stop when ||r||_2 <= tol ||b||_2
//                       or ||r||_2 <= 2 u ||A||_inf ||x||_2  (FP64 floor)
//         d = solve(r);  x += d
//
// Every system (matrix of the batch, right-hand side) is tested on its own;
// a matrix stops taking corrections once all its right-hand sides pass.
// The residual uses both triangles of A by rows (one lane per row, entries
// in a fixed order) and all reductions use a fixed tree, so results are
// bit-reproducible.
#include <cfloat>

#include "device.hpp"

namespace {

// r = b - A x for every (matrix, rhs) with active[matrix] != 0
__global__ __launch_bounds__(256) void k_resid(
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
    const int64_t *__restrict__ vidx, const double *__restrict__ vals, int64_t ldv,
    const double *__restrict__ B, const double *__restrict__ X, double *__restrict__ R,
    int64_t ldb, int64_t n, int nrhs, const int32_t *__restrict__ active) {
    const int br = blockIdx.y;
    const int b = br / nrhs;
    if (active && !active[b]) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *v = vals + int64_t(b) * ldv;
    const double *x = X + int64_t(br) * ldb;
    double t = 0.0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; e++) t += v[vidx[e]] * x[col[e]];
    R[int64_t(br) * ldb + i] = B[int64_t(br) * ldb + i] - t;
}

// ||A||_inf of every matrix: max over rows of sum |A_ij|
__global__ __launch_bounds__(256) void k_anorm(
    const int64_t *__restrict__ ptr, const int64_t *__restrict__ vidx,
    const double *__restrict__ vals, int64_t ldv, int64_t n, double *__restrict__ anorm) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    const double *v = vals + int64_t(b) * ldv;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double s = 0.0;
        for (int64_t e = ptr[i]; e < ptr[i + 1]; e++) s += fabs(v[vidx[e]]);
        m = fmax(m, s);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) anorm[b] = red[0];
}

// Stop test for every system: sums of squares of r, b, x by a fixed tree,
// then the two clauses.  stat layout per system: [iters, clause, relres,
// rnorm, bnorm, xnorm].  conv[br] = 1 once the system passes.
__global__ __launch_bounds__(256) void k_check(
    const double *__restrict__ R, const double *__restrict__ B,
    const double *__restrict__ X, int64_t ldb, int64_t n, int nrhs,
    const double *__restrict__ anorm, double tol, int iter,
    const int32_t *__restrict__ active, int32_t *__restrict__ conv,
    double *__restrict__ stat) {
    __shared__ double sr[256], sb[256], sx[256];
    const int br = blockIdx.x;
    const int b = br / nrhs;
    if (active && !active[b]) return;
    const double *r = R + int64_t(br) * ldb;
    const double *bb = B + int64_t(br) * ldb;
    const double *x = X + int64_t(br) * ldb;
    double a = 0.0, c = 0.0, d = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        a += r[i] * r[i];
        c += bb[i] * bb[i];
        d += x[i] * x[i];
    }
    sr[threadIdx.x] = a;
    sb[threadIdx.x] = c;
    sx[threadIdx.x] = d;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
            sx[threadIdx.x] += sx[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double rn = sqrt(sr[0]), bn = sqrt(sb[0]), xn = sqrt(sx[0]);
        const double relres = bn > 0.0 ? rn / bn : rn;
        int clause = 0;
        if (relres <= tol) clause = 1;
        else if (rn <= 2.0 * DBL_EPSILON * 0.5 * anorm[b] * xn) clause = 2;
        double *st = stat + int64_t(br) * 6;
        st[0] = iter;
        st[1] = clause;
        st[2] = relres;
        st[3] = rn;
        st[4] = bn;
        st[5] = xn;
        conv[br] = clause != 0;
    }
}

// active[b] = some right-hand side of matrix b has not passed;
// count[0] = number of active matrices
__global__ void k_active(const int32_t *__restrict__ conv, int batch, int nrhs,
                         int32_t *__restrict__ active, int32_t *__restrict__ count) {
    __shared__ int32_t cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < batch; b += blockDim.x) {
        if (!active[b]) continue;
        int all = 1;
        for (int r = 0; r < nrhs; r++) all &= conv[b * nrhs + r];
        active[b] = !all;
        if (!all) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) count[0] = cnt;
}

__global__ void k_axpy(double *__restrict__ X, const double *__restrict__ D, int64_t ldb,
                       int64_t n, int nrhs, const int32_t *__restrict__ active) {
    const int br = blockIdx.y;
    if (active && !active[br / nrhs]) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) X[int64_t(br) * ldb + i] += D[int64_t(br) * ldb + i];
}

__global__ void k_set_i32(int32_t *p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t spchol_refine_run(const sc_plan *P, sc_numeric *N, const double *vals,
                             int64_t ldv, const double *b, double *x, int32_t nrhs,
                             int64_t ldb, double tol, int32_t maxit, double *stat_host,
                             int32_t *nactive_out, hipStream_t st) {
    DevPlan *D = P->dev;
    RefineWs &W = N->rws;
    const int batch = N->batch;
    const int nsys = batch * nrhs;
    const int64_t n = P->n;
    const dim3 vgrid(unsigned((n + 255) / 256), unsigned(nsys));
    hipError_t e;
    // x0 = solve(b)
    e = hipMemcpy2DAsync(x, ldb * sizeof(double), b, ldb * sizeof(double), n * sizeof(double),
                         nsys, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_set_i32, dim3((batch + 255) / 256), dim3(256), 0, st, W.active, batch,
                       int32_t(1));
    e = spchol_solve_run(P, N, x, nrhs, ldb, st, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_anorm, dim3(batch), dim3(256), 0, st, D->csr_ptr, D->csr_vidx, vals,
                       ldv, n, W.anorm);
    int32_t nact = batch;
    for (int it = 0;; it++) {
        hipLaunchKernelGGL(k_resid, vgrid, dim3(256), 0, st, D->csr_ptr, D->csr_col,
                           D->csr_vidx, vals, ldv, b, x, W.r, ldb, n, nrhs, W.active);
        hipLaunchKernelGGL(k_check, dim3(nsys), dim3(256), 0, st, W.r, b, x, ldb, n, nrhs,
                           W.anorm, tol, it, W.active, W.conv, W.stat);
        hipLaunchKernelGGL(k_active, dim3(1), dim3(256), 0, st, W.conv, batch, nrhs, W.active,
                           W.count);
        e = hipMemcpyAsync(&nact, W.count, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (nact == 0 || it >= maxit) break;
        e = spchol_solve_run(P, N, W.r, nrhs, ldb, st, W.active);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_axpy, vgrid, dim3(256), 0, st, x, W.r, ldb, n, nrhs, W.active);
    }
    *nactive_out = nact;
    e = hipMemcpyAsync(stat_host, W.stat, sizeof(double) * 6 * nsys, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}
