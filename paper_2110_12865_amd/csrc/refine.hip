// Iterative refinement on the GPU: the factor (FP32 or FP64) gives the
// corrections, the residual b - A x, the norms, the stop test and the update
// x += d run in FP64.
//
//   x_0 = solve(b)
//   loop: r = b - A x;  stop when ||r||_2 <= tol ||b||_2
//                       or ||r||_2 <= 2 u ||A||_inf ||x||_2  (FP64 floor)
//         d = solve(r);  x += d
//
// Every system (matrix of the batch, right-hand side, diagonal block) is
// tested on its own and takes no corrections once it passes; the blocks are
// the patterns of a group plan (one block otherwise), and a system's norms
// run over its block's rows only.  Vector kernels index systems as
// seg = (matrix * nrhs + rhs) * nblk + block.
// The residual uses both triangles of A by rows (one lane per row, entries
// in a fixed order) and all reductions use a fixed tree, so results are
// bit-reproducible.
#include <algorithm>
#include <cfloat>

#include "device.hpp"

namespace {

// The values of A in the order of its sliced row structure (both
// triangles), one copy per matrix: vc[b * nsell + e] = values[b][vidx[e]]
// (0 for padding).  Made once per refinement call so that every later
// product reads A contiguously.  A thread takes entry e of kGatherMats
// consecutive matrices, so the shared index is read once for all of them.
constexpr int kGatherMats = 8;
__global__ __launch_bounds__(256) void k_gather_rows(
    const int64_t *__restrict__ vidx, const double *__restrict__ vals, int64_t ldv,
    int64_t nsell, int batch, double *__restrict__ vc) {
    const int b0 = blockIdx.y * kGatherMats;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nsell) return;
    const int64_t v = vidx[e];
    const int nb = min(kGatherMats, batch - b0);
    double a[kGatherMats];
#pragma unroll
    for (int k = 0; k < kGatherMats; k++)
        a[k] = (v >= 0 && k < nb) ? vals[int64_t(b0 + k) * ldv + (v >= 0 ? v : 0)] : 0.0;
#pragma unroll
    for (int k = 0; k < kGatherMats; k++)
        if (k < nb) vc[int64_t(b0 + k) * nsell + e] = a[k];
}

// Sum of v over the 64 lanes of a wave, by a fixed butterfly; lane 0's
// result is the one used (other lanes may round differently).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The entries of one 64-row slice of the sliced row structure, read by the
// wave that owns the slice (lane = row): the slice's padded length (uniform
// over the wave) and the wave's base entry.  Waves past the last slice get
// length 0.
struct SliceRef {
    int64_t e0;  // entry of lane 0 in row position 0
    int len;     // padded entries per row
};
__device__ inline SliceRef slice_of(const int64_t *__restrict__ sptr, int64_t i, int64_t n) {
    const int64_t s = __builtin_amdgcn_readfirstlane(int(i / kSellRows));
    const int64_t nsl = (n + kSellRows - 1) / kSellRows;
    SliceRef r;
    r.e0 = s < nsl ? sptr[s] : 0;
    r.len = s < nsl ? int((sptr[s + 1] - r.e0) / kSellRows) : 0;
    return r;
}

// t[r] += sum_k a_k X[base + r ldb + j_k] over the entries of row i in
// order (k < len), each chunk of U entries loaded (values, columns, then the
// U * NR entries of X) before its sums; positions past the row's length but
// inside the slice are padding (column 0, value 0) and are loaded but not
// added.
template <int NR, int U>
__device__ inline void row_dot(const SliceRef &sl, int len, const double *__restrict__ v,
                               const int32_t *__restrict__ cl, const double *__restrict__ X,
                               int64_t base, int64_t ldb, double *t, double &asum) {
    for (int k0 = 0; k0 < sl.len; k0 += U) {
        double a[U], x[U][NR];
        int32_t j[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t k = min(k0 + u, sl.len - 1);
            a[u] = v[k * kSellRows];
            j[u] = cl[k * kSellRows];
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int r = 0; r < NR; r++) x[u][r] = X[base + r * ldb + j[u]];
#pragma unroll
        for (int u = 0; u < U; u++)
            if (k0 + u < len) {
#pragma unroll
                for (int r = 0; r < NR; r++) t[r] += a[u] * x[u][r];
                asum += fabs(a[u]);
            }
    }
}

// Maximum of v over the 64 lanes of a wave (any order gives the same value).
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Y = B - A X (mode 1) or Y = A X (mode 0) for every right-hand side of the
// matrices with active[matrix] != 0: one lane per row of A, entries in row
// order from the sliced layout (entry k of the 64 rows of a wave's slice is
// one contiguous load of values and of column indices), all NR right-hand
// sides of the matrix at once so every value of A is read once per matrix.
// Workgroups of consecutive matrices cover the same rows, so the shared row
// structure is reused from cache.  With psum (plans of one block), also the
// workgroup's partial sums per right-hand side, in mode 1 of Y.Y, B.B and
// X.X, in mode 0 of X.Y and B.X (B is then read for these sums only):
// psum[((matrix * nrhs + r) * nrb + block of rows) * 3 + {0, 1, 2}], lanes
// in a fixed butterfly, waves in order.  With amax (right-hand sides from
// r0 = 0), the workgroup's largest row sum of |A|: amax[matrix * nrb + block
// of rows], each row summed in entry order.
template <int NR>
__global__ __launch_bounds__(256) void k_apply(
    const int64_t *__restrict__ ptr, const int64_t *__restrict__ sptr,
    const int32_t *__restrict__ col, const double *__restrict__ vc, int64_t nsell,
    const double *__restrict__ B, const double *__restrict__ X, double *__restrict__ Y,
    int64_t ldb, int64_t n, int nrhs, int r0, int mode, const int32_t *__restrict__ active,
    double *__restrict__ psum, int nrb, double *__restrict__ amax) {
    __shared__ double red[4][NR][3];
    __shared__ double redm[4];
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const int64_t i = int64_t(blockIdx.y) * blockDim.x + threadIdx.x;
    const bool in = i < n;
    if (!in && !psum && !amax) return;
    const int64_t ic = in ? i : n - 1;  // rows past n compute row n - 1 and add nothing
    const SliceRef sl = slice_of(sptr, i, n);
    const int len = in ? int(ptr[i + 1] - ptr[i]) : 0;
    const int64_t e0 = sl.e0 + i % kSellRows;
    const int64_t base = (int64_t(b) * nrhs + r0) * ldb;
    double t[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) t[r] = 0.0;
    double asum = 0.0;
    row_dot<NR, 8>(sl, len, vc + int64_t(b) * nsell + e0, col + e0, X, base, ldb, t, asum);
    double y[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        y[r] = mode ? B[base + r * ldb + ic] - t[r] : t[r];
        if (in) Y[base + r * ldb + i] = y[r];
    }
    if (!psum && !amax) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (amax) {
        const double m = wave_max(asum);  // rows past n have asum = 0
        if (lane == 0) redm[wv] = m;
    }
    if (psum) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const double bb = B[base + r * ldb + ic], xx = X[base + r * ldb + ic];
            const double s0 = wave_sum(in ? (mode ? y[r] * y[r] : xx * y[r]) : 0.0);
            const double s1 = wave_sum(in ? (mode ? bb * bb : bb * xx) : 0.0);
            const double s2 = wave_sum(in && mode ? xx * xx : 0.0);
            if (lane == 0) {
                red[wv][r][0] = s0;
                red[wv][r][1] = s1;
                red[wv][r][2] = s2;
            }
        }
    }
    __syncthreads();
    if (psum && threadIdx.x < 3 * NR) {
        const int r = threadIdx.x / 3, q = threadIdx.x % 3;
        psum[((int64_t(b) * nrhs + r0 + r) * nrb + blockIdx.y) * 3 + q] =
            ((red[0][r][q] + red[1][r][q]) + red[2][r][q]) + red[3][r][q];
    }
    if (amax && threadIdx.x == 0)
        amax[int64_t(b) * nrb + blockIdx.y] = fmax(fmax(redm[0], redm[1]), fmax(redm[2], redm[3]));
}

// anorm[matrix] = the largest of the nrb row-block maxima of k_apply (one
// wave per matrix; the maximum does not depend on the order).
__global__ __launch_bounds__(256) void k_anorm_blocks(const double *__restrict__ amax, int nrb,
                                                      int batch, double *__restrict__ anorm) {
    const int b = blockIdx.x * 4 + int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (b >= batch) return;
    double m = 0.0;
    for (int q = lane; q < nrb; q += 64) m = fmax(m, amax[int64_t(b) * nrb + q]);
    m = wave_max(m);
    if (lane == 0) anorm[b] = m;
}

// Y1 = B - A X1 and Y2 = A X2 in one pass over A (each sum in the order
// k_apply uses), for the matrices with active[matrix] != 0.  With psum
// (plans of one block), also the workgroup's partial sums of Y1.Y1, X2.Y2
// and X1.X1 per right-hand side: psum[((matrix * nrhs + r) * nrb + block
// of rows) * 3 + {0, 1, 2}], lanes in a fixed butterfly, waves in order.
template <int NR>
__global__ __launch_bounds__(256) void k_apply2(
    const int64_t *__restrict__ ptr, const int64_t *__restrict__ sptr,
    const int32_t *__restrict__ col, const double *__restrict__ vc, int64_t nsell,
    const double *__restrict__ B, const double *__restrict__ X1, double *__restrict__ Y1,
    const double *__restrict__ X2, double *__restrict__ Y2, int64_t ldb, int64_t n, int nrhs,
    int r0, const int32_t *__restrict__ active, double *__restrict__ psum, int nrb) {
    __shared__ double red[4][NR][3];
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const int64_t i = int64_t(blockIdx.y) * blockDim.x + threadIdx.x;
    const bool in = i < n;
    const int64_t ic = in ? i : n - 1;  // rows past n compute row n - 1 and add nothing
    const SliceRef sl = slice_of(sptr, i, n);
    const int len = in ? int(ptr[i + 1] - ptr[i]) : 0;
    const int64_t e0 = sl.e0 + i % kSellRows;
    const int64_t base = (int64_t(b) * nrhs + r0) * ldb;
    double t1[NR], t2[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) t1[r] = t2[r] = 0.0;
    {
        const double *v = vc + int64_t(b) * nsell + e0;
        const int32_t *cl = col + e0;
        for (int k0 = 0; k0 < sl.len; k0 += 4) {
            double a[4], x1[4][NR], x2[4][NR];
            int32_t j[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int64_t k = min(k0 + u, sl.len - 1);
                a[u] = v[k * kSellRows];
                j[u] = cl[k * kSellRows];
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    x1[u][r] = X1[base + r * ldb + j[u]];
                    x2[u][r] = X2[base + r * ldb + j[u]];
                }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (k0 + u < len)
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        t1[r] += a[u] * x1[u][r];
                        t2[r] += a[u] * x2[u][r];
                    }
        }
    }
    double y1[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        y1[r] = B[base + r * ldb + ic] - t1[r];
        if (in) {
            Y1[base + r * ldb + i] = y1[r];
            Y2[base + r * ldb + i] = t2[r];
        }
    }
    if (!psum) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const double x1 = X1[base + r * ldb + ic], x2 = X2[base + r * ldb + ic];
        const double s0 = wave_sum(in ? y1[r] * y1[r] : 0.0);
        const double s1 = wave_sum(in ? x2 * t2[r] : 0.0);
        const double s2 = wave_sum(in ? x1 * x1 : 0.0);
        if (lane == 0) {
            red[wv][r][0] = s0;
            red[wv][r][1] = s1;
            red[wv][r][2] = s2;
        }
    }
    __syncthreads();
    if (threadIdx.x < 3 * NR) {
        const int r = threadIdx.x / 3, q = threadIdx.x % 3;
        psum[((int64_t(b) * nrhs + r0 + r) * nrb + blockIdx.y) * 3 + q] =
            ((red[0][r][q] + red[1][r][q]) + red[2][r][q]) + red[3][r][q];
    }
}

// Block of vector element i (colblk is null for a plan of one block).
__device__ inline int seg_of(int br, int nblk, const int32_t *colblk, int64_t i) {
    return br * nblk + (colblk ? colblk[i] : 0);
}

// ||A_k||_inf of every (matrix, block): max over the block's rows of
// sum |A_ij|, in 32 slices (partial maxima in part[bk * 32 + slice]), then
// the max of the slices (the maximum does not depend on the order).
__global__ __launch_bounds__(256) void k_anorm_part(
    const int64_t *__restrict__ ptr, const int64_t *__restrict__ sptr,
    const double *__restrict__ vc, int64_t nsell, const int64_t *__restrict__ col0, int nblk,
    double *__restrict__ part) {
    __shared__ double red[256];
    const int bk = blockIdx.y, slice = blockIdx.x;
    const int b = bk / nblk, k = bk - b * nblk;
    const int64_t r0 = col0[k], nr = col0[k + 1] - r0;
    const int64_t len = (nr + 31) / 32;
    const int64_t i0 = r0 + slice * len, i1 = min(r0 + nr, i0 + len);
    const double *v = vc + int64_t(b) * nsell;
    double m = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const int64_t e0 = sptr[i / kSellRows] + i % kSellRows;
        const int len = int(ptr[i + 1] - ptr[i]);
        double s = 0.0;
        for (int k = 0; k < len; k++) s += fabs(v[e0 + int64_t(k) * kSellRows]);
        m = fmax(m, s);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[int64_t(bk) * 32 + slice] = red[0];
}

__global__ void k_anorm_final(const double *__restrict__ part, int nbk,
                              double *__restrict__ anorm) {
    const int bk = blockIdx.x * blockDim.x + threadIdx.x;
    if (bk >= nbk) return;
    double m = 0.0;
    for (int q = 0; q < 32; q++) m = fmax(m, part[int64_t(bk) * 32 + q]);
    anorm[bk] = m;
}

// Per-system reductions in two stages: kRB workgroups per system each sum
// a contiguous slice of the system's rows (fixed tree), then one wave of the
// consumer adds the partials (lane l: partials l, l + 64, ... in order, then
// a fixed butterfly), so every result is bit-reproducible.
constexpr int kRB = 32;

__device__ inline double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// nq = 3: partial sums of r.r, b.b, x.x (A = r, B = b, C = x); nq = 4: r.r
// and x.x only (slots 0 and 2; b.b does not change between tests);
// nq = 2: partial sums of A.B and B.C; nq = 1: partial sum of A.B.
// part[(seg * kRB + slice) * 3 + q].
__global__ __launch_bounds__(256) void k_sums(
    const double *__restrict__ A, const double *__restrict__ Bv, const double *__restrict__ C,
    int nq, int64_t ldb, const int64_t *__restrict__ col0, int nblk, int nrhs,
    const int32_t *__restrict__ active, const int32_t *__restrict__ skip,
    double *__restrict__ part) {
    __shared__ double red[256];
    const int sg = blockIdx.y, slice = blockIdx.x;
    const int br = sg / nblk, k = sg - br * nblk;
    if (active && !active[br / nrhs]) return;
    if (skip && skip[sg]) return;
    const int64_t r0 = col0[k], nr = col0[k + 1] - r0;
    const int64_t len = (nr + kRB - 1) / kRB;
    const int64_t i0 = r0 + slice * len, i1 = min(r0 + nr, i0 + len);
    const double *a = A + int64_t(br) * ldb;
    const double *bb = nq == 4 ? A + int64_t(br) * ldb : Bv + int64_t(br) * ldb;
    const double *cc = nq >= 2 ? C + int64_t(br) * ldb : nullptr;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double ai = a[i];
        if (nq == 4) {
            const double ci = cc[i];
            s0 += ai * ai;
            s2 += ci * ci;
            continue;
        }
        const double bi = bb[i];
        if (nq == 3) {
            const double ci = cc[i];
            s0 += ai * ai;
            s1 += bi * bi;
            s2 += ci * ci;
        } else if (nq == 2) {
            s0 += ai * bi;
            s1 += bi * cc[i];
        } else {
            s0 += ai * bi;
        }
    }
    double *o = part + (int64_t(sg) * kRB + slice) * 3;
    const double t0 = block_sum(s0, red);
    if (nq == 4) {
        const double t2 = block_sum(s2, red);
        if (threadIdx.x == 0) { o[0] = t0; o[2] = t2; }
    } else if (nq == 3) {
        const double t1 = block_sum(s1, red);
        const double t2 = block_sum(s2, red);
        if (threadIdx.x == 0) { o[0] = t0; o[1] = t1; o[2] = t2; }
    } else if (nq == 2) {
        const double t1 = block_sum(s1, red);
        if (threadIdx.x == 0) { o[0] = t0; o[1] = t1; }
    } else if (threadIdx.x == 0) {
        o[0] = t0;
    }
}

// out[seg] = sum of the nsl partial sums of system seg in slice order
// (component comp), out2[seg] the same for component comp + 1 when given
__global__ __launch_bounds__(256) void k_sums_final(
    const double *__restrict__ part, int nsl, int comp, int nseg, int per_matrix,
    const int32_t *__restrict__ active, double *__restrict__ out, double *__restrict__ out2) {
    // one wave per system: lane l adds partials l, l + 64, ... in order and
    // the lanes' sums meet in a fixed butterfly
    const int sg = blockIdx.x * 4 + int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (sg >= nseg || !active[sg / per_matrix]) return;
    double t = 0.0, t2 = 0.0;
    for (int q = lane; q < nsl; q += 64) {
        t += part[(int64_t(sg) * nsl + q) * 3 + comp];
        if (out2) t2 += part[(int64_t(sg) * nsl + q) * 3 + comp + 1];
    }
    t = wave_sum(t);
    if (out2) t2 = wave_sum(t2);
    if (lane == 0) {
        out[sg] = t;
        if (out2) out2[sg] = t2;
    }
}

// Stop test for every system from the partial sums of r.r, b.b and x.x.
// stat layout per system: [iters, clause, relres, rnorm, bnorm, xnorm].
// conv[seg] = 1 once the system passes; a system that passed earlier (and
// is no longer updated) keeps its record.
// iter > 0 takes ||b||_2 from the record of the first test (part holds no
// b.b then).
__global__ __launch_bounds__(256) void k_check(
    const double *__restrict__ part, int nsl, int nseg, int nrhs, int nblk,
    const double *__restrict__ anorm, double tol, int iter, const int32_t *__restrict__ active,
    int32_t *__restrict__ conv, double *__restrict__ stat) {
    // one wave per system, partial sums added as in k_sums_final
    const int sg = blockIdx.x * 4 + int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (sg >= nseg) return;
    const int b = sg / (nrhs * nblk), k = sg % nblk;
    if (!active[b] || conv[sg]) return;
    double a = 0.0, c = 0.0, d = 0.0;
    for (int q = lane; q < nsl; q += 64) {
        const double *o = part + (int64_t(sg) * nsl + q) * 3;
        a += o[0];
        if (iter == 0) c += o[1];
        d += o[2];
    }
    a = wave_sum(a);
    c = wave_sum(c);
    d = wave_sum(d);
    if (lane != 0) return;
    const double rn = sqrt(a), xn = sqrt(d);
    const double bn = iter == 0 ? sqrt(c) : stat[int64_t(sg) * 6 + 4];
    const double relres = bn > 0.0 ? rn / bn : rn;
    int clause = 0;
    if (relres <= tol) clause = 1;
    else if (rn <= 2.0 * DBL_EPSILON * 0.5 * anorm[b * nblk + k] * xn) clause = 2;
    double *st = stat + int64_t(sg) * 6;
    st[0] = iter;
    st[1] = clause;
    st[2] = relres;
    st[3] = rn;
    st[4] = bn;
    st[5] = xn;
    conv[sg] = clause != 0;
}

// active[b] = some system of matrix b has not passed;
// count[0] = number of active matrices
__global__ void k_active(const int32_t *__restrict__ conv, int batch, int per_matrix,
                         int32_t *__restrict__ active, int32_t *__restrict__ count) {
    __shared__ int32_t cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < batch; b += blockDim.x) {
        if (!active[b]) continue;
        int all = 1;
        for (int q = 0; q < per_matrix; q++) all &= conv[b * per_matrix + q];
        active[b] = !all;
        if (!all) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) count[0] = cnt;
}

// The vector kernels below take several elements per thread (kVecPer, or
// PER; strided by the workgroup size, so every load is coalesced), with
// their loads issued before the per-system scalars are tested: a workgroup
// covers 256 * kVecPer consecutive elements of one system vector.
constexpr int kVecPer = 4;
constexpr int kVecSpan = 256 * kVecPer;

// x += d on the systems that have not passed
__global__ __launch_bounds__(256) void k_axpy(
    double *__restrict__ X, const double *__restrict__ D, int64_t ldb, int64_t n, int nrhs,
    int nblk, const int32_t *__restrict__ colblk, const int32_t *__restrict__ active,
    const int32_t *__restrict__ conv) {
    const int br = blockIdx.y;
    if (!active[br / nrhs]) return;
    const int64_t i0 = int64_t(blockIdx.x) * kVecSpan + threadIdx.x, o0 = int64_t(br) * ldb;
    double x[kVecPer], d[kVecPer];
#pragma unroll
    for (int q = 0; q < kVecPer; q++) {
        const int64_t i = i0 + 256 * q;
        x[q] = i < n ? X[o0 + i] : 0.0;
        d[q] = i < n ? D[o0 + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kVecPer; q++) {
        const int64_t i = i0 + 256 * q;
        if (i < n && !conv[seg_of(br, nblk, colblk, i)]) X[o0 + i] = x[q] + d[q];
    }
}

__global__ void k_set_i32(int32_t *p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// CG step on systems that have not passed: alpha = rz / pq,
// x += alpha p, r -= alpha q (a system with pq <= 0 is left unchanged; x
// only when R is null: the last step of a fixed budget, whose recursive
// residual nobody reads); PER elements per thread (four vectors in flight
// at PER = 1 already keep this kernel at the bandwidth of the others)
template <int PER>
__global__ __launch_bounds__(256) void k_cg_xr(
    double *__restrict__ X, double *__restrict__ R, const double *__restrict__ Pv,
    const double *__restrict__ Q, int64_t ldb, int64_t n, int nrhs, int nblk,
    const int32_t *__restrict__ colblk, const int32_t *__restrict__ active,
    const int32_t *__restrict__ conv, const double *__restrict__ rz,
    const double *__restrict__ pq) {
    const int br = blockIdx.y;
    if (!active[br / nrhs]) return;
    const int64_t i0 = int64_t(blockIdx.x) * (256 * PER) + threadIdx.x, o0 = int64_t(br) * ldb;
    double x[PER], r[PER], p[PER], q4[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t i = i0 + 256 * q;
        const bool on = i < n;
        x[q] = on ? X[o0 + i] : 0.0;
        p[q] = on ? Pv[o0 + i] : 0.0;
        r[q] = on && R ? R[o0 + i] : 0.0;
        q4[q] = on && R ? Q[o0 + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t i = i0 + 256 * q;
        if (i >= n) continue;
        const int sg = seg_of(br, nblk, colblk, i);
        const double den = pq[sg];
        if (conv[sg] || !(den > 0.0)) continue;
        const double alpha = rz[sg] / den;
        X[o0 + i] = x[q] + alpha * p[q];
        if (R) R[o0 + i] = r[q] - alpha * q4[q];
    }
}

// p = z + beta p with beta = z_new.(r_new - r_old) / (z_old.r_old), the form
// that tolerates a preconditioner applied in lower precision (Golub and Ye,
// inexact preconditioned CG).  With r_new - r_old = -alpha q and alpha =
// z_old.r_old / p.q this is beta = -z_new.q / p.q.
__global__ __launch_bounds__(256) void k_cg_p(
    double *__restrict__ Pv, const double *__restrict__ Z, int64_t ldb, int64_t n, int nrhs,
    int nblk, const int32_t *__restrict__ colblk, const int32_t *__restrict__ active,
    const int32_t *__restrict__ conv, const double *__restrict__ zq,
    const double *__restrict__ pq) {
    const int br = blockIdx.y;
    if (!active[br / nrhs]) return;
    const int64_t i0 = int64_t(blockIdx.x) * kVecSpan + threadIdx.x, o0 = int64_t(br) * ldb;
    double p[kVecPer], z[kVecPer];
#pragma unroll
    for (int q = 0; q < kVecPer; q++) {
        const int64_t i = i0 + 256 * q;
        p[q] = i < n ? Pv[o0 + i] : 0.0;
        z[q] = i < n ? Z[o0 + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kVecPer; q++) {
        const int64_t i = i0 + 256 * q;
        if (i >= n) continue;
        const int sg = seg_of(br, nblk, colblk, i);
        if (conv[sg]) continue;
        const double beta = pq[sg] > 0.0 ? -zq[sg] / pq[sg] : 0.0;
        Pv[o0 + i] = z[q] + beta * p[q];
    }
}

}  // namespace

namespace {

// Algorithmic HBM bytes of the refinement kernels (used for per-launch
// timing only).  A x over nmat matrices with nrhs vectors each: every value
// of A (both triangles, row order) once per matrix, the shared column
// indices and row pointers once, nvec vectors of n per right-hand side.
double spmv_bytes(const sc_plan *P, double nmat, int nrhs, int nvec) {
    const double nnz = double(P->csr_ptr[P->n]);
    return nmat * (8.0 * nnz + double(nrhs) * nvec * 8.0 * double(P->n)) + 4.0 * nnz +
           8.0 * double(P->n);
}
double vec_bytes(const sc_plan *P, double nsys, int nvec) {
    return nsys * double(P->n) * 8.0 * nvec;
}

// Y = B - A X (mode 1) or A X (mode 0) for all right-hand sides of the
// active matrices, up to four right-hand sides per pass; psum and amax as
// in k_apply.
void apply_A(const sc_plan *P, const double *vc, const double *B,
             const double *X, double *Y, int64_t ldb, int batch, int nrhs, int mode,
             const int32_t *active, hipStream_t st, double *psum = nullptr,
             double *amax = nullptr) {
    const DevPlan *D = P->dev;
    const int64_t nsell = P->sell_ptr.back();
    const dim3 grid(unsigned(batch), unsigned((P->n + 255) / 256));
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
        const int nr = std::min(4, nrhs - r0);
#define SPCHOL_APPLY(NR)                                                                   \
    hipLaunchKernelGGL(k_apply<NR>, grid, dim3(256), 0, st, D->csr_ptr, D->sell_ptr,        \
                       D->sell_col, vc, nsell, B, X, Y, ldb, P->n, nrhs, r0, mode, active,   \
                       psum, int(grid.y), r0 == 0 ? amax : nullptr)
        if (nr == 1) SPCHOL_APPLY(1);
        else if (nr == 2) SPCHOL_APPLY(2);
        else if (nr == 3) SPCHOL_APPLY(3);
        else SPCHOL_APPLY(4);
#undef SPCHOL_APPLY
    }
}

// Y1 = B - A X1 and Y2 = A X2 with one read of A.
void apply_A2(const sc_plan *P, const double *vc, const double *B, const double *X1, double *Y1,
              const double *X2, double *Y2, int64_t ldb, int batch, int nrhs,
              const int32_t *active, double *psum, hipStream_t st) {
    const DevPlan *D = P->dev;
    const int64_t nsell = P->sell_ptr.back();
    const dim3 grid(unsigned(batch), unsigned((P->n + 255) / 256));
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
        const int nr = std::min(4, nrhs - r0);
#define SPCHOL_APPLY2(NR)                                                                  \
    hipLaunchKernelGGL(k_apply2<NR>, grid, dim3(256), 0, st, D->csr_ptr, D->sell_ptr,       \
                       D->sell_col, vc, nsell, B, X1, Y1, X2, Y2, ldb, P->n, nrhs, r0, active,  \
                       psum, int(grid.y))
        if (nr == 1) SPCHOL_APPLY2(1);
        else if (nr == 2) SPCHOL_APPLY2(2);
        else if (nr == 3) SPCHOL_APPLY2(3);
        else SPCHOL_APPLY2(4);
#undef SPCHOL_APPLY2
    }
}

// ||A_k||_inf of every (matrix, block) of a group plan into W.anorm, from
// the values in row order (W.vc)
void anorm_blocks(const sc_plan *P, RefineWs &W, int batch, int64_t nsell, hipStream_t st) {
    const DevPlan *D = P->dev;
    const int nblk = P->nblk;
    hipLaunchKernelGGL(k_anorm_part, dim3(32, batch * nblk), dim3(256), 0, st, D->csr_ptr,
                       D->sell_ptr, W.vc, nsell, D->blk_col0, nblk, W.part);
    hipLaunchKernelGGL(k_anorm_final, dim3((batch * nblk + 255) / 256), dim3(256), 0, st,
                       W.part, batch * nblk, W.anorm);
}

hipError_t refine_classical(const sc_plan *P, sc_numeric *N, const double *vals,
                            int64_t ldv, const double *b, double *x, int32_t nrhs,
                            int64_t ldb, double tol, int32_t maxit, double *stat_host,
                            int32_t *nactive_out, bool sync, hipStream_t st) {
    DevPlan *D = P->dev;
    RefineWs &W = N->rws;
    Profiler &prof = N->prof;
    const int batch = N->batch, nblk = P->nblk;
    const int nsys = batch * nrhs, nseg = nsys * nblk, per = nrhs * nblk;
    const int64_t n = P->n;
    const int32_t *colblk = nblk > 1 ? D->colblk : nullptr;
    const dim3 vgrid(unsigned((n + kVecSpan - 1) / kVecSpan), unsigned(nsys));
    const dim3 sgrid(unsigned((nseg + 255) / 256));
    const dim3 rgrid(unsigned((nseg + 3) / 4));  // one wave per system
    hipError_t e;
    // x0 = solve(b)
    hipLaunchKernelGGL(k_set_i32, dim3((batch + 255) / 256), dim3(256), 0, st, W.active, batch,
                       int32_t(1));
    hipLaunchKernelGGL(k_set_i32, sgrid, dim3(256), 0, st, W.conv, nseg, int32_t(0));
    e = spchol_solve_run(P, N, x, nrhs, ldb, st, nullptr, b);
    if (e != hipSuccess) return e;
    const int64_t nsell = P->sell_ptr.back();
    hipLaunchKernelGGL(k_gather_rows,
                       dim3(unsigned((nsell + 255) / 256), unsigned((batch + kGatherMats - 1) / kGatherMats)),
                       dim3(256), 0, st, D->sell_vidx, vals, ldv, nsell, batch, W.vc);
    int32_t nact = batch;
    // plans of one block: the norms of the test come from the residual's own
    // pass (partial sums per 256-row block), ||A||_inf from the first one
    const int nrb = int((n + 255) / 256);
    const bool fuse = nblk == 1;
    double *amax = W.part2 + size_t(3) * nsys * nrb;
    if (!fuse) anorm_blocks(P, W, batch, nsell, st);
    for (int it = 0;; it++) {
        prof.begin(KK_Spmv, 0.0, spmv_bytes(P, nact, nrhs, 3), st, 12.0 * double(P->nnzA) * nact);
        apply_A(P, W.vc, b, x, W.r, ldb, batch, nrhs, 1, W.active, st, fuse ? W.part2 : nullptr,
                fuse && it == 0 ? amax : nullptr);
        prof.end(st);
        if (fuse && it == 0)
            hipLaunchKernelGGL(k_anorm_blocks, dim3((batch + 3) / 4), dim3(256), 0, st, amax, nrb,
                               batch, W.anorm);
        if (!fuse) {
            prof.begin(KK_Vec, 0.0, vec_bytes(P, nact * nrhs, it == 0 ? 3 : 2), st);
            hipLaunchKernelGGL(k_sums, dim3(kRB, nseg), dim3(256), 0, st, W.r, b, x,
                               it == 0 ? 3 : 4, ldb, D->blk_col0, nblk, nrhs, W.active, W.conv,
                               W.part);
            prof.end(st);
        }
        hipLaunchKernelGGL(k_check, rgrid, dim3(256), 0, st, fuse ? W.part2 : W.part,
                           fuse ? nrb : kRB, nseg, nrhs, nblk, W.anorm, tol, it, W.active, W.conv,
                           W.stat);
        hipLaunchKernelGGL(k_active, dim3(1), dim3(256), 0, st, W.conv, batch, per, W.active,
                           W.count);
        if (sync) {
            e = hipMemcpyAsync(&nact, W.count, sizeof(int32_t), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return e;
        }
        if (nact == 0 || it >= maxit) break;
        e = spchol_solve_run(P, N, W.r, nrhs, ldb, st, W.active);
        if (e != hipSuccess) return e;
        prof.begin(KK_Vec, 0.0, vec_bytes(P, nact * nrhs, 3), st);
        hipLaunchKernelGGL(k_axpy, vgrid, dim3(256), 0, st, x, W.r, ldb, n, nrhs, nblk, colblk,
                           W.active, W.conv);
        prof.end(st);
    }
    if (!sync) return hipGetLastError();
    *nactive_out = nact;
    e = hipMemcpyAsync(stat_host, W.stat, sizeof(double) * 6 * nseg, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}

// Preconditioned conjugate gradients on A (FP64 vectors and products) with
// the stored factor as preconditioner; the stop rule is tested on the true
// residual b - A x after every step.  Every system runs its own recurrence
// (its own step lengths), so the blocks of a group plan stay independent.
hipError_t refine_pcg(const sc_plan *P, sc_numeric *N, const double *vals, int64_t ldv,
                      const double *b, double *x, int32_t nrhs, int64_t ldb, double tol,
                      int32_t maxit, double *stat_host, int32_t *nactive_out, bool sync,
                      hipStream_t st) {
    DevPlan *D = P->dev;
    RefineWs &W = N->rws;
    Profiler &prof = N->prof;
    const int batch = N->batch, nblk = P->nblk;
    const int nsys = batch * nrhs, nseg = nsys * nblk, per = nrhs * nblk;
    const int64_t n = P->n;
    const int32_t *colblk = nblk > 1 ? D->colblk : nullptr;
    const dim3 vgrid(unsigned((n + kVecSpan - 1) / kVecSpan), unsigned(nsys));
    const dim3 xgrid(unsigned((n + 255) / 256), unsigned(nsys));
    const dim3 sgrid(unsigned((nseg + 255) / 256));
    const dim3 rgrid(unsigned((nseg + 3) / 4));  // one wave per system
    const size_t vsz = size_t(nsys) * ldb;
    double *r = W.r, *z = W.r + vsz, *pv = W.r + 2 * vsz, *q = W.r + 3 * vsz, *rt = W.r + 4 * vsz;
    double *rz0 = W.sc, *rz1 = W.sc + nseg, *pq = W.sc + 2 * nseg, *zq = W.sc + 3 * nseg;
    hipError_t e;
    hipLaunchKernelGGL(k_set_i32, dim3((batch + 255) / 256), dim3(256), 0, st, W.active, batch,
                       int32_t(1));
    hipLaunchKernelGGL(k_set_i32, sgrid, dim3(256), 0, st, W.conv, nseg, int32_t(0));
    e = spchol_solve_run(P, N, x, nrhs, ldb, st, nullptr, b);  // x0 = M^{-1} b
    if (e != hipSuccess) return e;
    const int64_t nsell = P->sell_ptr.back();
    hipLaunchKernelGGL(k_gather_rows,
                       dim3(unsigned((nsell + 255) / 256), unsigned((batch + kGatherMats - 1) / kGatherMats)),
                       dim3(256), 0, st, D->sell_vidx, vals, ldv, nsell, batch, W.vc);
    int32_t nact = batch;
    // true residual b - A x into res, stop test; with pnext, q = A pnext in
    // the same pass over A, and for a plan of one block the norms of the test
    // and p.q of the next step from that pass too (pq_ready); ||A||_inf from
    // the first residual's pass (plans of one block)
    const int nrb = int((n + 255) / 256);
    double *amax = W.part2 + size_t(3) * nsys * nrb;
    if (nblk > 1) anorm_blocks(P, W, batch, nsell, st);
    bool pq_ready = false;
    auto check = [&](int it, double *res, const double *pnext) -> hipError_t {
        const bool fuse = pnext && nblk == 1 && it > 0;
        if (pnext) {
            prof.begin(KK_Spmv, 0.0, spmv_bytes(P, nact, nrhs, 5), st, 12.0 * double(P->nnzA) * nact);
            apply_A2(P, W.vc, b, x, res, pnext, q, ldb, batch, nrhs, W.active,
                     fuse ? W.part2 : nullptr, st);
        } else {
            prof.begin(KK_Spmv, 0.0, spmv_bytes(P, nact, nrhs, 3), st, 12.0 * double(P->nnzA) * nact);
            apply_A(P, W.vc, b, x, res, ldb, batch, nrhs, 1, W.active, st,
                    nblk == 1 ? W.part2 : nullptr, nblk == 1 && it == 0 ? amax : nullptr);
        }
        prof.end(st);
        if (nblk == 1 && it == 0)
            hipLaunchKernelGGL(k_anorm_blocks, dim3((batch + 3) / 4), dim3(256), 0, st, amax, nrb,
                               batch, W.anorm);
        if (!pnext && nblk == 1) {  // the test's norms came with the residual
            hipLaunchKernelGGL(k_check, rgrid, dim3(256), 0, st, W.part2, nrb, nseg, nrhs, nblk,
                               W.anorm, tol, it, W.active, W.conv, W.stat);
        } else if (fuse) {
            hipLaunchKernelGGL(k_check, rgrid, dim3(256), 0, st, W.part2, nrb, nseg, nrhs, nblk,
                               W.anorm, tol, it, W.active, W.conv, W.stat);
            hipLaunchKernelGGL(k_sums_final, rgrid, dim3(256), 0, st, W.part2, nrb, 1, nseg, per,
                               W.active, pq, nullptr);
            pq_ready = true;
        } else {
            prof.begin(KK_Vec, 0.0, vec_bytes(P, nact * nrhs, it == 0 ? 3 : 2), st);
            hipLaunchKernelGGL(k_sums, dim3(kRB, nseg), dim3(256), 0, st, res, b, x,
                               it == 0 ? 3 : 4, ldb, D->blk_col0, nblk, nrhs, W.active, W.conv,
                               W.part);
            prof.end(st);
            hipLaunchKernelGGL(k_check, rgrid, dim3(256), 0, st, W.part, kRB, nseg, nrhs, nblk,
                               W.anorm, tol, it, W.active, W.conv, W.stat);
        }
        hipLaunchKernelGGL(k_active, dim3(1), dim3(256), 0, st, W.conv, batch, per, W.active,
                           W.count);
        if (!sync) return hipSuccess;  // every step runs; converged systems are skipped on device
        hipError_t e2 = hipMemcpyAsync(&nact, W.count, sizeof(int32_t), hipMemcpyDeviceToHost,
                                       st);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
        return e2;
    };
    // dot products <a, c> of every system into out[seg]
    auto dots = [&](const double *a, const double *c, double *out) {
        prof.begin(KK_Vec, 0.0, vec_bytes(P, nact * nrhs, 2), st);
        hipLaunchKernelGGL(k_sums, dim3(kRB, nseg), dim3(256), 0, st, a, c, nullptr, 1, ldb,
                           D->blk_col0, nblk, nrhs, W.active, nullptr, W.part);
        prof.end(st);
        hipLaunchKernelGGL(k_sums_final, rgrid, dim3(256), 0, st, W.part, kRB, 0, nseg, per,
                           W.active, out, nullptr);
    };
    // <a, c> into out and <c, d> into out2, in one pass over c
    auto dots2 = [&](const double *a, const double *c, const double *d, double *out,
                     double *out2) {
        prof.begin(KK_Vec, 0.0, vec_bytes(P, nact * nrhs, 3), st);
        hipLaunchKernelGGL(k_sums, dim3(kRB, nseg), dim3(256), 0, st, a, c, d, 2, ldb,
                           D->blk_col0, nblk, nrhs, W.active, nullptr, W.part);
        prof.end(st);
        hipLaunchKernelGGL(k_sums_final, rgrid, dim3(256), 0, st, W.part, kRB, 0, nseg, per,
                           W.active, out, out2);
    };
    e = check(0, r, nullptr);  // r_0 = b - A x_0
    if (e != hipSuccess) return e;
    if (nact > 0 && maxit > 0) {
        e = spchol_solve_run(P, N, pv, nrhs, ldb, st, W.active, r);  // p_1 = z_0 = M^{-1} r_0
        if (e != hipSuccess) return e;
        double *rz = rz0, *rzn = rz1;
        if (nblk == 1) {
            // q_1 = A p_1 with r_0.p_1 and p_1.q_1 from the same pass
            prof.begin(KK_Spmv, 0.0, spmv_bytes(P, nact, nrhs, 3), st, 12.0 * double(P->nnzA) * nact);
            apply_A(P, W.vc, r, pv, q, ldb, batch, nrhs, 0, W.active, st, W.part2);
            prof.end(st);
            hipLaunchKernelGGL(k_sums_final, rgrid, dim3(256), 0, st, W.part2, nrb, 0, nseg, per,
                               W.active, pq, rz0);
            pq_ready = true;
        } else {
            dots(r, pv, rz0);
            prof.begin(KK_Spmv, 0.0, spmv_bytes(P, nact, nrhs, 2), st, 12.0 * double(P->nnzA) * nact);
            apply_A(P, W.vc, nullptr, pv, q, ldb, batch, nrhs, 0, W.active, st);  // q_1 = A p_1
            prof.end(st);
        }
        for (int it = 1; it <= maxit; it++) {
            if (!pq_ready) dots(pv, q, pq);
            pq_ready = false;
            // at the last step of the budget only x changes (the test below
            // forms the true residual)
            const bool last = it == maxit;
            prof.begin(KK_Vec, 0.0, vec_bytes(P, nact * nrhs, last ? 3 : 6), st);
            hipLaunchKernelGGL(k_cg_xr<1>, xgrid, dim3(256), 0, st, x, last ? nullptr : r, pv, q,
                               ldb, n, nrhs, nblk, colblk, W.active, W.conv, rz, pq);
            prof.end(st);
            if (it == maxit) {
                e = check(it, rt, nullptr);
                if (e != hipSuccess) return e;
                break;
            }
            // Without host synchronization (a fixed budget, as in a captured
            // graph) the next direction comes before this step's test, so that
            // the test's product and q = A p share one pass over A (a system
            // that passes the test is frozen from here on; its new p is
            // unused).  With it, the test comes first and a step that ends
            // the refinement costs no further solve; q = A p then takes a pass
            // of its own.  Both orders give the same bits: every sum is formed
            // by the same products in the same order.
            if (sync) {
                e = check(it, rt, nullptr);
                if (e != hipSuccess) return e;
                if (nact == 0) break;
            }
            e = spchol_solve_run(P, N, z, nrhs, ldb, st, W.active, r);
            if (e != hipSuccess) return e;
            dots2(r, z, q, rzn, zq);
            prof.begin(KK_Vec, 0.0, vec_bytes(P, nact * nrhs, 3), st);
            hipLaunchKernelGGL(k_cg_p, vgrid, dim3(256), 0, st, pv, z, ldb, n, nrhs, nblk,
                               colblk, W.active, W.conv, zq, pq);
            prof.end(st);
            std::swap(rz, rzn);
            if (!sync) {
                e = check(it, rt, pv);
                if (e != hipSuccess) return e;
            } else if (nblk == 1) {
                // q = A p with p.q from the same pass (component 0)
                prof.begin(KK_Spmv, 0.0, spmv_bytes(P, nact, nrhs, 3), st, 12.0 * double(P->nnzA) * nact);
                apply_A(P, W.vc, r, pv, q, ldb, batch, nrhs, 0, W.active, st, W.part2);
                prof.end(st);
                hipLaunchKernelGGL(k_sums_final, rgrid, dim3(256), 0, st, W.part2, nrb, 0, nseg,
                                   per, W.active, pq, nullptr);
                pq_ready = true;
            } else {
                prof.begin(KK_Spmv, 0.0, spmv_bytes(P, nact, nrhs, 2), st, 12.0 * double(P->nnzA) * nact);
                apply_A(P, W.vc, nullptr, pv, q, ldb, batch, nrhs, 0, W.active, st);
                prof.end(st);
            }
        }
    }
    if (!sync) return hipGetLastError();
    *nactive_out = nact;
    e = hipMemcpyAsync(stat_host, W.stat, sizeof(double) * 6 * nseg, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}

// Value gradients of the adjoint, one thread per (stored entry, matrix):
// entry k = (i, j) of the caller's lower triangle stands for A_ij and A_ji,
// so g = -sum_r (lam_i x_j + lam_j x_i) off the diagonal and -sum_r lam_i x_i
// on it (right-hand sides ascending).
__global__ __launch_bounds__(256) void k_adjoint_values(
    const int32_t *__restrict__ vrow, const int32_t *__restrict__ vcol, int64_t nnz,
    const double *__restrict__ X, const double *__restrict__ LAM, int nrhs, int64_t ldb,
    double *__restrict__ G, int64_t ldv) {
    const int b = blockIdx.y;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int64_t i = vrow[k], j = vcol[k];
    double g = 0.0;
    for (int r = 0; r < nrhs; r++) {
        const double *x = X + (int64_t(b) * nrhs + r) * ldb;
        const double *l = LAM + (int64_t(b) * nrhs + r) * ldb;
        const double t = l[i] * x[j];
        g -= i == j ? t : t + l[j] * x[i];
    }
    G[int64_t(b) * ldv + k] = g;
}

}  // namespace

hipError_t spchol_refine_run(const sc_plan *P, sc_numeric *N, const double *vals, int64_t ldv,
                             const double *b, double *x, int32_t nrhs, int64_t ldb, double tol,
                             int32_t maxit, int32_t method, double *stat_host,
                             int32_t *nactive_out, bool sync, hipStream_t st) {
    if (method == 1)
        return refine_pcg(P, N, vals, ldv, b, x, nrhs, ldb, tol, maxit, stat_host, nactive_out,
                          sync, st);
    return refine_classical(P, N, vals, ldv, b, x, nrhs, ldb, tol, maxit, stat_host,
                            nactive_out, sync, st);
}

hipError_t spchol_adjoint_values(const sc_plan *P, int batch, const double *x, const double *lam,
                                 int32_t nrhs, int64_t ldb, double *g, int64_t ldv,
                                 hipStream_t st) {
    const int64_t nnz = P->nnzA;
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adjoint_values, dim3(unsigned((nnz + 255) / 256), unsigned(batch)),
                       dim3(256), 0, st, P->dev->val_row, P->dev->val_col, nnz, x, lam, nrhs,
                       ldb, g, ldv);
    return hipGetLastError();
}
