// Forward and backward triangular solves with the supernodal factor
// (gfx950).  y = L^{-1} P b by levels ascending, z = L^{-T} y by levels
// descending, x = P^T z.  The factor may be stored in FP64 or FP32; the
// solves always compute in FP64.
//
// Every supernode s owns a front vector FV_s of c_s entries: the first w_s
// hold its right-hand side, the last m_s its negated update vector
// u~_s = -sum over its subtree of L[R_s, k] y_k, which the parent pulls.
// Every value is written by exactly one workgroup, children are folded in a
// fixed order and reductions use fixed trees, so results are
// bit-reproducible and free of floating-point atomics.
//
// Small supernodes are solved by one workgroup out of LDS.  Wide or tall
// ones are solved by 64-column panels across many workgroups, using the
// inverted 64x64 diagonal blocks computed after the factorization:
//   forward  y_p = D_p^{-1} v_p (every workgroup recomputes it), then each
//            workgroup updates its own 64 rows below the panel;
//   backward each workgroup forms partial dot products for a chunk of rows,
//            the last one to finish (atomic counter, no waiting) sums them
//            in chunk order and applies D_p^{-T}.
#include <algorithm>

#include "device.hpp"

namespace {

constexpr int kP = kSolvePanel;

// Inverse of every 64x64 diagonal block of every panel-solved supernode:
// X = L_pp^{-1} by forward substitution, one lane per column of X kept in
// registers (loops fully unrolled), L_pp read from LDS as broadcasts.
template <typename T>
__global__ __launch_bounds__(64) void k_dinv(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const T *__restrict__ L, int64_t Lsize, double *__restrict__ Dinv, int64_t dsize) {
    __shared__ double Lp[kP * (kP + 1)];  // [i][t] row-major
    const int s = list[blockIdx.y];
    const int b = blockIdx.z;
    const SnDesc d = sn[s];
    const int p = blockIdx.x;
    const int c0 = p * kP;
    if (c0 >= d.w) return;
    const int kb = min(kP, d.w - c0);
    const int c = d.c;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    const int lane = threadIdx.x;
#pragma unroll 8
    for (int t = 0; t < kP; t++)
        Lp[lane * (kP + 1) + t] =
            (lane < kb && t < kb) ? double(Lb[int64_t(c0 + t) * c + c0 + lane]) : (lane == t ? 1.0 : 0.0);
    __syncthreads();
    double x[kP];
#pragma unroll
    for (int i = 0; i < kP; i++) {
        double sum = lane == i ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < i; t++) sum -= Lp[i * (kP + 1) + t] * x[t];
        x[i] = sum / Lp[i * (kP + 1) + i];
    }
    double *D = Dinv + int64_t(b) * dsize + d.dinv + int64_t(p) * kP * kP;
    __syncthreads();  // every read of Lp above precedes the transpose below
#pragma unroll
    for (int i = 0; i < kP; i++)  // column-major: D[col * 64 + i] = X[i][col], col = lane
        Lp[lane * (kP + 1) + i] = (lane < kb && i < kb) ? x[i] : 0.0;
    __syncthreads();
#pragma unroll 8
    for (int col = 0; col < kP; col++) D[col * kP + lane] = Lp[col * (kP + 1) + lane];
}

// Gather of the right-hand side and the children's update vectors into
// FV_s for the panel-solved supernodes of a level (their triangular solve
// runs in k_fwd_panel).  Item = (supernode, matrix and right-hand side).
__global__ __launch_bounds__(256) void k_fwd_gather(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ relmap,
    const int32_t *__restrict__ chlist, const double *__restrict__ B, int64_t ldb,
    double *__restrict__ FV, int64_t fvsize, int nrhs, const int32_t *__restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *v = reinterpret_cast<double *>(smem_raw);
    const int s = list[blockIdx.x];
    const int br = blockIdx.y;
    const int b = br / nrhs;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w;
    const int tid = threadIdx.x, nt = blockDim.x;
    const double *bb = B + int64_t(br) * ldb;
    double *fvb = FV + int64_t(br) * fvsize;

    for (int i = tid; i < c; i += nt) v[i] = i < w ? bb[perm[d.first + i]] : 0.0;
    for (int q = d.chbeg; q < d.chend; q++) {
        const SnDesc cd = sn[chlist[q]];
        const int32_t *rm = relmap + cd.relptr;
        const double *uc = fvb + cd.rowptr + cd.w;
        __syncthreads();
        for (int i = tid; i < cd.m; i += nt) v[rm[i]] += uc[i];
    }
    __syncthreads();
    for (int i = tid; i < c; i += nt) fvb[d.rowptr + i] = v[i];
}

__device__ inline void wave_sync_solve() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double bcast_lane(double v, int src) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(u & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane(int(u >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                (static_cast<unsigned int>(lo)));
}

constexpr int kWaveSlots = 8;  // rows per lane: c <= 512 for wave-solved supernodes

// Forward step of one level for supernodes solved by one wave each (w <= 64,
// c <= 512), NR right-hand sides of one matrix at a time: the right-hand
// side and the children's update vectors are gathered in LDS, then lane i
// keeps rows i + 64k in registers and the pivot value is broadcast with
// readlane.  Item = (supernode, matrix); four waves per workgroup.
template <typename T, int NR, int SL>
__global__ __launch_bounds__(256) void k_fwd_wave(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int nlist, int nitems,
    int r0, const int32_t *__restrict__ perm, const int32_t *__restrict__ relmap,
    const int32_t *__restrict__ chlist, const T *__restrict__ L, int64_t Lsize,
    const double *__restrict__ B, int64_t ldb, double *__restrict__ Y,
    double *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs, int cmax,
    const int32_t *__restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = blockIdx.x * 4 + wv;
    if (item >= nitems) return;
    const int s = list[item % nlist];
    const int b = item / nlist;
    if (active && !active[b]) return;
    double *v = reinterpret_cast<double *>(smem_raw) + size_t(wv) * NR * cmax;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w;
    const int br0 = b * nrhs + r0;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const double *bb = B + int64_t(br0 + r) * ldb;
        for (int i = lane; i < c; i += 64) v[r * cmax + i] = i < w ? bb[perm[d.first + i]] : 0.0;
    }
    for (int q = d.chbeg; q < d.chend; q++) {
        const SnDesc cd = sn[chlist[q]];
        const int32_t *rm = relmap + cd.relptr;
        wave_sync_solve();
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const double *uc = FV + int64_t(br0 + r) * fvsize + cd.rowptr + cd.w;
            for (int i = lane; i < cd.m; i += 64) v[r * cmax + rm[i]] += uc[i];
        }
    }
    wave_sync_solve();
    double x[SL][NR];
#pragma unroll
    for (int k = 0; k < SL; k++)
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const int i = lane + 64 * k;
            x[k][r] = i < c ? v[r * cmax + i] : 0.0;
        }
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    for (int j0 = 0; j0 < w; j0 += 8) {
        // eight columns of L in flight at once
        T lc[8][SL];
#pragma unroll
        for (int jj = 0; jj < 8; jj++)
#pragma unroll
            for (int k = 0; k < SL; k++) {
                const int i = lane + 64 * k;
                lc[jj][k] = (j0 + jj < w && i < c) ? Lb[int64_t(j0 + jj) * c + i] : T(0);
            }
#pragma unroll
        for (int jj = 0; jj < 8; jj++) {
            const int j = j0 + jj;
            if (j < w) {
                const double ljj = bcast_lane(double(lc[jj][0]), j);
                double yj[NR];
#pragma unroll
                for (int r = 0; r < NR; r++) yj[r] = bcast_lane(x[0][r], j) / ljj;
                if (lane == j) {
#pragma unroll
                    for (int r = 0; r < NR; r++) x[0][r] = yj[r];
                }
#pragma unroll
                for (int k = 0; k < SL; k++) {
                    const int i = lane + 64 * k;
                    if (i > j && i < c) {
                        const double l = double(lc[jj][k]);
#pragma unroll
                        for (int r = 0; r < NR; r++) x[k][r] -= l * yj[r];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double *y = Y + int64_t(br0 + r) * n;
        double *fv = FV + int64_t(br0 + r) * fvsize + d.rowptr;
#pragma unroll
        for (int k = 0; k < SL; k++) {
            const int i = lane + 64 * k;
            if (i < w) y[d.first + i] = x[k][r];
            else if (i < c) fv[i] = x[k][r];
        }
    }
}

// Backward step of one level for wave-solved supernodes: lane i keeps rows
// i + 64k of the solution; each column's dot product is a wave reduction
// (fixed butterfly order) and the lane owning the pivot row applies it.
template <typename T, int NR, int SL>
__global__ __launch_bounds__(256) void k_bwd_wave(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int nlist, int nitems,
    int r0, const int32_t *__restrict__ perm, const int32_t *__restrict__ rows,
    const T *__restrict__ L, int64_t Lsize, double *__restrict__ X, int64_t ldb,
    double *__restrict__ Y, int64_t n, int nrhs, const int32_t *__restrict__ active) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = blockIdx.x * 4 + wv;
    if (item >= nitems) return;
    const int s = list[item % nlist];
    const int b = item / nlist;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w;
    const int br0 = b * nrhs + r0;
    const int32_t *R = rows + d.rowptr;
    double x[SL][NR];
#pragma unroll
    for (int k = 0; k < SL; k++) {
        const int i = lane + 64 * k;
        const int64_t pos = i < w ? d.first + i : (i < c ? R[i] : 0);
#pragma unroll
        for (int r = 0; r < NR; r++) x[k][r] = i < c ? Y[int64_t(br0 + r) * n + pos] : 0.0;
    }
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    for (int j1 = w - 1; j1 >= 0; j1 -= 8) {
        // columns j1, j1-1, ..., j1-7 in flight at once
        T lc[8][SL];
#pragma unroll
        for (int jj = 0; jj < 8; jj++)
#pragma unroll
            for (int k = 0; k < SL; k++) {
                const int i = lane + 64 * k;
                lc[jj][k] = (j1 - jj >= 0 && i < c) ? Lb[int64_t(j1 - jj) * c + i] : T(0);
            }
#pragma unroll
        for (int jj = 0; jj < 8; jj++) {
            const int j = j1 - jj;
            if (j >= 0) {
                double t[NR];
#pragma unroll
                for (int r = 0; r < NR; r++) t[r] = 0.0;
#pragma unroll
                for (int k = 0; k < SL; k++) {
                    const int i = lane + 64 * k;
                    if (i > j && i < c) {
                        const double l = double(lc[jj][k]);
#pragma unroll
                        for (int r = 0; r < NR; r++) t[r] += l * x[k][r];
                    }
                }
#pragma unroll
                for (int r = 0; r < NR; r++) {
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) t[r] += __shfl_xor(t[r], off);
                }
                if (lane == j) {
                    const double ljj = double(lc[jj][0]);
#pragma unroll
                    for (int r = 0; r < NR; r++) x[0][r] = (x[0][r] - t[r]) / ljj;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double *y = Y + int64_t(br0 + r) * n;
        double *xo = X + int64_t(br0 + r) * ldb;
        if (lane < w) {
            y[d.first + lane] = x[0][r];
            xo[perm[d.first + lane]] = x[0][r];
        }
    }
}

// Forward step of one level for supernodes with c <= CM rows, one lane per
// (supernode, matrix, right-hand side): lane-private registers hold the
// front vector; the right-hand side and the children's update vectors are
// pulled through the gather map (no shared scatter), and the triangular
// solve runs in registers (every index a compile-time constant; rows and
// columns beyond the supernode are masked, their loads clamped in bounds).
template <typename T, int CM>
__global__ __launch_bounds__(256) void k_fwd_lane(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int nlist, int nitems,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ gptr,
    const int32_t *__restrict__ gidx, const T *__restrict__ L, int64_t Lsize,
    const double *__restrict__ B, int64_t ldb, double *__restrict__ Y, double *__restrict__ FV,
    int64_t n, int64_t fvsize, int nrhs, const int32_t *__restrict__ active) {
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= nitems) return;
    const int br = item / nlist;
    const int b = br / nrhs;
    if (active && !active[b]) return;
    const SnDesc d = sn[list[item - br * nlist]];
    const int c = d.c, w = d.w;
    const double *bb = B + int64_t(br) * ldb;
    double *fv = FV + int64_t(br) * fvsize;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    double x[CM];
#pragma unroll
    for (int i = 0; i < CM; i++) {
        double a = 0.0;
        if (i < c) {
            if (i < w) a = bb[perm[d.first + i]];
            const int g1 = gptr[d.rowptr + i + 1];
            for (int g = gptr[d.rowptr + i]; g < g1; g++) a += fv[gidx[g]];
        }
        x[i] = a;
    }
    // row by row: x_i -= sum_{j < min(i, w)} L_ij y_j (ascending j), then the
    // pivot division for the supernode's own columns
#pragma unroll
    for (int i = 1; i < CM; i++) {
        if (i - 1 < w) x[i - 1] /= double(Lb[(i - 1) * c + i - 1]);
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < i; j++) {
            const bool ok = j < w && i < c;
            const double l = double(Lb[ok ? j * c + i : 0]);
            t += ok ? l * x[j] : 0.0;
        }
        x[i] -= t;
    }
    if (CM - 1 < w) x[CM - 1] /= double(Lb[(CM - 1) * c + CM - 1]);
    double *y = Y + int64_t(br) * n + d.first;
#pragma unroll
    for (int i = 0; i < CM; i++) {
        if (i < w) y[i] = x[i];
        else if (i < c) fv[d.rowptr + i] = x[i];
    }
}

// Backward step of one level for supernodes with c <= CM rows, one lane per
// (supernode, matrix, right-hand side): rows below the supernode's columns
// are read from the solved ancestors, then columns are solved from the
// last to the first (dot products in ascending row order).
template <typename T, int CM>
__global__ __launch_bounds__(256) void k_bwd_lane(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int nlist, int nitems,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ rows,
    const T *__restrict__ L, int64_t Lsize, double *__restrict__ X, int64_t ldb,
    double *__restrict__ Y, int64_t n, int nrhs, const int32_t *__restrict__ active) {
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= nitems) return;
    const int br = item / nlist;
    const int b = br / nrhs;
    if (active && !active[b]) return;
    const SnDesc d = sn[list[item - br * nlist]];
    const int c = d.c, w = d.w;
    const double *y = Y + int64_t(br) * n;
    const int32_t *R = rows + d.rowptr;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    double x[CM];
#pragma unroll
    for (int i = 0; i < CM; i++) x[i] = i < w ? y[d.first + i] : (i < c ? y[R[i]] : 0.0);
#pragma unroll
    for (int j = CM - 1; j >= 0; j--) {
        asm volatile("" ::: "memory");  // one column of L in flight at a time
        const bool cj = j < w;
        double t = 0.0;
#pragma unroll
        for (int i = j + 1; i < CM; i++) {
            const bool ok = cj && i < c;
            const double l = double(Lb[ok ? j * c + i : 0]);
            t += ok ? l * x[i] : 0.0;
        }
        if (cj) x[j] = (x[j] - t) / double(Lb[j * c + j]);
    }
    double *yo = Y + int64_t(br) * n + d.first;
    double *xo = X + int64_t(br) * ldb;
#pragma unroll
    for (int i = 0; i < CM; i++)
        if (i < w) {
            yo[i] = x[i];
            xo[perm[d.first + i]] = x[i];
        }
}

// Forward panel p of panel-solved supernodes.  Workgroup 0 writes y_p;
// workgroup t >= 1 updates rows [c0 + kb + 64 (t-1), +64) of FV_s.
template <typename T>
__global__ __launch_bounds__(64) void k_fwd_panel(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int p,
    const T *__restrict__ L, int64_t Lsize, const double *__restrict__ Dinv,
    int64_t dsize, double *__restrict__ Y, double *__restrict__ FV, int64_t n,
    int64_t fvsize, int nrhs, const int32_t *__restrict__ active) {
    __shared__ double y[kP];
    const int s = list[blockIdx.y];
    const int br = blockIdx.z;
    const int b = br / nrhs;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c0 = p * kP;
    if (c0 >= d.w) return;
    const int kb = min(kP, d.w - c0);
    const int c = d.c;
    const int tile = blockIdx.x;
    const int r0 = tile == 0 ? c0 : c0 + kb + (tile - 1) * kP;
    if (r0 >= c) return;
    double *fv = FV + int64_t(br) * fvsize + d.rowptr;
    const double *Dp = Dinv + int64_t(b) * dsize + d.dinv + int64_t(p) * kP * kP;
    const int lane = threadIdx.x;
    __shared__ double vp[kP];
    vp[lane] = lane < kb ? fv[c0 + lane] : 0.0;
    __syncthreads();
    double yi = 0.0;
#pragma unroll 16
    for (int t = 0; t < kP; t++) yi += Dp[t * kP + lane] * vp[t];  // D is zero-padded
    y[lane] = yi;
    __syncthreads();
    if (tile == 0) {
        if (lane < kb) Y[int64_t(br) * n + d.first + c0 + lane] = yi;
        return;
    }
    const int r = r0 + lane;
    if (r < c) {
        const T *Lb = L + int64_t(b) * Lsize + d.loff + int64_t(c0) * c + r;
        double acc0 = 0.0, acc1 = 0.0;
        int t = 0;
#pragma unroll 8
        for (; t + 1 < kb; t += 2) {
            acc0 += double(Lb[int64_t(t) * c]) * y[t];
            acc1 += double(Lb[int64_t(t + 1) * c]) * y[t + 1];
        }
        if (t < kb) acc0 += double(Lb[int64_t(t) * c]) * y[t];
        fv[r] -= acc0 + acc1;
    }
}

// Backward panel p of panel-solved supernodes, NR right-hand sides of one
// matrix per workgroup: partial sums of L[r, c0 + t] z_r over a chunk of
// kSolveChunk rows below the panel (wave g owns columns g + 4k, each thread
// four rows); the last workgroup of the (supernode, matrix) sums the chunks
// in order and solves with D_p^T.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_bwd_panel(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int list0, int p, int r0,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ rows,
    const T *__restrict__ L, int64_t Lsize, const double *__restrict__ Dinv, int64_t dsize,
    double *__restrict__ X, int64_t ldb, double *__restrict__ Y, int64_t n,
    double *__restrict__ PART, int64_t psize, int32_t *__restrict__ cnt, int batch, int nrhs,
    const int32_t *__restrict__ active) {
    __shared__ double rhs[NR][kP];
    __shared__ double Dt[kP * (kP + 1)];
    __shared__ int last;
    const int s = list[blockIdx.y];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c0 = p * kP;
    if (c0 >= d.w) return;
    const int kb = min(kP, d.w - c0);
    const int c = d.c, w = d.w;
    const int rbeg = c0 + kb;
    const int nch = max(1, (c - rbeg + kSolveChunk - 1) / kSolveChunk);
    const int chunk = blockIdx.x;
    if (chunk >= nch) return;
    const int tid = threadIdx.x, lane = tid & 63, cg = tid >> 6;
    const int br0 = b * nrhs + r0;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    const int32_t *R = rows + d.rowptr;
    const int rb = rbeg + chunk * kSolveChunk;
    double z[4][NR];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int r = rb + 64 * q + lane;
        const int64_t pos = r < c ? (r < w ? d.first + r : R[r]) : 0;
#pragma unroll
        for (int k = 0; k < NR; k++) z[q][k] = r < c ? Y[int64_t(br0 + k) * n + pos] : 0.0;
    }
    double acc[16][NR];
#pragma unroll
    for (int j = 0; j < 16; j++)
#pragma unroll
        for (int k = 0; k < NR; k++) acc[j][k] = 0.0;
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int t = cg + 4 * j;
        if (t < kb) {
            const T *lc = Lb + int64_t(c0 + t) * c;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int r = rb + 64 * q + lane;
                const double l = r < c ? double(lc[r]) : 0.0;
#pragma unroll
                for (int k = 0; k < NR; k++) acc[j][k] += l * z[q][k];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 16; j++)
#pragma unroll
        for (int k = 0; k < NR; k++) {
            double v = acc[j][k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            acc[j][k] = v;
        }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int t = cg + 4 * j;
            if (t < kb)
#pragma unroll
                for (int k = 0; k < NR; k++)
                    PART[int64_t(br0 + k) * psize + d.part + chunk * kP + t] = acc[j][k];
        }
    }
    __threadfence();
    __syncthreads();
    int32_t *ctr = cnt + int64_t(list0 + blockIdx.y) * batch + b;
    if (tid == 0) last = atomicAdd(ctr, 1) == nch - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    {
        // the inverse block, coalesced into LDS: Dt[t][i] = Dp[t * 64 + i]
        const double *Dp = Dinv + int64_t(b) * dsize + d.dinv + int64_t(p) * kP * kP;
#pragma unroll
        for (int q = 0; q < kP * kP / 256; q++) {
            const int e = q * 256 + tid;
            Dt[(e >> 6) * (kP + 1) + (e & 63)] = Dp[e];
        }
    }
    if (tid < kb) {
#pragma unroll
        for (int k = 0; k < NR; k++) {
            const double *part = PART + int64_t(br0 + k) * psize + d.part;
            double s0 = 0.0;
            for (int q = 0; q < nch; q++) s0 += part[q * kP + tid];
            rhs[k][tid] = Y[int64_t(br0 + k) * n + d.first + c0 + tid] - s0;
        }
    }
    __syncthreads();
    if (tid < kb) {
        // x_t = sum_i (L_pp^{-1})[i][t] rhs_i; column t of the inverse is Dt[t][.]
        double xt[NR];
#pragma unroll
        for (int k = 0; k < NR; k++) xt[k] = 0.0;
        for (int i = 0; i < kb; i++) {
            const double dti = Dt[tid * (kP + 1) + i];
#pragma unroll
            for (int k = 0; k < NR; k++) xt[k] += dti * rhs[k][i];
        }
#pragma unroll
        for (int k = 0; k < NR; k++) {
            Y[int64_t(br0 + k) * n + d.first + c0 + tid] = xt[k];
            X[int64_t(br0 + k) * ldb + perm[d.first + c0 + tid]] = xt[k];
        }
    }
    if (tid == 0) *ctr = 0;
}

template <typename T>
hipError_t dinv_impl(const sc_plan *P, sc_numeric *N, hipStream_t st) {
    if (P->npan == 0) return hipSuccess;
    DevPlan *D = P->dev;
    const T *L = static_cast<const T *>(N->L);
    const int64_t maxp = (P->max_width + kP - 1) / kP;
    N->prof.begin(KK_Dinv, 0.0, 0.0, st);
    hipLaunchKernelGGL(k_dinv<T>, dim3(unsigned(maxp), unsigned(P->npan), unsigned(N->batch)),
                       dim3(64), 0, st, D->sn, D->slv_pan, L, P->Lsize, N->dinv, P->dinv_size);
    N->prof.end(st);
    return hipGetLastError();
}

template <typename T>
hipError_t solve_impl(const sc_plan *P, sc_numeric *N, double *b, int32_t nrhs,
                      int64_t ldb, hipStream_t st, const int32_t *active) {
    DevPlan *D = P->dev;
    for (const SLaunch &l : D->ssched) {
        if (size_t(l.maxc_pan) * sizeof(double) > size_t(g_max_lds)) return hipErrorInvalidValue;
        if (size_t(16) * l.maxc_small * sizeof(double) > size_t(g_max_lds))
            return hipErrorInvalidValue;
        if (l.maxc_small > 64 * kWaveSlots) return hipErrorInvalidValue;
    }
    const T *L = static_cast<const T *>(N->L);
    const int nbr = N->batch * nrhs;
    const unsigned gy = unsigned(nbr);
    const int64_t fvsize = int64_t(P->rows.size());
    Profiler &prof = N->prof;
    const double sz = double(sizeof(T)), nr = double(gy);
    for (const SLaunch &l : D->ssched) {
        if (l.nlane > 0) {
            prof.begin(KK_Fwd, l.f_lane * nr, (l.w_lane * sz * N->batch + l.v_lane * nr), st);
            const int nitems = l.nlane * nbr;
            const dim3 g(unsigned((nitems + 255) / 256));
#define SPCHOL_FWDL(CM)                                                                      \
    hipLaunchKernelGGL((k_fwd_lane<T, CM>), g, dim3(256), 0, st, D->sn,                       \
                       D->slv_small + l.lane0, l.nlane, nitems, D->perm, D->gptr, D->gidx, L, \
                       P->Lsize, b, ldb, N->ws_y, N->ws_u, P->n, fvsize, nrhs, active)
            if (l.maxc_lane <= 16) SPCHOL_FWDL(16);
            else SPCHOL_FWDL(32);
#undef SPCHOL_FWDL
            prof.end(st);
        }
        if (l.nsmall > 0) {
            prof.begin(KK_Fwd, l.f_small * nr, (l.w_small * sz * N->batch + l.v_small * nr), st);
            const int nitems = l.nsmall * N->batch;
            for (int r0 = 0; r0 < nrhs; r0 += 4) {
                const int nrr = std::min(4, nrhs - r0);
                const size_t lds = size_t(4) * nrr * l.maxc_small * sizeof(double);
                const dim3 g(unsigned((nitems + 3) / 4));
                const int32_t *lst = D->slv_small + l.small0;
                const int sl = l.maxc_small <= 64 ? 1 : l.maxc_small <= 128 ? 2
                             : l.maxc_small <= 256 ? 4 : 8;
#define SPCHOL_FWD(NRV, SLV)                                                                \
    hipLaunchKernelGGL((k_fwd_wave<T, NRV, SLV>), g, dim3(256), lds, st, D->sn, lst,        \
                       l.nsmall, nitems, r0, D->perm, D->relmap, D->chlist, L, P->Lsize, b,  \
                       ldb, N->ws_y, N->ws_u, P->n, fvsize, nrhs, l.maxc_small, active)
#define SPCHOL_FWD_SL(NRV)                                                                  \
    if (sl == 1) SPCHOL_FWD(NRV, 1);                                                        \
    else if (sl == 2) SPCHOL_FWD(NRV, 2);                                                   \
    else if (sl == 4) SPCHOL_FWD(NRV, 4);                                                   \
    else SPCHOL_FWD(NRV, 8)
                if (nrr == 1) { SPCHOL_FWD_SL(1); }
                else if (nrr == 2) { SPCHOL_FWD_SL(2); }
                else if (nrr == 3) { SPCHOL_FWD_SL(3); }
                else { SPCHOL_FWD_SL(4); }
#undef SPCHOL_FWD_SL
#undef SPCHOL_FWD
            }
            prof.end(st);
        }
        if (l.npan > 0) {
            prof.begin(KK_Fwd, 0.0, l.v_pan * nr, st);
            hipLaunchKernelGGL(k_fwd_gather, dim3(unsigned(l.npan), gy), dim3(256),
                               size_t(l.maxc_pan) * sizeof(double), st, D->sn,
                               D->slv_pan + l.pan0, D->perm, D->relmap, D->chlist, b, ldb,
                               N->ws_u, fvsize, nrhs, active);
            prof.end(st);
            for (size_t q = 0; q < l.panels.size(); q++) {
                const SPanel &pp = l.panels[q];
                prof.begin(KK_FwdPanel, pp.flops * nr, (pp.words * sz + pp.vbytes) * nr, st);
                hipLaunchKernelGGL(k_fwd_panel<T>,
                                   dim3(unsigned(1 + pp.fwd_tiles), unsigned(l.npan), gy),
                                   dim3(64), 0, st, D->sn, D->slv_pan + l.pan0, int(q), L,
                                   P->Lsize, N->dinv, P->dinv_size, N->ws_y, N->ws_u, P->n,
                                   fvsize, nrhs, active);
                prof.end(st);
            }
        }
    }
    for (auto it = D->ssched.rbegin(); it != D->ssched.rend(); ++it) {
        const SLaunch &l = *it;
        if (l.npan > 0) {
            for (size_t q = l.panels.size(); q-- > 0;) {
                const SPanel &pp = l.panels[q];
                prof.begin(KK_BwdPanel, pp.flops * nr,
                           pp.words * sz * N->batch + pp.vbytes * nr, st);
                for (int r0 = 0; r0 < nrhs; r0 += 4) {
                    const int nrr = std::min(4, nrhs - r0);
                    const dim3 g(unsigned(pp.bwd_chunks), unsigned(l.npan), unsigned(N->batch));
#define SPCHOL_BWDP(NRV)                                                                       \
    hipLaunchKernelGGL((k_bwd_panel<T, NRV>), g, dim3(256), 0, st, D->sn, D->slv_pan + l.pan0, \
                       l.pan0, int(q), r0, D->perm, D->rows, L, P->Lsize, N->dinv, P->dinv_size, \
                       b, ldb, N->ws_y, P->n, N->ws_part, P->part_size, N->ws_cnt, N->batch,    \
                       nrhs, active)
                    if (nrr == 1) SPCHOL_BWDP(1);
                    else if (nrr == 2) SPCHOL_BWDP(2);
                    else if (nrr == 3) SPCHOL_BWDP(3);
                    else SPCHOL_BWDP(4);
#undef SPCHOL_BWDP
                }
                prof.end(st);
            }
        }
        if (l.nsmall > 0) {
            prof.begin(KK_Bwd, l.f_small * nr, (l.w_small * sz * N->batch + l.v_small * nr), st);
            const int nitems = l.nsmall * N->batch;
            for (int r0 = 0; r0 < nrhs; r0 += 4) {
                const int nrr = std::min(4, nrhs - r0);
                const dim3 g(unsigned((nitems + 3) / 4));
                const int32_t *lst = D->slv_small + l.small0;
                const int sl = l.maxc_small <= 64 ? 1 : l.maxc_small <= 128 ? 2
                             : l.maxc_small <= 256 ? 4 : 8;
#define SPCHOL_BWD(NRV, SLV)                                                                 \
    hipLaunchKernelGGL((k_bwd_wave<T, NRV, SLV>), g, dim3(256), 0, st, D->sn, lst, l.nsmall, \
                       nitems, r0, D->perm, D->rows, L, P->Lsize, b, ldb, N->ws_y, P->n,     \
                       nrhs, active)
#define SPCHOL_BWD_SL(NRV)                                                                   \
    if (sl == 1) SPCHOL_BWD(NRV, 1);                                                         \
    else if (sl == 2) SPCHOL_BWD(NRV, 2);                                                    \
    else if (sl == 4) SPCHOL_BWD(NRV, 4);                                                    \
    else SPCHOL_BWD(NRV, 8)
                if (nrr == 1) { SPCHOL_BWD_SL(1); }
                else if (nrr == 2) { SPCHOL_BWD_SL(2); }
                else if (nrr == 3) { SPCHOL_BWD_SL(3); }
                else { SPCHOL_BWD_SL(4); }
#undef SPCHOL_BWD_SL
#undef SPCHOL_BWD
            }
            prof.end(st);
        }
        if (l.nlane > 0) {
            prof.begin(KK_Bwd, l.f_lane * nr, (l.w_lane * sz * N->batch + l.v_lane * nr), st);
            const int nitems = l.nlane * nbr;
            const dim3 g(unsigned((nitems + 255) / 256));
#define SPCHOL_BWDL(CM)                                                                      \
    hipLaunchKernelGGL((k_bwd_lane<T, CM>), g, dim3(256), 0, st, D->sn,                       \
                       D->slv_small + l.lane0, l.nlane, nitems, D->perm, D->rows, L,          \
                       P->Lsize, b, ldb, N->ws_y, P->n, nrhs, active)
            if (l.maxc_lane <= 16) SPCHOL_BWDL(16);
            else SPCHOL_BWDL(32);
#undef SPCHOL_BWDL
            prof.end(st);
        }
    }
    return hipGetLastError();
}

template <typename T, int NR>
void set_fwd_wave_lds(int big) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_wave<T, NR, 1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_wave<T, NR, 2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_wave<T, NR, 4>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_wave<T, NR, 8>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

template <typename T>
void set_solve_lds(int big) {
    set_fwd_wave_lds<T, 1>(big);
    set_fwd_wave_lds<T, 2>(big);
    set_fwd_wave_lds<T, 3>(big);
    set_fwd_wave_lds<T, 4>(big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_gather),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

}  // namespace

// Solve schedule per level, with the algorithmic work of each launch (per
// matrix and right-hand side).
void spchol_build_solve_schedule(const sc_plan *P, DevPlan *D) {
    D->ssched.clear();
    for (int32_t l = 0; l < P->nlevels; l++) {
        SLaunch s{};
        s.level = l;
        s.lane0 = P->slv_small_ptr[l];
        s.nlane = P->slv_lane_n[l];
        s.maxc_lane = P->slv_lane_maxc[l];
        s.small0 = s.lane0 + s.nlane;
        s.nsmall = P->slv_small_ptr[l + 1] - s.small0;
        for (int32_t e = s.lane0; e < s.lane0 + s.nlane; e++) {
            const SnDesc &d = P->sn[P->slv_small[e]];
            const double lw = double(d.c) * d.w - double(d.w) * (d.w - 1) / 2;
            s.f_lane += 2.0 * lw;
            s.w_lane += lw;
            s.v_lane += 8.0 * (2.0 * d.c + d.m) + 4.0 * d.c;
        }
        s.pan0 = P->slv_pan_ptr[l];
        s.npan = P->slv_pan_ptr[l + 1] - s.pan0;
        s.maxc_small = P->slv_small_maxc[l];
        s.maxc_pan = P->slv_pan_maxc[l];
        s.maxc = std::max(s.maxc_small, s.maxc_pan);
        for (int32_t e = s.small0; e < s.small0 + s.nsmall; e++) {
            const SnDesc &d = P->sn[P->slv_small[e]];
            const double lw = double(d.c) * d.w - double(d.w) * (d.w - 1) / 2;
            s.f_small += 2.0 * lw;
            s.w_small += lw;
            s.v_small += 8.0 * (2.0 * d.c + d.m) + 4.0 * d.c;
        }
        for (int32_t e = s.pan0; e < s.pan0 + s.npan; e++) {
            const SnDesc &d = P->sn[P->slv_pan[e]];
            s.v_pan += 8.0 * (2.0 * d.c) + 4.0 * d.c;
        }
        const int np = (P->slv_pan_maxw[l] + kP - 1) / kP;
        for (int q = 0; q < np; q++) {
            SPanel pp{};
            for (int32_t e = s.pan0; e < s.pan0 + s.npan; e++) {
                const SnDesc &d = P->sn[P->slv_pan[e]];
                const int c0 = q * kP;
                if (c0 >= d.w) continue;
                const int kb = std::min(kP, d.w - c0);
                const int64_t below = d.c - c0 - kb;
                pp.fwd_tiles = std::max<int64_t>(pp.fwd_tiles, (below + kP - 1) / kP);
                pp.bwd_chunks = std::max<int64_t>(
                    pp.bwd_chunks, std::max<int64_t>(1, (below + kSolveChunk - 1) / kSolveChunk));
                const double lw = double(below) * kb;
                pp.flops += 2.0 * lw + 2.0 * kb * kb;
                pp.words += lw;
                pp.vbytes += 8.0 * (below + 2.0 * kb) + 8.0 * kb * kb;
            }
            s.panels.push_back(pp);
        }
        D->ssched.push_back(s);
    }
}

hipError_t spchol_solve_init() {
    set_solve_lds<double>(g_max_lds);
    set_solve_lds<float>(g_max_lds);
    (void)hipGetLastError();
    return hipSuccess;
}

hipError_t spchol_dinv_run(const sc_plan *P, sc_numeric *N, hipStream_t st) {
    if (N->dtype == SC_F64) return dinv_impl<double>(P, N, st);
    return dinv_impl<float>(P, N, st);
}

hipError_t spchol_solve_run(const sc_plan *P, sc_numeric *N, double *b, int32_t nrhs,
                            int64_t ldb, hipStream_t st, const int32_t *active) {
    if (N->dtype == SC_F64) return solve_impl<double>(P, N, b, nrhs, ldb, st, active);
    return solve_impl<float>(P, N, b, nrhs, ldb, st, active);
}
