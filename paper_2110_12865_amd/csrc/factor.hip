// Numeric multifrontal Cholesky, level by level (gfx950).
//
// Every supernode s owns a front F_s of c_s rows: its first w_s columns are
// L's columns (stored as a c x w column-major block) and the trailing
// m x m block (m = c - w) is the update block U_s that its parent
// consumes.  A level of the supernodal tree is one group in the sense of
// the paper's grouping (Sec. 4.3): its members share no dependency, so all
// of them run in the same launch.
//
//   assembly   F_s  = A's columns of s (the value scatter, converted to the
//              factor precision on load) + sum over children of U_child
//              mapped through relative row indices.  Children are added in
//              a fixed order by the owner of each target entry, so results
//              are bit-reproducible and free of floating-point atomics.
//   factor     dense partial Cholesky of the first w columns of F_s and
//              Schur update of U_s.
//
// Fronts with few rows run entirely in one workgroup out of LDS.  Larger
// fronts are assembled one target column per workgroup and then factored by
// a right-looking blocked algorithm whose trailing update runs on the
// matrix cores (MFMA 16x16x4, FP64 or FP32).
#include <algorithm>
#include <climits>
#include <cmath>

#include "device.hpp"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA, one block.  Operands: lane l supplies A[l%16][l/16] and
// B[l/16][l%16].  Result: lane l, item q holds D[row(l/16, q)][l%16], where
// the row differs between the FP64 and FP32 instructions (measured on
// gfx950 with one-hot operands): FP64 rows are 4q + l/16, FP32 rows are
// 4(l/16) + q.
template <typename T> struct Mma;
template <> struct Mma<double> {
    typedef d4 acc_t;
    __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lk, int q) { return 4 * q + lk; }
};
template <> struct Mma<float> {
    typedef f4 acc_t;
    __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lk, int q) { return 4 * lk + q; }
};

__device__ inline double dsqrt(double x) { return sqrt(x); }
__device__ inline float dsqrt(float x) { return sqrtf(x); }

// Pivot of the diagonal-block factor, on its serial chain: rinv = 1 /
// sqrt(d) from the hardware estimate refined by Newton steps for the
// reciprocal square root, rinv <- rinv + rinv (1 - d rinv^2) / 2 (two in
// FP64, one in FP32), and ljj = d rinv; within a unit or two in the last
// place of the correctly rounded values, in far fewer dependent operations
// than a square root followed by a division.
__device__ inline void pivot_rs(double d, double &ljj, double &rinv) {
    double r = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const double e = fma(-(d * r), r, 1.0);
        r = fma(0.5 * r, e, r);
    }
    rinv = r;
    ljj = d * r;
}
__device__ inline void pivot_rs(float d, float &ljj, float &rinv) {
    float r = __builtin_amdgcn_rsqf(d);
    const float e = fmaf(-(d * r), r, 1.0f);
    r = fmaf(0.5f * r, e, r);
    rinv = r;
    ljj = d * r;
}

// Column j of a front: L columns live in the c x w block, update columns in
// the m x m block.  Returns a pointer p with the front entry (i, j) at p[i]
// (only rows i >= j are ever touched for update columns).
template <typename T>
__device__ inline T *front_col(T *Lb, T *Ub, int c, int w, int m, int j) {
    return j < w ? Lb + int64_t(j) * c : Ub + int64_t(j - w) * m - w;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ inline void wave_fence_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broadcast lane `src` (wave-uniform) of v to the whole wave.
__device__ inline double rl(double v, int src) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(u & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane(int(u >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<unsigned int>(lo));
}
__device__ inline float rl(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Value of lane `src` of the calling lane's segment of G lanes (G == 64:
// the whole wave, src wave-uniform).
template <int G, typename T>
__device__ inline T seg_bc(T v, int src) {
    if constexpr (G == 64)
        return rl(v, src);
    else
        return __shfl(v, src, G);
}

// Small fronts (c <= CM <= G) held in registers, one segment of G lanes per
// (front, matrix): a wave covers one front for 64 / G consecutive matrices
// (the same structure, so control flow is uniform), four fronts per
// workgroup.  Lane i of a segment keeps row i of the front, f[k] = F[i][k]
// for k <= i (entries above the diagonal are scratch).
//   assembly  A's entries are loaded lane-parallel and handed to their row
//             by broadcasts inside the segment; a child's update block is
//             read row-wise through the inverse of its relative map (an
//             LDS table shared by the segments).
//   factor    right-looking: the pivot is broadcast in the segment and
//             the column of L goes through LDS (row j + k at slot k, read
//             16 bytes at a time); after each step the registers shift left
//             by one so that the current column is always f[0] (every
//             register index is a compile-time constant).  Columns past
//             the front's last row are scratch and stop being updated.
template <typename T, int CM, int G>
__global__ __launch_bounds__(256) void k_front_reg(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int nlist, int batch,
    const int32_t *__restrict__ relmap, const int32_t *__restrict__ chlist,
    const int64_t *__restrict__ acolptr, const int32_t *__restrict__ aoff,
    const int64_t *__restrict__ avidx, const double *__restrict__ vals, int64_t ldv,
    T *__restrict__ L, int64_t Lsize, T *__restrict__ U, int64_t Usize,
    int32_t *__restrict__ info, int nblk) {
    static_assert(CM <= G && (G == 16 || G == 32 || G == 64), "segment shape");
    constexpr int NSEG = 64 / G;
    constexpr int V = 16 / int(sizeof(T));  // column entries per 16-byte LDS read
    __shared__ int32_t inv_all[4][64];
    // per segment: the current column of L, padded so that the segments of a
    // wave read from different banks
    __shared__ __align__(16) T cbuf[4][NSEG][G + 4];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int e = blockIdx.x * 4 + wv;
    if (e >= nlist) return;
    const int li = lane % G, sg = lane / G;
    const int b = blockIdx.y * NSEG + sg;
    const bool bok = b < batch;
    const int64_t bb = bok ? b : int64_t(blockIdx.y) * NSEG;  // in-bounds matrix for loads
    int32_t *inv = inv_all[wv];
    const int s = list[e];
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w, m = d.m;
    L += bb * Lsize;
    U += bb * Usize;
    vals += bb * ldv;

    T f[CM];
#pragma unroll
    for (int k = 0; k < CM; k++) f[k] = T(0);

    // A's columns of the front: entries [a0, a1), sorted by column
    const int64_t a0 = acolptr[d.first], a1 = acolptr[d.first + w];
    // first entry of column li, relative to a0
    const int acol = li < w ? int(acolptr[d.first + li] - a0) : int(a1 - a0);
    for (int64_t base = a0; base < a1; base += G) {
        const int64_t q = base + li;
        int row = -1;
        T val = T(0);
        if (q < a1) {
            row = aoff[q] % c;
            val = T(vals[avidx[q]]);
        }
        const int rb = int(base - a0);                       // this round: entries
        const int re = int((base + G < a1 ? base + G : a1) - a0);  // [rb, re)
#pragma unroll
        for (int k = 0; k < CM; k++) {
            // column k's entries in this round (none once k >= w)
            const int lo = k < w ? __builtin_amdgcn_readlane(acol, k) : re;
            const int hi = k + 1 < w ? __builtin_amdgcn_readlane(acol, (k + 1) % G) : int(a1 - a0);
            const int t0 = (lo > rb ? lo : rb) - rb;
            const int t1 = (hi < re ? hi : re) - rb;
            for (int t = t0; t < t1; t++) {
                const int r = __builtin_amdgcn_readlane(row, t);  // same in every segment
                const T v = seg_bc<G>(val, t);
                if (li == r) f[k] += v;
            }
        }
    }

    // children's update blocks
    for (int q = d.chbeg; q < d.chend; q++) {
        const SnDesc cd = sn[chlist[q]];
        const int mc = cd.m;
        const T *Uc = U + cd.uoff;
        if (sg == 0) inv[li] = -1;
        wave_fence_sync();
        if (sg == 0 && li < mc) inv[relmap[cd.relptr + li]] = li;
        wave_fence_sync();
        const int pi = inv[li];  // child row landing in front row li, or -1
        wave_fence_sync();
        // eight target columns at a time: all loads issued before any use
        // (addresses of absent entries are clamped to the block's first)
#pragma unroll
        for (int k0 = 0; k0 < CM; k0 += 8) {
            int qk[8];
#pragma unroll
            for (int t = 0; t < 8; t++) qk[t] = __builtin_amdgcn_readlane(pi, (k0 + t) % G);
            if ((qk[0] & qk[1] & qk[2] & qk[3] & qk[4] & qk[5] & qk[6] & qk[7]) == -1)
                continue;  // no column of this child lands here
            T v[8];
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const bool ok = qk[t] >= 0 && pi >= qk[t];
                v[t] = Uc[ok ? int64_t(qk[t]) * mc + pi : 0];
            }
#pragma unroll
            for (int t = 0; t < 8; t++)
                if (qk[t] >= 0 && pi >= qk[t]) f[k0 + t] += v[t];
        }
    }

    // partial factorization of the first w columns
    const int64_t infoidx = bb * nblk + d.blk;
    T *Lb = L + d.loff;
    T *cb = &cbuf[wv][sg][0];
    for (int j = 0; j < w; j++) {
        T djj = seg_bc<G>(f[0], j);
        const bool bad = !(djj > T(0));
        if (bad) {
            djj = T(1);
            if (li == 0 && bok) atomicMin(info + infoidx, d.first - d.bcol0 + j + 1);
        }
        const T ljj = dsqrt(djj);
        const T rinv = T(1) / ljj;
        const T lij = li == j ? ljj : (li > j ? f[0] * rinv : T(0));
        if (li < c && bok) Lb[int64_t(j) * c + li] = lij;
        if (li >= j) cb[li - j] = lij;
        wave_fence_sync();
        // f[k - 1] <- column j + k minus L_{., j} L_{j + k, j}; registers of
        // columns j + k >= c (all chunks from the first such one) keep
        // whatever they hold: those columns are never read
        // (groups of four reads: all issued before the first product)
#pragma unroll
        for (int k0 = 0; k0 < CM; k0 += 4 * V) {
            if (j + k0 >= c) continue;
            T v[4 * V];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                if (k0 + r * V >= CM) break;
                if constexpr (V == 4) {
                    const float4 q = *reinterpret_cast<const float4 *>(cb + k0 + 4 * r);
                    v[4 * r] = q.x; v[4 * r + 1] = q.y; v[4 * r + 2] = q.z; v[4 * r + 3] = q.w;
                } else {
                    const double2 q = *reinterpret_cast<const double2 *>(cb + k0 + 2 * r);
                    v[2 * r] = q.x; v[2 * r + 1] = q.y;
                }
            }
#pragma unroll
            for (int t = 0; t < 4 * V; t++) {
                const int k = k0 + t;
                if (k >= 1 && k < CM) f[k - 1] = fma(-lij, v[t], f[k]);
            }
        }
        wave_fence_sync();  // the column is read before the next step rewrites it
    }
    // f[k] now holds column w + k: the update block
    T *Us = U + d.uoff;
#pragma unroll
    for (int k = 0; k < CM; k++)
        if (k < m && li >= w + k && li < c && bok) Us[int64_t(k) * m + li - w] = f[k];
}

// Large fronts: assembly with one wave per (target column, matrix), `per`
// columns per workgroup (c_max scalars of LDS per wave).  The column is
// built in LDS from zeros, A's entries and then the children's pieces in
// their order (a front row receives at most one value per child, so each
// entry sums over the children in order), and written to L or U.  Pieces
// go four at a time, all their loads issued before the adds.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble_cols(
    const AsmCol *__restrict__ cols, const AsmPiece *__restrict__ pcs, int64_t ncols, int per,
    int cmax, const int32_t *__restrict__ relmap, const int32_t *__restrict__ aoff,
    const int64_t *__restrict__ avidx, const double *__restrict__ vals, int64_t ldv,
    T *__restrict__ L, int64_t Lsize, T *__restrict__ U, int64_t Usize) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (wv >= per) return;
    const int64_t g = int64_t(blockIdx.x) * per + wv;
    if (g >= ncols) return;
    T *col = reinterpret_cast<T *>(smem_raw) + size_t(wv) * cmax;
    const AsmCol a = cols[g];
    const int64_t b = blockIdx.y;
    const T *Ub = U + b * Usize;
    vals += b * ldv;
    for (int i = a.tj + lane; i < a.c; i += 64) col[i] = T(0);
    wave_fence_sync();
    for (int q = lane; q < a.na; q += 64) col[aoff[a.a0 + q] - a.base] = T(vals[avidx[a.a0 + q]]);
    constexpr int kU = 4;
    for (int k0 = 0; k0 < a.nch; k0 += kU) {
        int r[kU];
        T v[kU];
        bool ok[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const AsmPiece p = pcs[a.ch0 + min(k0 + u, a.nch - 1)];
            ok[u] = k0 + u < a.nch && lane < p.cnt;
            const int64_t o = ok[u] ? lane : 0;
            r[u] = relmap[p.rmp + o];
            v[u] = Ub[p.src + o];
        }
#pragma unroll
        for (int u = 0; u < kU; u++) {
            wave_fence_sync();
            if (ok[u]) col[r[u]] += v[u];
        }
    }
    wave_fence_sync();
    T *dst = (a.isU ? U + b * Usize : L + b * Lsize) + a.dst;
    for (int i = a.tj + lane; i < a.c; i += 64) dst[i] = col[i];
}

// Value of lane `src` (wave-uniform) broadcast to the whole wave.
template <typename T>
__device__ inline T lane_bcast(T v, int src);
template <>
__device__ inline double lane_bcast<double>(double v, int src) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(u & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane(int(u >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                (static_cast<unsigned int>(lo)));
}
template <>
__device__ inline float lane_bcast<float>(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Widest front held in registers; wider small fronts take the workgroup kernel.
constexpr int kFrontRegMaxC = 64;

// Factor and invert the kb x kb diagonal block (kb <= 64) whose top-left
// corner is (r0, r0) of a column-major L block, with one workgroup of 256
// threads.
//   factor   lane i of wave g keeps row i of columns 16 g .. 16 g + 15 in
//            registers (f).  Step j forms the pivot and column j of L
//            (i > j: L_ij = F_ij / L_jj) and every later column t takes
//            F_it -= L_ij L_tj.  Columns go in blocks of 16, one per wave:
//            the owning wave runs the block's 16 steps back to back (its own
//            columns need nothing from the other waves), publishing each
//            column of L in LDS; after one barrier the waves of later
//            columns replay the 16 steps on their registers.  Every entry
//            sees the same operations in the same order as with a barrier
//            per step.  A pivot that fails d > 0 is recorded (smallest
//            1-based step wins) and replaced by 1.
//   inverse  X = L^{-1} by 16 x 16 blocks once L is complete: wave g inverts
//            its diagonal block by forward substitution (rows in order,
//            X_kk = 1 / L_kk, row k broadcast through LDS), then the blocks
//            below the diagonal by distance d = 1, 2, 3 from it:
//            X_IJ = -X_II (sum_{K=J}^{I-1} L_IK X_KJ), one block per wave,
//            the 16 x 16 x 16 products on the matrix cores.
// Past kb the block is taken as the identity.  The factor is written back
// (zeros above the diagonal) and the inverse to PIg column-major
// (PIg[col * 64 + i] = X[i][col], zero outside the kb x kb block), and to Dg
// as well when given.
constexpr int kDiagLds = 2 * kTile * kTile + kTile + 4 * 16 * 16;  // L (column buffers first), X, 1/L_jj, T

template <typename T>
__device__ __forceinline__ void wg_diag_factor(T *Lb, int c, int r0, int kb, T *lds, T *PIg, T *Dg,
                                               int col0, int32_t *info_b) {
    T *cbuf = lds;                  // factor: [2][16][64] columns of L, by block parity
    T *Lsh = lds;                   // inverse: L, 64 x 64 column-major
    T *Xsh = lds + kTile * kTile;   // X, 64 x 64 column-major
    T *rv = Xsh + kTile * kTile;    // [64] 1 / L_jj (1 past kb)
    T *Tsh = rv + kTile;            // [4][16][16] one product per wave
    const int tid = threadIdx.x, li = tid & 63, g = tid >> 6;
    const int gu = __builtin_amdgcn_readfirstlane(g);  // the wave's index, as a scalar
    T f[16];
#pragma unroll
    for (int tt = 0; tt < 16; tt++) {
        const int col = 16 * g + tt;
        f[tt] = (li < kb && col < kb) ? Lb[int64_t(r0 + col) * c + r0 + li] : (li == col ? T(1) : T(0));
    }
    if (gu == 0) rv[li] = T(1);
    for (int J = 0; J < 4; J++) {
        if (16 * J >= kb) break;
        T *cbJ = cbuf + (J & 1) * 16 * kTile;
        if (gu == J) {
#pragma unroll
            for (int jj = 0; jj < 16; jj++) {
                const int j = 16 * J + jj;
                if (j < kb) {
                    T djj = lane_bcast(f[jj], j);
                    const bool bad = !(djj > T(0));
                    if (bad) djj = T(1);
                    T ljj, rinv;
                    pivot_rs(djj, ljj, rinv);
                    const T lij = li == j ? ljj : (li > j ? f[jj] * rinv : T(0));
                    f[jj] = lij;
                    cbJ[jj * kTile + li] = lij;
                    if (li == j) {
                        rv[j] = rinv;
                        if (bad) atomicMin(info_b, col0 + j + 1);
                    }
                    wave_fence_sync();
                    T cv[16];
#pragma unroll
                    for (int tt = 0; tt < 16; tt++) cv[tt] = cbJ[jj * kTile + 16 * J + tt];
#pragma unroll
                    for (int tt = 0; tt < 16; tt++)
                        if (tt > jj) f[tt] = fma(-lij, cv[tt], f[tt]);
                }
            }
        }
        __syncthreads();  // the block's columns of L are visible
        if (gu > J) {
#pragma unroll
            for (int jj = 0; jj < 16; jj++) {
                const int j = 16 * J + jj;
                if (j < kb) {
                    const T lij = cbJ[jj * kTile + li];
                    T cv[16];
#pragma unroll
                    for (int tt = 0; tt < 16; tt++) cv[tt] = cbJ[jj * kTile + 16 * g + tt];
#pragma unroll
                    for (int tt = 0; tt < 16; tt++) f[tt] = fma(-lij, cv[tt], f[tt]);
                }
            }
        }
    }
    __syncthreads();  // every replay has read the column buffers
#pragma unroll
    for (int tt = 0; tt < 16; tt++) {
        const int col = 16 * g + tt;
        if (li < kb && col < kb) Lb[int64_t(r0 + col) * c + r0 + li] = li >= col ? f[tt] : T(0);
        Lsh[col * kTile + li] = li >= col ? f[tt] : T(0);
    }
    // diagonal block g of X: lane 16 g + i keeps row i, x[t] = X[16 g + i][16 g + t]
    {
        const int ii = li - 16 * g;
        const bool mine = ii >= 0 && ii < 16;
        T *xrow = Tsh + 256 * gu;
        T x[16];
#pragma unroll
        for (int t = 0; t < 16; t++) x[t] = mine && t == ii ? T(1) : T(0);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (mine && ii == k) {
                const T r = rv[16 * g + k];
#pragma unroll
                for (int t = 0; t < 16; t++) {
                    x[t] *= r;
                    xrow[t] = x[t];
                }
            }
            wave_fence_sync();
            T xk[16];
#pragma unroll
            for (int t = 0; t < 16; t++) xk[t] = xrow[t];
            if (mine && ii > k) {
                const T lik = f[k];
#pragma unroll
                for (int t = 0; t < 16; t++) x[t] = fma(-lik, xk[t], x[t]);
            }
            wave_fence_sync();  // row k is read before the next one is written
        }
        if (mine) {
#pragma unroll
            for (int t = 0; t < 16; t++) Xsh[(16 * g + t) * kTile + li] = x[t];
        }
        // zeros above the diagonal blocks
#pragma unroll
        for (int tt = 0; tt < 16; tt++)
            if (li < 16 * g) Xsh[(16 * g + tt) * kTile + li] = T(0);
    }
    __syncthreads();
    const int lk = li >> 4, lm = li & 15;
    for (int dd = 1; dd < 4; dd++) {
        if (gu + dd < 4) {
            const int Jb = gu, Ib = gu + dd;
            T *Tw = Tsh + 256 * gu;
            // T = sum_K L_IK X_KJ: C[m][n] = sum_k A(m, k) B(n, k) with
            // A(m, k) = L[16 I + m][16 K + k], B(n, k) = X[16 K + k][16 J + n]
            typename Mma<T>::acc_t acc = Mma<T>::zero();
            for (int Kb = Jb; Kb < Ib; Kb++) {
#pragma unroll
                for (int kk = 0; kk < 16; kk += 4) {
                    const T av = Lsh[(16 * Kb + kk + lk) * kTile + 16 * Ib + lm];
                    const T bv = Xsh[(16 * Jb + lm) * kTile + 16 * Kb + kk + lk];
                    acc = Mma<T>::mma(av, bv, acc);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; r++) Tw[Mma<T>::row(lk, r) * 16 + lm] = acc[r];
            wave_fence_sync();
            // X_IJ = -X_II T: A(m, k) = X[16 I + m][16 I + k], B(n, k) = T[k][n]
            typename Mma<T>::acc_t acc2 = Mma<T>::zero();
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const T av = Xsh[(16 * Ib + kk + lk) * kTile + 16 * Ib + lm];
                const T bv = Tw[(kk + lk) * 16 + lm];
                acc2 = Mma<T>::mma(av, bv, acc2);
            }
#pragma unroll
            for (int r = 0; r < 4; r++)
                Xsh[(16 * Jb + lm) * kTile + 16 * Ib + Mma<T>::row(lk, r)] = -acc2[r];
        }
        __syncthreads();
    }
#pragma unroll
    for (int tt = 0; tt < 16; tt++) {
        const int col = 16 * g + tt;
        const bool in = li < kb && col < kb;
        const T xv = (in && li >= col) ? Xsh[col * kTile + li] : T(0);
        PIg[col * kTile + li] = xv;
        if (Dg) Dg[col * kTile + li] = xv;
    }
}

// C[j][i] += sum_t sA[t][j] * sB[t][i] for the wave's 32 x 32 quadrant of a
// 64 x 64 tile (rows j: 32 (wave & 1) + ..., columns i: 32 (wave >> 1) + ...),
// both operands in LDS as [t][64]; accumulates onto acc.
template <typename T>
__device__ inline void tile_mma(const T *sA, const T *sB, int kbr,
                                typename Mma<T>::acc_t (&acc)[2][2]) {
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    const int jw = (wv & 1) * 32, iw = (wv >> 1) * 32;
    const int lk = lane >> 4, lm = lane & 15;
    for (int kk = 0; kk < kbr; kk += 4) {
        const T *rA = sA + (kk + lk) * kTile;
        const T *rB = sB + (kk + lk) * kTile;
        T av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; a++) av[a] = rA[jw + 16 * a + lm];
#pragma unroll
        for (int q = 0; q < 2; q++) bv[q] = rB[iw + 16 * q + lm];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int q = 0; q < 2; q++) acc[a][q] = Mma<T>::mma(av[a], bv[q], acc[a][q]);
    }
}

template <typename T>
__device__ inline void acc_zero(typename Mma<T>::acc_t (&acc)[2][2]) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int q = 0; q < 2; q++) acc[a][q] = Mma<T>::zero();
}

// Position of accumulator item (a, q, r) of this lane inside the 64 x 64 tile
// computed by tile_mma: row j (first operand) and column i (second operand).
template <typename T>
__device__ inline void tile_pos(int a, int q, int r, int &j, int &i) {
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    j = (wv & 1) * 32 + 16 * a + Mma<T>::row(lane >> 4, r);
    i = (wv >> 1) * 32 + 16 * q + (lane & 15);
}

// Whole-block inverse X = L11^{-1} of the diagonal block of a panel-solved
// supernode, by 64-column block columns J (one workgroup of 256 threads per
// (J, supernode, matrix)): X_JJ = D_J, the inverted diagonal block the
// factor already holds, and below it, for I = J + 1, J + 2, ...,
//   X_IJ = -D_I (sum_{K=J}^{I-1} L_IK X_KJ),
// the standard block recurrence of the inverse of a lower-triangular matrix
// (from L X = I, block row I).  The 64 x 64 products run on the matrix cores
// with the K sum in ascending order; the next pair of operand tiles is in
// flight while the current one is multiplied.  The grid runs matrices
// fastest and the supernodes widest first, so the longest chains (block
// column 0 of the widest blocks) start first.  X is stored column-major
// with leading dimension w (entry (i, j) at j w + i); blocks above the
// diagonal blocks are never written nor read.
constexpr int kXPitch = kTile + 1;  // LDS pitch of the [t][i] operand written across lanes
template <typename T>
__device__ inline void xtile_mma(const T *sA, const T *sB, typename Mma<T>::acc_t (&acc)[2][2]) {
    // C[j][i] += sum_t sA[t * 64 + j] sB[t * kXPitch + i], the wave's 32 x 32 quadrant
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    const int jw = (wv & 1) * 32, iw = (wv >> 1) * 32;
    const int lk = lane >> 4, lm = lane & 15;
#pragma unroll 4
    for (int kk = 0; kk < kTile; kk += 4) {
        const T *rA = sA + (kk + lk) * kTile;
        const T *rB = sB + (kk + lk) * kXPitch;
        T av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; a++) av[a] = rA[jw + 16 * a + lm];
#pragma unroll
        for (int q = 0; q < 2; q++) bv[q] = rB[iw + 16 * q + lm];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int q = 0; q < 2; q++) acc[a][q] = Mma<T>::mma(av[a], bv[q], acc[a][q]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trtri(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int64_t *__restrict__ xoff, const T *__restrict__ L, int64_t Lsize,
    const T *__restrict__ Dinv, int64_t dsize, T *__restrict__ X, int64_t xsize) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sA = reinterpret_cast<T *>(smem_raw);  // [t][j]: L_IK[j][t], then D_I[j][t]
    T *sB = sA + kTile * kTile;               // [t][i] (pitch kXPitch): X_KJ[t][i], then T[t][i]
    const int b = blockIdx.x;
    const int J = blockIdx.y;
    const int s = list[blockIdx.z];
    const SnDesc d = sn[s];
    const int w = d.w, c = d.c;
    const int nb = (w + kTile - 1) / kTile;
    if (J >= nb) return;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    const T *Db = Dinv + int64_t(b) * dsize + d.dinv;
    T *Xb = X + int64_t(b) * xsize + xoff[s];
    const int tid = threadIdx.x, li = tid & 63, lt = tid >> 6;
    const int cJ = kTile * J, kbJ = min(kTile, w - cJ);
    // X_JJ = D_J (column-major, zero-padded past kbJ)
#pragma unroll
    for (int q = 0; q < 16; q++) {
        const int col = lt + 4 * q;
        if (col < kbJ && li < kbJ)
            Xb[int64_t(cJ + col) * w + cJ + li] = Db[int64_t(J) * kTile * kTile + col * kTile + li];
    }
    // below J every block column is whole: only block I may be partial
    T ra[16], rb[16];
    // operands of step (I, K): K < I gives L_IK and X_KJ, K == I gives D_I
    auto load = [&](int I, int K) {
        const int cI = kTile * I, kbI = min(kTile, w - cI);
        if (K < I) {
            const int cK = kTile * K;
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int t = lt + 4 * q;  // ra: L_IK[li][t]; rb: X_KJ[li][t] (t = column)
                ra[q] = li < kbI ? Lb[int64_t(cK + t) * c + cI + li] : T(0);
                rb[q] = Xb[int64_t(cJ + t) * w + cK + li];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int t = lt + 4 * q;  // D_I[li][t], zero-padded
                ra[q] = Db[int64_t(I) * kTile * kTile + t * kTile + li];
            }
        }
    };
    if (J + 1 < nb) load(J + 1, J);
    for (int I = J + 1; I < nb; I++) {
        const int cI = kTile * I, kbI = min(kTile, w - cI);
        typename Mma<T>::acc_t acc[2][2];
        acc_zero<T>(acc);
        for (int K = J; K < I; K++) {
            __syncthreads();  // the previous products have read sA and sB
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int t = lt + 4 * q;
                sA[t * kTile + li] = ra[q];
                sB[li * kXPitch + t] = rb[q];
            }
            __syncthreads();
            load(I, K + 1);  // the next pair (or D_I), in flight during the products
            xtile_mma(sA, sB, acc);
        }
        __syncthreads();  // the last products have read sA and sB
        // sB <- T (rows t of T are the K index of the next product), sA <- D_I
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int q = 0; q < 2; q++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    int j, i;
                    tile_pos<T>(a, q, r, j, i);
                    sB[j * kXPitch + i] = acc[a][q][r];
                }
#pragma unroll
        for (int q = 0; q < 16; q++) sA[(lt + 4 * q) * kTile + li] = ra[q];
        __syncthreads();
        if (I + 1 < nb) load(I + 1, J);
        typename Mma<T>::acc_t acc2[2][2];
        acc_zero<T>(acc2);
        xtile_mma(sA, sB, acc2);
        __syncthreads();  // sA is read; it now stages X_IJ for a coalesced store
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int q = 0; q < 2; q++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    int j, i;
                    tile_pos<T>(a, q, r, j, i);
                    sA[i * kTile + j] = -acc2[a][q][r];
                }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int col = lt + 4 * q;
            if (li < kbI) Xb[int64_t(cJ + col) * w + cI + li] = sA[col * kTile + li];
        }
    }
}

// Fronts of 64 < c <= kFrontWgMaxC rows, one workgroup of 256 threads per
// (front, matrix).  The front's lower triangle is packed in LDS (column t
// from t c - t (t - 1) / 2, rows t .. c - 1): A's entries are placed and the
// children's update blocks added (children in order; a child's entries land
// on distinct positions).  The first w columns are factored right-looking
// among themselves; L's block is written out and its rows below the
// diagonal block are copied, per 64-row tile, to a [k][64] layout; the update
// block is then the assembled values minus L21 L21^T, formed tile by tile on
// the matrix cores and written straight to U.

template <typename T>
__global__ __launch_bounds__(256) void k_front_wg(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int32_t *__restrict__ relmap, const int32_t *__restrict__ chlist,
    const int64_t *__restrict__ acolptr, const int32_t *__restrict__ aoff,
    const int64_t *__restrict__ avidx, const double *__restrict__ vals, int64_t ldv,
    T *__restrict__ L, int64_t Lsize, T *__restrict__ U, int64_t Usize,
    int32_t *__restrict__ info, int nblk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *F = reinterpret_cast<T *>(smem_raw);
    __shared__ int32_t rm[kFrontWgMaxC];  // relative map of the current child
    const int s = list[blockIdx.x];
    const int b = blockIdx.y;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w, m = d.m;
    L += int64_t(b) * Lsize;
    U += int64_t(b) * Usize;
    vals += int64_t(b) * ldv;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    auto cb = [c](int t) { return t * c - t * (t - 1) / 2; };  // packed offset of (t, t)
    const int ntri = c * (c + 1) / 2;
    const int wr = (w + 3) & ~3;                  // K of the products, padded
    const int nt = (m + kTile - 1) / kTile;       // 64-row tiles of the update block
    T *Lt = F + ntri;                             // [tile][k][64] rows of L21
    for (int q = tid; q < ntri; q += 256) F[q] = T(0);
    __syncthreads();
    const int64_t a0 = acolptr[d.first], a1 = acolptr[d.first + w];
    for (int64_t q = a0 + tid; q < a1; q += 256) {
        const int o = aoff[q];  // (column - first) c + row position
        const int j = o / c, i = o - j * c;
        F[cb(j) + i - j] = T(vals[avidx[q]]);
    }
    for (int q = d.chbeg; q < d.chend; q++) {
        const SnDesc cd = sn[chlist[q]];
        const int mc = cd.m;
        __syncthreads();  // the previous child's additions (and map reads) are done
        for (int i = tid; i < mc; i += 256) rm[i] = relmap[cd.relptr + i];
        __syncthreads();
        const T *Uc = U + cd.uoff;
        // the child's block as mc x mc column-major, upper part skipped;
        // four entries per thread in flight at once
        const int ne = mc * mc;
        int jc = tid / mc, ic = tid - jc * mc;
        for (int e0 = 0; e0 < ne; e0 += 4 * 256) {
            T v[4];
            int pos[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const bool ok = e0 + u * 256 + tid < ne && ic >= jc;
                v[u] = Uc[ok ? int64_t(jc) * mc + ic : 0];
                pos[u] = ok ? cb(rm[jc]) + rm[ic] - rm[jc] : -1;
                ic += 256;
                while (ic >= mc) { ic -= mc; jc++; }
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (pos[u] >= 0) F[pos[u]] += v[u];
        }
    }
    __syncthreads();
    // the first w columns, right-looking among themselves
    const int64_t infoidx = int64_t(b) * nblk + d.blk;
    for (int j = 0; j < w; j++) {
        const int cj = cb(j);
        T djj = F[cj];
        const bool bad = !(djj > T(0));
        if (bad) djj = T(1);
        const T ljj = dsqrt(djj), rinv = T(1) / ljj;
        __syncthreads();  // every thread has read the pivot
        if (tid == 0) {
            F[cj] = ljj;
            if (bad) atomicMin(info + infoidx, d.first - d.bcol0 + j + 1);
        }
        for (int i = j + 1 + tid; i < c; i += 256) F[cj + i - j] *= rinv;
        __syncthreads();
        for (int t = j + 1 + wv; t < w; t += 4) {
            const T ltj = F[cj + t - j];
            const int ct = cb(t);
            for (int i = t + lane; i < c; i += 64) F[ct + i - t] -= F[cj + i - j] * ltj;
        }
        __syncthreads();
    }
    // L's block out; rows w .. c - 1 of its columns into the tiles
    T *Ls = L + d.loff;
    for (int j = wv; j < w; j += 4) {
        const int cj = cb(j);
        for (int i = lane; i < c; i += 64) Ls[int64_t(j) * c + i] = i >= j ? F[cj + i - j] : T(0);
    }
    for (int e = tid; e < nt * wr * kTile; e += 256) {
        const int tile = e / (wr * kTile), r = e - tile * wr * kTile;
        const int k = r / kTile, i = tile * kTile + (r & (kTile - 1));
        Lt[e] = (k < w && i < m) ? F[cb(k) + w + i - k] : T(0);
    }
    __syncthreads();
    // update block: U[i][t] = F[w + i][w + t] - sum_k L21[i][k] L21[t][k]
    T *Us = U + d.uoff;
    for (int TI = 0; TI < nt; TI++)
        for (int TJ = 0; TJ <= TI; TJ++) {
            typename Mma<T>::acc_t acc[2][2];
            acc_zero<T>(acc);
            tile_mma(Lt + TJ * wr * kTile, Lt + TI * wr * kTile, wr, acc);
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int q = 0; q < 2; q++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        int jj, ii;
                        tile_pos<T>(a, q, r, jj, ii);
                        const int col = TJ * kTile + jj, row = TI * kTile + ii;
                        if (row < m && col <= row)
                            Us[int64_t(col) * m + row] = F[cb(w + col) + row - col] - acc[a][q][r];
                    }
        }
}

// Diagonal block of panel k of each large front: factor and invert (one
// workgroup per front and matrix).  The inverse also goes to the solve's
// inverted diagonal blocks when the supernode is solved by panels (the
// factor's 64-column panels are the solve's).
static_assert(kTile == kSolvePanel, "factor and solve panels coincide");
template <typename T>
__global__ __launch_bounds__(256) void k_potrf(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int k,
    T *__restrict__ L, int64_t Lsize, T *__restrict__ PI, int64_t pistride,
    T *__restrict__ Dinv, int64_t dsize, int32_t *__restrict__ info, int nblk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int s = list[blockIdx.x];
    const int b = blockIdx.y;
    const SnDesc d = sn[s];
    if (k >= d.w) return;
    const int kb = min(kTile, d.w - k);
    T *Lb = L + int64_t(b) * Lsize + d.loff;
    T *PIg = PI + int64_t(b) * pistride + int64_t(blockIdx.x) * kTile * kTile;
    // a panel-solved supernode keeps the inverse for the solves as well
    T *Dg = d.dinv >= 0 ? Dinv + int64_t(b) * dsize + d.dinv + int64_t(k / kTile) * kTile * kTile
                        : nullptr;
    wg_diag_factor(Lb, d.c, k, kb, lds, PIg, Dg, d.first - d.bcol0 + k,
                   info + int64_t(b) * nblk + d.blk);
}

// Panel rows below the diagonal block: X <- X L_kk^{-T} = X (L_kk^{-1})^T,
// a 64 x 64 x kb product per 64-row tile on the matrix cores.  A workgroup
// takes nt consecutive tiles (nt = kTrsmTiles when the launch has tiles
// enough to fill the chip that way, else 1): the inverse is staged once and
// the next tile's rows are in flight while the current one is multiplied.
constexpr int kTrsmTiles = 4;
constexpr int64_t kTrsmMultiMin = 512;  // tiles of a launch from which nt = kTrsmTiles
template <typename T>
__global__ __launch_bounds__(256) void k_trsm(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int k,
    T *__restrict__ L, int64_t Lsize, const T *__restrict__ PI, int64_t pistride, int nt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sX = reinterpret_cast<T *>(smem_raw);  // [t][r] panel rows
    T *sP = sX + kTile * kTile;               // [t][j] = inverse[j][t]
    const int s = list[blockIdx.y];
    const int b = blockIdx.z;
    const SnDesc d = sn[s];
    if (k >= d.w) return;
    const int kb = min(kTile, d.w - k);
    const int c = d.c;
    const int rfirst = k + kb + blockIdx.x * nt * kTile;
    if (rfirst >= c) return;
    T *Lb = L + int64_t(b) * Lsize + d.loff;
    const T *PIg = PI + int64_t(b) * pistride + int64_t(blockIdx.y) * kTile * kTile;
    const int tid = threadIdx.x;
    const int kbr = (kb + 3) & ~3;
    const int li = tid & 63, lt = tid >> 6;
    T rX[16];
    auto load_x = [&](int r0) {
        const bool rowok = r0 + li < c;
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int t = lt + 4 * q;
            rX[q] = (t < kb && rowok) ? Lb[int64_t(k + t) * c + r0 + li] : T(0);
        }
    };
    {
        T rP[16];
#pragma unroll
        for (int q = 0; q < 16; q++) rP[q] = PIg[(lt + 4 * q) * kTile + li];  // zero-padded
        load_x(rfirst);
#pragma unroll
        for (int q = 0; q < 16; q++) sP[(lt + 4 * q) * kTile + li] = rP[q];
    }
    for (int u = 0; u < nt; u++) {
        const int r0 = rfirst + u * kTile;
        if (r0 >= c) break;
        if (u > 0) __syncthreads();  // the previous tile's products are done
#pragma unroll
        for (int q = 0; q < 16; q++) sX[(lt + 4 * q) * kTile + li] = rX[q];
        __syncthreads();
        if (u + 1 < nt && r0 + kTile < c) load_x(r0 + kTile);
        typename Mma<T>::acc_t acc[2][2];
        acc_zero<T>(acc);
        tile_mma(sP, sX, kbr, acc);
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int q = 0; q < 2; q++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    int j, i;
                    tile_pos<T>(a, q, r, j, i);
                    if (j < kb && r0 + i < c) Lb[int64_t(k + j) * c + r0 + i] = acc[a][q][r];
                }
    }
}

// Update region of a trailing-update launch for one front: columns
// [cbeg, cend), rows [column, c), with the panel columns [k0, k0 + kw).
// Inner update (outer = 0): panel k of block K0 updates the rest of its
// block.  Outer update: the whole block updates everything beyond it
// (outer = 1), or only the next kBlock columns (2, the next block's panel
// chain needs them first) or only the columns after those (3, which can run
// beside that chain).
struct SyrkRegion {
    int k0, kw, cbeg, cend;
};
__host__ __device__ inline bool syrk_region(int w, int c, int K0, int k, int outer,
                                            SyrkRegion &r) {
    if (K0 >= w) return false;
    const int K1 = min(K0 + kBlock, w);
    if (outer) {
        r.k0 = K0;
        r.kw = K1 - K0;
        r.cbeg = outer == 3 ? K1 + kBlock : K1;
        r.cend = outer == 2 ? min(K1 + kBlock, c) : c;
    } else {
        if (k >= K1) return false;
        r.k0 = k;
        r.kw = min(kTile, w - k);
        r.cbeg = k + r.kw;
        r.cend = K1;
    }
    return r.cbeg < r.cend;
}
__host__ __device__ inline int64_t syrk_pairs(int c, const SyrkRegion &r) {
    const int64_t nct = (r.cend - r.cbeg + kTile - 1) / kTile;
    const int64_t nrt = (c - r.cbeg + kTile - 1) / kTile;
    return nct * nrt - nct * (nct - 1) / 2;
}

// Trailing update F[i, j] -= sum_t P[i, t] P[j, t] over the lower 64 x 64
// tiles of a region, P = panel columns after the TRSM, K in chunks of KC
// through LDS; MFMA 16x16x4 with four waves of 32 x 32.  The MFMA's row
// index runs over matrix columns so that each lane group writes 16
// consecutive rows of one column (column-major storage).  The tile's
// current entries are read at the start, so that their latency overlaps
// the products.  FP64 takes chunks of 32 (32 KiB of LDS, more workgroups
// per CU), FP32 chunks of 64.
template <typename T> struct SyrkKC { static constexpr int value = sizeof(T) == 8 ? 32 : 64; };
template <typename T>
__global__ __launch_bounds__(256) void k_syrk(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int K0, int k,
    int outer, T *__restrict__ L, int64_t Lsize, T *__restrict__ U, int64_t Usize) {
    constexpr int KC = SyrkKC<T>::value;
    constexpr int QN = KC / 4;                // chunk rows per thread and operand
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sI = reinterpret_cast<T *>(smem_raw);  // [t][i] panel rows of tile I
    T *sJ = sI + KC * kTile;                  // [t][j] panel rows of tile J
    const int s = list[blockIdx.y];
    const int b = blockIdx.z;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w, m = d.m;
    SyrkRegion R;
    if (!syrk_region(w, c, K0, k, outer, R)) return;
    const int64_t npairs = syrk_pairs(c, R);
    int64_t p = blockIdx.x;
    if (p >= npairs) return;
    const int nrt = (c - R.cbeg + kTile - 1) / kTile;
    int J = 0;
    while (p >= nrt - J) { p -= nrt - J; J++; }
    const int I = J + int(p);
    const int row0 = R.cbeg + I * kTile, col0 = R.cbeg + J * kTile;
    T *Lb = L + int64_t(b) * Lsize + d.loff;
    T *Ub = U + int64_t(b) * Usize + d.uoff;
    const int tid = threadIdx.x;
    const int li = tid & 63, lt = tid >> 6;
    const bool rowok = row0 + li < c, colok = col0 + li < R.cend;
    // panel chunk kc: thread (li, lt) holds rows row0 + li / col0 + li of
    // panel columns k0 + kc + lt + 4q, q < QN, in registers
    T rI[QN], rJ[QN];
    auto load_chunk = [&](int kc) {
        const int kb = min(KC, R.kw - kc);
#pragma unroll
        for (int q = 0; q < QN; q++) {
            const int t = lt + 4 * q;
            const T *pc = Lb + int64_t(R.k0 + kc + t) * c;
            rI[q] = (t < kb && rowok) ? pc[row0 + li] : T(0);
            rJ[q] = (t < kb && colok) ? pc[col0 + li] : T(0);
        }
    };
    typename Mma<T>::acc_t acc[2][2];
    acc_zero<T>(acc);
    load_chunk(0);
    // the tile's entries (absent ones read from the front's first entry)
    T cur[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int q = 0; q < 2; q++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                int jj, ii;
                tile_pos<T>(a, q, r, jj, ii);
                const int j = col0 + jj, i = row0 + ii;
                const bool ok = i < c && j < R.cend && i >= j;
                const T *src = ok ? front_col(Lb, Ub, c, w, m, j) + i : Lb;
                cur[a][q][r] = *src;
            }
    for (int kc = 0; kc < R.kw; kc += KC) {
        const int kb = min(KC, R.kw - kc);
        const int kbr = (kb + 3) & ~3;
        if (kc > 0) __syncthreads();  // the previous chunk's products are done
#pragma unroll
        for (int q = 0; q < QN; q++) {
            sI[(lt + 4 * q) * kTile + li] = rI[q];
            sJ[(lt + 4 * q) * kTile + li] = rJ[q];
        }
        __syncthreads();
        if (kc + KC < R.kw) load_chunk(kc + KC);  // in flight during the MFMAs
        tile_mma(sJ, sI, kbr, acc);
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int q = 0; q < 2; q++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                int jj, ii;
                tile_pos<T>(a, q, r, jj, ii);
                const int j = col0 + jj, i = row0 + ii;
                if (i < c && j < R.cend && i >= j) {
                    T *pcol = front_col(Lb, Ub, c, w, m, j);
                    pcol[i] = cur[a][q][r] - acc[a][q][r];
                }
            }
}

template <typename T>
void set_lds_limits(int big) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_syrk<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_trsm<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_front_wg<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_assemble_cols<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_potrf<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_trtri<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

// Flops of the partial factorization of the first w columns of a c-row
// front, Schur update included: sum_{j<w} (c - j)^2.
double front_flops(double c, double w) {
    double s = 0.0;
    for (int j = 0; j < int(w); j++) s += (c - j) * (c - j);
    return s;
}

// Factor schedule: launches of every level, built once per plan, with the
// algorithmic work of each launch (per matrix of a batch).
void build_schedule(const sc_plan *P, DevPlan *D) {
    D->fsched.clear();
    auto children_words = [&](const SnDesc &d) {
        double w = 0.0;
        for (int32_t q = d.chbeg; q < d.chend; q++) {
            const double mc = P->sn[P->chlist[q]].m;
            w += mc * (mc + 1) / 2;
        }
        return w;
    };
    auto a_entries = [&](const SnDesc &d) {
        return double(P->acolptr[d.first + d.w] - P->acolptr[d.first]);
    };
    // exact entries of L (amalgamation padding excluded) in column j with
    // row index below rlim, and in the w columns of a supernode
    auto exact_rows_below = [&](int32_t j, int64_t rlim) {
        const int64_t t = int64_t(std::upper_bound(P->ffirst.begin(), P->ffirst.end(), j) -
                                  P->ffirst.begin()) - 1;
        const int32_t *a = P->frows.data() + P->frowptr[t] + (j - P->ffirst[t]);
        const int32_t *b = P->frows.data() + P->frowptr[t + 1];
        return double(std::lower_bound(a, b, rlim) - a);
    };
    auto l_exact = [&](const SnDesc &d) {
        double c = 0.0;
        for (int32_t j = d.first; j < d.first + d.w; j++) c += double(P->colcount[j]);
        return c;
    };
    for (int32_t l = 0; l < P->nlevels; l++) {
        const int32_t s0 = P->lvl_small_ptr[l], s1 = P->lvl_small_ptr[l + 1];
        if (s1 > s0) {
            // k = the level's widest front; lds = its packed triangle (in
            // scalars) when it is too tall for registers
            const int cm = P->lvl_small_maxc[l];
            int wlds = 0;
            if (cm > kFrontRegMaxC)
                for (int32_t e = s0; e < s1; e++)
                    wlds = std::max(wlds, front_wg_lds(P->sn[P->lvl_small[e]].c,
                                                       P->sn[P->lvl_small[e]].w));
            FLaunch f{FLaunch::Small, l, cm, 0, 0, s0, s1 - s0, s1 - s0, wlds, 0.0, 0.0, 0.0};
            for (int32_t e = s0; e < s1; e++) {
                const SnDesc &d = P->sn[P->lvl_small[e]];
                f.flops += front_flops(d.c, d.w);
                f.words += children_words(d) + double(d.c) * d.w + double(d.m) * (d.m + 1) / 2;
                f.ibytes += a_entries(d) * 20.0;
                f.a_entries += a_entries(d);
                f.l_exact += l_exact(d);
            }
            D->fsched.push_back(f);
        }
        const int32_t b0 = P->lvl_big_ptr[l], b1 = P->lvl_big_ptr[l + 1];
        if (b1 == b0) continue;
        FLaunch fa{FLaunch::Assemble, l, 0, 0, 0, b0, b1 - b0, P->lvl_bigcols[l],
                   P->lvl_big_maxc[l], 0.0, 0.0, 0.0};
        for (int32_t e = b0; e < b1; e++) {
            const SnDesc &d = P->sn[P->lvl_big[e]];
            const double cw = children_words(d);
            fa.flops += cw;
            fa.words += cw + double(d.c) * d.w + double(d.m) * (d.m + 1) / 2;
            fa.ibytes += a_entries(d) * 20.0;
            fa.a_entries += a_entries(d);
        }
        D->fsched.push_back(fa);
        auto make_syrk = [&](int K0, int k, int outer) {
            FLaunch fs{FLaunch::Syrk, l, k, K0, outer, b0, b1 - b0, 0, 2 * kTile * kTile,
                       0.0, 0.0, 0.0};
            for (int32_t e = b0; e < b1; e++) {
                const SnDesc &d = P->sn[P->lvl_big[e]];
                SyrkRegion R;
                if (!syrk_region(d.w, d.c, K0, k, outer, R)) continue;
                fs.gridx = std::max(fs.gridx, syrk_pairs(d.c, R));
                const double ncol = R.cend - R.cbeg;
                const double entries = ncol * d.c - (double(R.cend - 1) * R.cend / 2.0 -
                                                     double(R.cbeg - 1) * R.cbeg / 2.0);
                fs.flops += 2.0 * R.kw * entries;
                fs.words += 2.0 * entries + double(d.c - R.cbeg) * R.kw;
            }
            return fs;
        };
        auto add_syrk = [&](int K0, int k, int outer) {
            const FLaunch fs = make_syrk(K0, k, outer);
            if (fs.gridx > 0) D->fsched.push_back(fs);
        };
        auto sync = [&](FLaunch::Kind kind) {
            D->fsched.push_back(FLaunch{kind, l, 0, 0, 0, b0, 0, 0, 0, 0.0, 0.0, 0.0});
        };
        // Lookahead: after the panel chain of block K0, the next block's
        // columns are updated on the main stream and the rest of the front on
        // the side stream, so the next block's chain runs beside that larger
        // update.  Updates of the same entries stay ordered: the side stream's
        // update of block K0 is joined before the main stream's update of
        // the following block (both write the columns two blocks on).
        bool pending = false;  // side-stream work not yet joined
        for (int32_t K0 = 0; K0 < P->lvl_big_maxw[l]; K0 += kBlock) {
            for (int32_t k = K0; k < std::min(K0 + kBlock, P->lvl_big_maxw[l]); k += kTile) {
                FLaunch fp{FLaunch::Potrf, l, k, 0, 0, b0, b1 - b0, b1 - b0, 0, 0.0, 0.0, 0.0};
                for (int32_t e = b0; e < b1; e++) {
                    const SnDesc &d = P->sn[P->lvl_big[e]];
                    if (k >= d.w) continue;
                    const int kb = std::min(kTile, d.w - k);
                    fp.flops += front_flops(kb, kb) + double(kb) * kb * kb / 3.0;
                    fp.words += double(kb) * (kb + 1) + double(kb) * kb;
                    for (int32_t j = d.first + k; j < d.first + k + kb; j++)
                        fp.l_exact += exact_rows_below(j, int64_t(d.first) + k + kb);
                }
                D->fsched.push_back(fp);
                FLaunch ft{FLaunch::Trsm, l, k, 0, 0, b0, b1 - b0, 0, 2 * kTile * kTile,
                           0.0, 0.0, 0.0};
                for (int32_t e = b0; e < b1; e++) {
                    const SnDesc &d = P->sn[P->lvl_big[e]];
                    if (k >= d.w) continue;
                    const int kb = std::min(kTile, d.w - k);
                    const int64_t nrem = d.c - k - kb;
                    ft.gridx = std::max<int64_t>(ft.gridx, (nrem + kTile - 1) / kTile);
                    ft.flops += 2.0 * double(nrem) * kb * kb;
                    ft.words += 2.0 * double(nrem) * kb + double(kb) * kb;
                    for (int32_t j = d.first + k; j < d.first + k + kb; j++)
                        ft.l_exact += double(P->colcount[j]) -
                                      exact_rows_below(j, int64_t(d.first) + k + kb);
                }
                if (ft.gridx > 0) D->fsched.push_back(ft);
                add_syrk(K0, k, 0);
            }
            FLaunch rest = make_syrk(K0, 0, 3);
            if (K0 + kBlock >= P->lvl_big_maxw[l] || rest.gridx == 0) {
                if (pending) sync(FLaunch::Join);
                pending = false;
                add_syrk(K0, 0, 1);
                continue;
            }
            sync(FLaunch::Fork);
            if (pending) sync(FLaunch::Join);
            add_syrk(K0, 0, 2);
            rest.side = 1;
            D->fsched.push_back(rest);
            pending = true;
        }
        if (pending) sync(FLaunch::Join);
    }
}

template <typename T>
hipError_t factor_impl(const sc_plan *P, sc_numeric *N, const double *vals,
                       int64_t ldv, hipStream_t st) {
    DevPlan *D = P->dev;
    T *L = static_cast<T *>(N->L);
    T *U = static_cast<T *>(N->U);
    T *PI = static_cast<T *>(N->pinv);
    const int64_t pistride = int64_t(P->max_lvl_big) * kTile * kTile;
    const int B = N->batch;
    {
        const int64_t ninfo = int64_t(B) * P->nblk;
        hipLaunchKernelGGL(k_fill_i32, dim3(unsigned((ninfo + 255) / 256)), dim3(256), 0, st,
                           N->info, ninfo, int32_t(INT_MAX));
    }
    for (const FLaunch &f : D->fsched)
        if (size_t(f.lds) * sizeof(T) > size_t(g_max_lds)) return hipErrorInvalidValue;
    Profiler &prof = N->prof;
    const double wsz = double(sizeof(T));
    // batch-interleaved objects: the copy of L to the interleaved layout runs
    // on a third stream as soon as the levels it covers are factored, beside
    // the levels above (it is joined before the factorization returns)
    const int32_t copy_lev = N->soa ? (N->xinv ? P->soa_copy_lev_x : P->soa_copy_lev) : -1;
    bool copy_forked = false;
    auto fork_copy = [&]() -> hipError_t {
        copy_forked = true;
        hipError_t e = hipEventRecord(N->ev_fork2, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(N->side2, N->ev_fork2, 0);
        if (e == hipSuccess) e = spchol_to_soa_run(P, N, N->side2);
        if (e == hipSuccess) e = hipEventRecord(N->ev_join2, N->side2);
        return e;
    };
    // the whole-block inverses of the small levels follow on the third
    // stream as soon as those levels are factored (after the copy when that
    // was forked first), beside the levels above
    const bool xs_side = N->side2 && N->xinv && !P->xs_list.empty() && P->xs_lev >= 0;
    bool xs_forked = false;
    auto fork_xs = [&]() -> hipError_t {
        xs_forked = true;
        hipError_t e = hipEventRecord(N->ev_fork2, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(N->side2, N->ev_fork2, 0);
        if (e == hipSuccess) e = spchol_dinv_run(P, N, N->side2, 1);
        if (e == hipSuccess) e = hipEventRecord(N->ev_join2, N->side2);
        return e;
    };
    for (const FLaunch &f : D->fsched) {
        if (copy_lev >= 0 && !copy_forked && f.level > copy_lev) {
            const hipError_t e = fork_copy();
            if (e != hipSuccess) return e;
        }
        if (xs_side && !xs_forked && f.level > P->xs_lev) {
            const hipError_t e = fork_xs();
            if (e != hipSuccess) return e;
        }
        if (f.kind == FLaunch::Fork || f.kind == FLaunch::Join) {
            const bool fork = f.kind == FLaunch::Fork;
            hipError_t e = hipEventRecord(fork ? N->ev_fork : N->ev_join, fork ? st : N->side);
            if (e == hipSuccess) e = hipStreamWaitEvent(fork ? N->side : st,
                                                       fork ? N->ev_fork : N->ev_join, 0);
            if (e != hipSuccess) return e;
            continue;
        }
        static const int kinds[] = {KK_SmallFront, KK_Assemble, KK_Potrf, KK_Trsm, KK_Syrk};
        const hipStream_t fst = f.side ? N->side : st;
        prof.begin(kinds[f.kind], f.flops * B, (f.words * wsz + f.ibytes) * B, fst,
                   (f.a_entries * 12.0 + f.l_exact * wsz) * B);
        switch (f.kind) {
        case FLaunch::Small: {
            const int cmax = f.k;
            if (cmax <= kFrontRegMaxC) {
                // fronts in registers, one segment of G lanes per (front,
                // matrix), 64 / G matrices per wave, four fronts per workgroup
#define SPCHOL_FRONT_REG(CM, G)                                                             \
    hipLaunchKernelGGL((k_front_reg<T, CM, G>),                                              \
                       dim3(unsigned((f.nlist + 3) / 4), unsigned((B + 64 / G - 1) / (64 / G))), \
                       dim3(256), 0, st, D->sn, D->lvl_small + f.list0, f.nlist, int(B),     \
                       D->relmap, D->chlist, D->acolptr, D->aoff, D->avidx, vals, ldv, L,    \
                       P->Lsize, U, P->Usize, N->info, P->nblk)
                if (cmax <= 16) SPCHOL_FRONT_REG(16, 16);
                else if (cmax <= 32) SPCHOL_FRONT_REG(32, 32);
                else if (cmax <= 48) SPCHOL_FRONT_REG(48, 64);
                else if (cmax <= 56) SPCHOL_FRONT_REG(56, 64);
                else SPCHOL_FRONT_REG(64, 64);
#undef SPCHOL_FRONT_REG
                break;
            }
            // wider fronts: one workgroup per (front, matrix), packed in LDS
            if (cmax > kFrontWgMaxC) return hipErrorInvalidValue;
            hipLaunchKernelGGL(k_front_wg<T>, dim3(unsigned(f.nlist), B), dim3(256),
                               size_t(f.lds) * sizeof(T), st, D->sn,
                               D->lvl_small + f.list0, D->relmap, D->chlist, D->acolptr, D->aoff,
                               D->avidx, vals, ldv, L, P->Lsize, U, P->Usize, N->info, P->nblk);
            break;
        }
        case FLaunch::Assemble: {
            const size_t per_lds = size_t(f.lds) * sizeof(T);
            const int per = int(std::max<size_t>(1, std::min<size_t>(4, g_max_lds / per_lds)));
            hipLaunchKernelGGL(k_assemble_cols<T>,
                               dim3(unsigned((f.gridx + per - 1) / per), B), dim3(64 * per),
                               per_lds * per, st, D->asm_col + P->lvl_colent_off[f.level],
                               D->asm_pc, int64_t(f.gridx), per, f.lds, D->relmap, D->aoff,
                               D->avidx, vals, ldv, L, P->Lsize, U, P->Usize);
            break;
        }
        case FLaunch::Potrf:
            hipLaunchKernelGGL(k_potrf<T>, dim3(unsigned(f.gridx), B), dim3(256),
                               size_t(kDiagLds) * sizeof(T), st,
                               D->sn, D->lvl_big + f.list0, f.k, L, P->Lsize, PI, pistride,
                               reinterpret_cast<T *>(N->dinv), P->dinv_size, N->info, P->nblk);
            break;
        case FLaunch::Trsm: {
            const int nt = f.gridx * f.nlist * B >= kTrsmMultiMin ? kTrsmTiles : 1;
            hipLaunchKernelGGL(k_trsm<T>, dim3(unsigned((f.gridx + nt - 1) / nt), f.nlist, B),
                               dim3(256), size_t(f.lds) * sizeof(T), st, D->sn,
                               D->lvl_big + f.list0, f.k, L, P->Lsize, PI, pistride, nt);
            break;
        }
        case FLaunch::Syrk:
            hipLaunchKernelGGL(k_syrk<T>, dim3(unsigned(f.gridx), f.nlist, B), dim3(256),
                               size_t(2 * SyrkKC<T>::value * kTile) * sizeof(T), fst, D->sn, D->lvl_big + f.list0,
                               f.K0, f.k, f.outer, L, P->Lsize, U, P->Usize);
            break;
        default:
            break;
        }
        prof.end(fst);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (copy_lev >= 0 && !copy_forked) e = fork_copy();
    if (e == hipSuccess && xs_side && !xs_forked) e = fork_xs();
    // inverted diagonal blocks for the solves (and the small levels' whole-
    // block inverses when they did not go to the third stream)
    if (e == hipSuccess) e = spchol_dinv_run(P, N, st, xs_forked ? 2 : 3);
    if (e == hipSuccess && N->xinv && !P->x_list.empty()) {
        // whole-block inverses from them
        prof.begin(KK_Dinv, 0.0, 0.0, st);
    hipLaunchKernelGGL(k_trtri<T>,
                       dim3(unsigned(N->batch), unsigned(P->x_nbmax), unsigned(P->x_list.size())),
                       dim3(256), size_t(kTile * kTile + kTile * kXPitch) * sizeof(T), st, D->sn,
                       D->x_list, D->xoff, L, P->Lsize, reinterpret_cast<const T *>(N->dinv),
                       P->dinv_size, static_cast<T *>(N->xinv), P->xsize);
        prof.end(st);
        e = hipGetLastError();
    }
    if (e == hipSuccess && (copy_forked || xs_forked)) e = hipStreamWaitEvent(st, N->ev_join2, 0);
    return e;
}

}  // namespace

void spchol_build_factor_schedule(const sc_plan *P, DevPlan *D) { build_schedule(P, D); }

int g_max_lds = 64 * 1024;

hipError_t spchol_kernels_init() {
    int dev = 0, lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    g_max_lds = lds;
    set_lds_limits<double>(lds);
    set_lds_limits<float>(lds);
    (void)hipGetLastError();  // an attribute the runtime refuses keeps the default
    return hipSuccess;
}

hipError_t spchol_factor_run(const sc_plan *P, sc_numeric *N, const double *vals,
                             int64_t ldv, hipStream_t st) {
    N->ls_ok = false;  // the interleaved copy of L is stale from here on
    if (N->dtype == SC_F64) return factor_impl<double>(P, N, vals, ldv, st);
    return factor_impl<float>(P, N, vals, ldv, st);
}
