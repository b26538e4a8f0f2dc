// Forward and backward triangular solves with the supernodal factor
// (gfx950).  y = L^{-1} P b by levels ascending, z = L^{-T} y by levels
// descending, x = P^T z.  The solves run in the precision of the stored
// factor (FP64, or FP32 vectors and arithmetic for an FP32 factor).
//
// Every supernode s owns a front vector FV_s of c_s entries: the first w_s
// hold its right-hand side, the last m_s its negated update vector
// u~_s = -sum over its subtree of L[R_s, k] y_k, which the parent pulls.
// Every value is written by exactly one workgroup, children are folded in a
// fixed order and reductions use fixed trees, so results are
// bit-reproducible and free of floating-point atomics.
//
// Small supernodes are solved by segments of a wave (row-major vectors) or
// one lane per matrix (batch-interleaved vectors).  Wide or tall ones are
// solved by 64-column panels with the inverted 64x64 diagonal blocks D_p:
//   forward  y_p = D_p^{-1} v_p, then the rows below the panel are updated;
//   backward partial dot products of chunks of rows below the panel, added
//            in chunk order, then D_p^{-T} is applied;
// either across many workgroups, one launch per step (few matrices), or by
// one workgroup per (supernode, matrix) walking all its panels (batches).
#include <algorithm>

#include "device.hpp"

namespace {

constexpr int kP = kSolvePanel;
constexpr int kMaxRhsPanel = 4;  // right-hand sides per pass of the panel gather

// p[idx] when ok, else 0, as an unconditional load of an in-bounds address
// (p[0] when !ok) and a select.  A load under a condition cannot be hoisted
// by the compiler and becomes a branch with its own wait for memory, which
// serializes the loads of a loop; every optional load below uses this.
template <typename V>
__device__ __forceinline__ V ldz(const V *p, int64_t idx, bool ok) {
    const V v = p[ok ? idx : 0];
    return ok ? v : V(0);
}

// A supernode's block of the interleaved L, read through a buffer resource:
// the block's address sits in a wave-uniform descriptor and a record's
// byte offset in a scalar register, the lane's slot is a constant vector
// offset, so a load needs no vector address arithmetic.  Offsets are
// 32-bit; a block of the interleaved layout (at most 512 x 64 entries x
// 64 lanes) is far below that.
constexpr int kBufWord3 = 0x00020000;  // raw buffer, gfx9-family data format
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename V>
struct SoaBlk {
    __amdgpu_buffer_rsrc_t r;
    unsigned voff;
    __device__ __forceinline__ SoaBlk(const V *base, unsigned lane)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<V *>(base), 0, 0x7fffffff, kBufWord3)),
          voff(lane * unsigned(sizeof(V))) {}
    // entry k, or entry 0 when !ok (no select; see Soa::ldc)
    __device__ __forceinline__ V ldc(int64_t k, bool ok) const {
        const unsigned so = ok ? unsigned(k) * unsigned(64 * sizeof(V)) : 0u;
        if constexpr (sizeof(V) == 4)
            return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, voff, so, 0));
        else
            return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, so, 0));
    }
    __device__ __forceinline__ V ldz(int64_t k, bool ok) const {
        const V v = ldc(k, ok);
        return ok ? v : V(0);
    }
    __device__ __forceinline__ void st(int64_t k, V v) const {
        const unsigned so = unsigned(k) * unsigned(64 * sizeof(V));
        if constexpr (sizeof(V) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, so, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, so, 0);
    }
};

// One group of an interleaved array: record k (64 scalars) holds entry k of
// 64 matrices, lane = matrix.  A lane's entry is reached from the record's
// wave-uniform address plus the lane's 32-bit byte offset, so an access
// takes a scalar base and no per-access vector address arithmetic.
template <typename V>
struct Soa {
    V *rec;         // wave-uniform: record 0 of the group
    unsigned lane;  // 0 .. 63
    __device__ __forceinline__ V &operator[](int64_t k) const { return (rec + k * 64)[lane]; }
    // entry k, or 0 when !ok (the load goes to record 0)
    __device__ __forceinline__ V ldz(int64_t k, bool ok) const {
        const V v = (rec + (ok ? k : 0) * 64)[lane];
        return ok ? v : V(0);
    }
    // entry k, or entry 0 when !ok (no select): for operands whose product
    // partner is exactly 0 or whose results are discarded when !ok
    __device__ __forceinline__ V ldc(int64_t k, bool ok) const {
        return (rec + (ok ? k : 0) * 64)[lane];
    }
};

// Inverse of every 64x64 diagonal block of the panel-solved supernodes that
// were factored as small fronts (the tiled factor writes the others):
// X = L_pp^{-1} by forward substitution, one lane per column of X kept in
// registers (loops fully unrolled), L_pp read from LDS as broadcasts.
template <typename T>
__global__ __launch_bounds__(64) void k_dinv(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const T *__restrict__ L, int64_t Lsize, T *__restrict__ Dinv, int64_t dsize) {
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
    // every load in flight at once: unconditional, at a clamped address
    T lv[kP];
#pragma unroll
    for (int t = 0; t < kP; t++) {
        const bool ok = lane < kb && t < kb;
        lv[t] = Lb[ok ? int64_t(c0 + t) * c + c0 + lane : 0];
    }
#pragma unroll
    for (int t = 0; t < kP; t++)
        Lp[lane * (kP + 1) + t] = (lane < kb && t < kb) ? double(lv[t]) : (lane == t ? 1.0 : 0.0);
    __syncthreads();
    double x[kP];
#pragma unroll
    for (int i = 0; i < kP; i++) {
        double sum = lane == i ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < i; t++) sum -= Lp[i * (kP + 1) + t] * x[t];
        x[i] = sum / Lp[i * (kP + 1) + i];
    }
    T *D = Dinv + int64_t(b) * dsize + d.dinv + int64_t(p) * kP * kP;
    __syncthreads();  // every read of Lp above precedes the transpose below
#pragma unroll
    for (int i = 0; i < kP; i++)  // column-major: D[col * 64 + i] = X[i][col], col = lane
        Lp[lane * (kP + 1) + i] = (lane < kb && i < kb) ? x[i] : 0.0;
    __syncthreads();
#pragma unroll 8
    for (int col = 0; col < kP; col++) D[col * kP + lane] = T(Lp[col * (kP + 1) + lane]);
}

// Whole-block inverse X = L11^{-1} of a supernode at most 64 wide (one wave
// per (matrix, supernode)), in the factor's precision with one lane per
// column of X (LDS and registers then allow nine waves per CU in FP32):
// column by column, x_i = b_i / L_ii and then b_t -= L_ti x_i for every
// later row t (independent updates, no serial sum chain); the reciprocals
// of the diagonal come first, one per lane.  Stored column-major with
// leading dimension w.
template <typename T>
__global__ __launch_bounds__(64) void k_xsmall(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int64_t *__restrict__ xoff, const T *__restrict__ L, int64_t Lsize,
    T *__restrict__ X, int64_t xsize) {
    __shared__ T Lc[kP * (kP + 1)];  // [t][i] = L[i][t]: column t of L11 at Lc + t (kP + 1)
    __shared__ T rv[kP];
    const int b = blockIdx.x;
    const int s = list[blockIdx.y];
    const SnDesc d = sn[s];
    const int w = d.w, c = d.c;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    const int lane = threadIdx.x;
    // every load in flight at once: unconditional, at a clamped address
    T lv[kP];
#pragma unroll
    for (int t = 0; t < kP; t++) {
        const bool ok = lane < w && t < w;
        lv[t] = Lb[ok ? int64_t(t) * c + lane : 0];
    }
#pragma unroll
    for (int t = 0; t < kP; t++)
        Lc[t * (kP + 1) + lane] = (lane < w && t < w) ? lv[t] : (lane == t ? T(1) : T(0));
    __syncthreads();
    rv[lane] = T(1) / Lc[lane * (kP + 1) + lane];
    __syncthreads();
    T x[kP];  // column `lane` of X; starts as column `lane` of the identity
#pragma unroll
    for (int i = 0; i < kP; i++) x[i] = lane == i ? T(1) : T(0);
#pragma unroll
    for (int i = 0; i < kP; i++) {
        x[i] *= rv[i];
#pragma unroll
        for (int t = i + 1; t < kP; t++) x[t] -= Lc[i * (kP + 1) + t] * x[i];
    }
    __syncthreads();  // every read of Lc above precedes the transpose below
#pragma unroll
    for (int i = 0; i < kP; i++) Lc[lane * (kP + 1) + i] = x[i];  // Lc[col][i] = X[i][col]
    __syncthreads();
    T *Xb = X + int64_t(b) * xsize + xoff[s];
    if (lane < w)
        for (int col = 0; col < w; col++) Xb[int64_t(col) * w + lane] = Lc[col * (kP + 1) + lane];
}

// Position of entry (matrix b, row, right-hand side r) in a solve vector
// set with `rows` rows per matrix.  Row-major per matrix (rows, then
// right-hand sides) or, batch-interleaved, groups of 64 matrices with the
// matrix index fastest, so that lane b of a wave reads consecutive words.
template <bool SOA>
__device__ __host__ inline int64_t vix(int b, int64_t row, int r, int64_t rows, int nrhs) {
    if constexpr (SOA)
        return ((int64_t(b >> 6) * rows + row) * nrhs + r) * 64 + (b & 63);
    else
        return (int64_t(b) * rows + row) * nrhs + r;
}

__device__ inline void wave_sync_solve() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of lane `src` of the calling lane's segment of G lanes (a segment
// lies inside one wave; G == 64 is the whole wave and src is then uniform).
template <int G>
__device__ inline double seg_bcast(double v, int src) {
    if constexpr (G == 64) {
        const long long u = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane(int(u & 0xffffffffll), src);
        const int hi = __builtin_amdgcn_readlane(int(u >> 32), src);
        return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                    (static_cast<unsigned int>(lo)));
    } else {
        return __shfl(v, src, G);
    }
}
template <int G>
__device__ inline float seg_bcast(float v, int src) {
    if constexpr (G == 64)
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
    else
        return __shfl(v, src, G);
}

// Ys[(b n + k) nrhs + r] = B[(b nrhs + r) ldb + perm[k]]: the permuted
// right-hand sides, interleaved so that one row of every right-hand side is
// one contiguous record.
template <typename T>
__global__ __launch_bounds__(256) void k_perm_in(
    const int32_t *__restrict__ perm, const double *__restrict__ B, int64_t ldb,
    T *__restrict__ Ys, int64_t n, int nrhs, const int32_t *__restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t src = perm[k];
    T *dst = Ys + (int64_t(b) * n + k) * nrhs;
    for (int r = 0; r < nrhs; r++) dst[r] = T(B[(int64_t(b) * nrhs + r) * ldb + src]);
}

// X[(b nrhs + r) ldb + i] = Ys[(b n + pinv[i]) nrhs + r]: writes in the
// caller's order (coalesced), reads gathered.
template <typename T>
__global__ __launch_bounds__(256) void k_perm_out(
    const int32_t *__restrict__ pinv, const T *__restrict__ Ys, double *__restrict__ X,
    int64_t ldb, int64_t n, int nrhs, const int32_t *__restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T *src = Ys + (int64_t(b) * n + pinv[i]) * nrhs;
    for (int r = 0; r < nrhs; r++) X[(int64_t(b) * nrhs + r) * ldb + i] = src[r];
}

// Front vectors of one level's supernodes (those not solved by panels):
// row q = rowptr_s + i of FV is the right-hand side (i < w, row y =
// first_s + i) plus the children's update entries (gather map, children in
// order), right-hand sides r0 .. r0 + NR - 1.  One thread per (row,
// matrix), so the short dependent chains of the gather overlap across the
// whole grid instead of stalling the solve kernels.
template <typename T, bool SOA, int NR>
__global__ __launch_bounds__(256) void k_gather(
    const int32_t *__restrict__ grow_q, const int32_t *__restrict__ grow_y, int nrow,
    const int32_t *__restrict__ gptr, const int32_t *__restrict__ gidx,
    const T *__restrict__ Ys, T *__restrict__ FV, int64_t n, int64_t fvsize,
    int nrhs, int r0, int batch, const int32_t *__restrict__ active) {
    int row, b;
    if constexpr (SOA) {
        row = blockIdx.x * 4 + (threadIdx.x >> 6);
        b = blockIdx.y * 64 + (threadIdx.x & 63);  // whole groups are allocated
        if (row >= nrow) return;
    } else {
        const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
        if (t >= int64_t(nrow) * batch) return;
        b = int(t / nrow);
        row = int(t - int64_t(b) * nrow);
        if (active && !active[b]) return;
    }
    const int q = grow_q[row], y = grow_y[row];
    const int g0 = gptr[q], g1 = gptr[q + 1];
    T a[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) a[r] = ldz(Ys, vix<SOA>(b, y, r0 + r, n, nrhs), y >= 0);
    for (int g = g0; g < g1; g++) {
        const int src = gidx[g];
#pragma unroll
        for (int r = 0; r < NR; r++) a[r] += FV[vix<SOA>(b, src, r0 + r, fvsize, nrhs)];
    }
#pragma unroll
    for (int r = 0; r < NR; r++) FV[vix<SOA>(b, q, r0 + r, fvsize, nrhs)] = a[r];
}

// Forward step of one level for the supernodes of one row class: a segment
// of G lanes per (supernode, matrix), lane i keeping rows i + G k (k < SL),
// right-hand sides r0 .. r0 + NR - 1.
//   front     row i of the front vector, gathered beforehand (k_gather);
//   triangle  the w x w diagonal block by columns: the owner of column j
//             scales by 1 / L_jj and its value is broadcast in the segment;
//   update    rows i >= w subtract L_ij y_j (ascending j), y read from LDS,
//             L's columns read by consecutive lanes (coalesced).
// Requires w <= G (w <= 64 for G == 64) and c <= G * SL.
template <typename T, int G, int SL, int NR, bool SOA>
__global__ __launch_bounds__(256) void k_fwd_seg(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int nlist, int nitems,
    int r0, const int32_t *__restrict__ gptr, const int32_t *__restrict__ gidx,
    const T *__restrict__ L, int64_t Lsize, T *__restrict__ Ys, T *__restrict__ FV,
    int64_t n, int64_t fvsize, int nrhs, const int32_t *__restrict__ active) {
    constexpr int NSEG = 256 / G;
    constexpr int WM = G < 64 ? G : 64;  // widest supernode of the class
    __shared__ T ys[NSEG][WM][NR];
    const int tid = threadIdx.x, seg = tid / G, li = tid % G;
    const int item = blockIdx.x * NSEG + seg;
    if (item >= nitems) return;
    const int b = item / nlist;
    if (active && !active[b]) return;
    const SnDesc d = sn[list[item - b * nlist]];
    const int c = d.c, w = d.w;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;

    T x[SL][NR];
#pragma unroll
    for (int k = 0; k < SL; k++) {
        const int i = li + G * k;
#pragma unroll
        for (int r = 0; r < NR; r++)
            x[k][r] = ldz(FV, vix<SOA>(b, d.rowptr + i, r0 + r, fvsize, nrhs), i < c);
    }
    // diagonal block (rows < w live in slot 0)
    const T dgl = T(ldz(Lb, int64_t(li) * c + li, li < w));
    const T rinv = li < w ? T(1) / dgl : T(0);
    // columns in chunks of 8, the next chunk's loads in flight while the
    // current one is processed; loads are unconditional from clamped
    // in-bounds addresses (column min(j, w - 1), row 0 for lanes past c) and
    // only the entries the update uses are read from them
    const int lrow = li < c ? li : 0;
    T lc[8];
#pragma unroll
    for (int jj = 0; jj < 8; jj++) lc[jj] = Lb[int64_t(min(jj, w - 1)) * c + lrow];
    for (int j0 = 0; j0 < w; j0 += 8) {
        T ln[8];
#pragma unroll
        for (int jj = 0; jj < 8; jj++)
            ln[jj] = Lb[int64_t(min(j0 + 8 + jj, w - 1)) * c + lrow];
#pragma unroll
        for (int jj = 0; jj < 8; jj++) {
            const int j = j0 + jj;
            if (j < w) {
                T y[NR];
#pragma unroll
                for (int r = 0; r < NR; r++) y[r] = seg_bcast<G>(x[0][r] * rinv, j);
                if (li == j) {
#pragma unroll
                    for (int r = 0; r < NR; r++) x[0][r] = y[r];
                } else if (li > j && li < w) {
                    const T l = T(lc[jj]);
#pragma unroll
                    for (int r = 0; r < NR; r++) x[0][r] -= l * y[r];
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < 8; jj++) lc[jj] = ln[jj];
    }
    if (li < w) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            ys[seg][li][r] = x[0][r];
            Ys[vix<SOA>(b, d.first + li, r0 + r, n, nrhs)] = x[0][r];
        }
    }
    wave_sync_solve();
    // rows below the diagonal block, JC columns of L in flight at once
    constexpr int JC = SL >= 8 ? 8 : 16;
    int irow[SL];  // the lane's rows below the block, clamped to row 0
#pragma unroll
    for (int k = 0; k < SL; k++) {
        const int i = li + G * k;
        irow[k] = i >= w && i < c ? i : 0;
    }
    for (int j0 = 0; j0 < w; j0 += JC) {
        T lc[JC][SL];
#pragma unroll
        for (int jj = 0; jj < JC; jj++) {
            const T *Lj = Lb + int64_t(min(j0 + jj, w - 1)) * c;
#pragma unroll
            for (int k = 0; k < SL; k++) lc[jj][k] = Lj[irow[k]];
        }
#pragma unroll
        for (int jj = 0; jj < JC; jj++) {
            const int j = j0 + jj;
            if (j < w) {
                T y[NR];
#pragma unroll
                for (int r = 0; r < NR; r++) y[r] = ys[seg][j][r];
#pragma unroll
                for (int k = 0; k < SL; k++) {
                    const int i = li + G * k;
                    if (i >= w && i < c) {
                        const T l = T(lc[jj][k]);
#pragma unroll
                        for (int r = 0; r < NR; r++) x[k][r] -= l * y[r];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < SL; k++) {
        const int i = li + G * k;
        if (i >= w && i < c) {
#pragma unroll
            for (int r = 0; r < NR; r++)
                FV[vix<SOA>(b, d.rowptr + i, r0 + r, fvsize, nrhs)] = x[k][r];
        }
    }
}

// Backward step of one level for the supernodes of one row class: a segment
// of G lanes per (supernode, matrix), lane j owning column j of the
// supernode (w <= G).  The rows of L's block are staged through LDS in
// chunks of kBwdRows (read from HBM by consecutive lanes), with the solved
// values x_i of those rows:
//   below     rows i >= w (ancestors' values) in blocks of kSoaRows rows:
//             acc_j -= (sum over the block, ascending i, of L_ij x_i);
//   diagonal  rows i = w-1 .. 0: the owner of column i finishes
//             x_i = acc_i / L_ii and broadcasts it; columns j < i subtract
//             L_ij x_i.
constexpr int kBwdRows = 16;
template <typename T, int G, int NR, bool SOA>
__global__ __launch_bounds__(256) void k_bwd_seg(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int nlist, int nitems,
    int r0, const int32_t *__restrict__ rows, const T *__restrict__ L, int64_t Lsize,
    T *__restrict__ Ys, int64_t n, int nrhs, const int32_t *__restrict__ active) {
    constexpr int NSEG = 256 / G;
    constexpr int NG = G / kBwdRows;  // column groups of the staging
    __shared__ T Ls[NSEG][kBwdRows][G + 1];
    __shared__ T xs[NSEG][kBwdRows][NR];
    const int tid = threadIdx.x, seg = tid / G, li = tid % G;
    const int item = blockIdx.x * NSEG + seg;
    if (item >= nitems) return;
    const int b = item / nlist;
    if (active && !active[b]) return;
    const SnDesc d = sn[list[item - b * nlist]];
    const int c = d.c, w = d.w;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    const int32_t *R = rows + d.rowptr;
    const int sr = li % kBwdRows, sg = li / kBwdRows;  // staging: row, column group

    T acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++)
        acc[r] = ldz(Ys, vix<SOA>(b, d.first + li, r0 + r, n, nrhs), li < w);
    const T rinv = li < w ? T(1) / T(Lb[li < w ? int64_t(li) * c + li : 0]) : T(0);
    // rows below in blocks of kSoaRows: each block's sum (ascending rows)
    // is formed on its own and then subtracted, the same order as the
    // batch-interleaved kernels, so both layouts give identical bits.  The
    // next block's entries of L and values x are in flight while the
    // current block is summed, and the row indices one block earlier still.
    static_assert(kSoaRows == kBwdRows, "one staging round per row block");
    auto load_l = [&](int i0, T (&v)[kBwdRows]) {
        const int i = i0 + sr;
#pragma unroll
        for (int q = 0; q < kBwdRows; q++) {
            const int j = sg + NG * q;
            v[q] = ldz(Lb, int64_t(j) * c + i, i < c && j < w);
        }
    };
    auto load_r = [&](int i0) { return ldz(R, i0 + sr, sg == 0 && i0 + sr < c); };
    auto load_x = [&](int i0, int ri, T (&xv)[NR]) {
        const bool xo = sg == 0 && i0 + sr < c;
#pragma unroll
        for (int r = 0; r < NR; r++) xv[r] = ldz(Ys, vix<SOA>(b, ri, r0 + r, n, nrhs), xo);
    };
    T vc[kBwdRows], xc[NR];
    int rnext = 0;
    if (w < c) {
        load_l(w, vc);
        load_x(w, load_r(w), xc);
        rnext = load_r(w + kBwdRows);
    }
    for (int rb = w; rb < c; rb += kBwdRows) {
        T vn[kBwdRows], xn[NR];
        const bool more = rb + kBwdRows < c;
        if (more) {
            load_l(rb + kBwdRows, vn);
            load_x(rb + kBwdRows, rnext, xn);
            rnext = load_r(rb + 2 * kBwdRows);
        }
#pragma unroll
        for (int q = 0; q < kBwdRows; q++) {
            const int j = sg + NG * q;
            if (j < w) Ls[seg][sr][j] = vc[q];
        }
        if (sg == 0 && rb + sr < c) {
#pragma unroll
            for (int r = 0; r < NR; r++) xs[seg][sr][r] = xc[r];
        }
        wave_sync_solve();
        T p[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) p[r] = T(0);
        const int nr = min(kBwdRows, c - rb);
        if (li < w) {
            for (int t = 0; t < nr; t++) {
                const T l = T(Ls[seg][t][li]);
#pragma unroll
                for (int r = 0; r < NR; r++) p[r] += l * xs[seg][t][r];
            }
        }
        wave_sync_solve();
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] -= p[r];
        if (more) {
#pragma unroll
            for (int q = 0; q < kBwdRows; q++) vc[q] = vn[q];
#pragma unroll
            for (int r = 0; r < NR; r++) xc[r] = xn[r];
        }
    }
    for (int i1 = w; i1 > 0; i1 -= kBwdRows) {
        const int i0 = max(0, i1 - kBwdRows);
        const int i = i0 + sr;
        {
            T v[kBwdRows];
#pragma unroll
            for (int q = 0; q < kBwdRows; q++) {
                const int j = sg + NG * q;
                v[q] = ldz(Lb, int64_t(j) * c + i, i < i1 && j < i);
            }
#pragma unroll
            for (int q = 0; q < kBwdRows; q++) {
                const int j = sg + NG * q;
                if (i < i1 && j < i) Ls[seg][sr][j] = v[q];
            }
        }
        wave_sync_solve();
        for (int t = i1 - 1; t >= i0; t--) {
            T xv[NR];
#pragma unroll
            for (int r = 0; r < NR; r++) xv[r] = seg_bcast<G>(acc[r] * rinv, t);
            if (li == t) {
#pragma unroll
                for (int r = 0; r < NR; r++) acc[r] = xv[r];
            } else if (li < t) {
                const T l = T(Ls[seg][t - i0][li]);
#pragma unroll
                for (int r = 0; r < NR; r++) acc[r] -= l * xv[r];
            }
        }
        wave_sync_solve();
    }
    if (li < w) {
#pragma unroll
        for (int r = 0; r < NR; r++) Ys[vix<SOA>(b, d.first + li, r0 + r, n, nrhs)] = acc[r];
    }
}

// Front vectors of the panel-solved supernodes of a level, then y_0 of
// their first panel.  Row i of FV_s is the right-hand side (i < w) plus the
// children's update entries (gather map, children in order); y_0 =
// D_0^{-1} v_0 with the zero-padded inverse block D_0 (column-major).
// Item = (supernode, matrix); 256 threads; right-hand sides in blocks of
// kMaxRhsPanel.
template <typename T, bool SOA>
__global__ __launch_bounds__(256) void k_pan_gather(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int32_t *__restrict__ gptr, const int32_t *__restrict__ gidx,
    const T *__restrict__ Dinv, int64_t dsize, T *__restrict__ Ys,
    T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs,
    const int32_t *__restrict__ active) {
    __shared__ T v0[kP][kMaxRhsPanel];
    const int s = list[blockIdx.x];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int kb = min(kP, d.w);
    const T *D = Dinv + int64_t(b) * dsize + d.dinv;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPanel) {
        const int nr = min(kMaxRhsPanel, nrhs - r0);
        for (int i = threadIdx.x; i < d.c; i += blockDim.x) {
            const int g0 = gptr[d.rowptr + i], g1 = gptr[d.rowptr + i + 1];
            for (int r = 0; r < nr; r++) {
                T a = ldz(Ys, vix<SOA>(b, d.first + i, r0 + r, n, nrhs), i < d.w);
                for (int g = g0; g < g1; g++) a += FV[vix<SOA>(b, gidx[g], r0 + r, fvsize, nrhs)];
                FV[vix<SOA>(b, d.rowptr + i, r0 + r, fvsize, nrhs)] = a;
                if (i < kP) v0[i][r] = a;
            }
        }
        __syncthreads();
        const int t = threadIdx.x;
        if (t < kb) {
            T y[kMaxRhsPanel] = {};
#pragma unroll 16
            for (int i = 0; i < kb; i++) {
                const T di = D[int64_t(i) * kP + t];
#pragma unroll
                for (int r = 0; r < kMaxRhsPanel; r++)
                    if (r < nr) y[r] += di * v0[i][r];
            }
            for (int r = 0; r < nr; r++) Ys[vix<SOA>(b, d.first + t, r0 + r, n, nrhs)] = y[r];
        }
        __syncthreads();
    }
}

// Forward panel p of panel-solved supernodes, right-hand sides r0 ..
// r0 + NR - 1: workgroup t updates rows [c0 + kb + 64 t, +64) of FV_s with
// y_p (stored by the previous step).  Workgroup 0 covers the rows of panel
// p + 1 when there is one; it then also forms y_{p+1} = D_{p+1}^{-1} v_{p+1}
// (every contribution to v_{p+1} is in once this update is done).
template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_fwd_panel(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int p, int r0,
    const T *__restrict__ L, int64_t Lsize, const T *__restrict__ Dinv,
    int64_t dsize, T *__restrict__ Ys, T *__restrict__ FV, int64_t n,
    int64_t fvsize, int nrhs, const int32_t *__restrict__ active) {
    __shared__ T yv[kP][NR];
    __shared__ T vn[kP][NR];
    const int s = list[blockIdx.y];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c0 = p * kP;
    if (c0 >= d.w) return;
    const int kb = min(kP, d.w - c0);
    const int c = d.c;
    const int tile = blockIdx.x;
    const int rt = c0 + kb + tile * kP;
    if (rt >= c) return;
    const int lane = threadIdx.x;
#pragma unroll
    for (int r = 0; r < NR; r++)
        yv[lane][r] = ldz(Ys, vix<SOA>(b, d.first + c0 + lane, r0 + r, n, nrhs), lane < kb);
    __syncthreads();
    const int row = rt + lane;
    const bool rok = row < c;
    const int rowc = rok ? row : rt;  // rows past the front read row rt (in bounds)
    T v[NR];
    {
        const T *Lr = L + int64_t(b) * Lsize + d.loff + int64_t(c0) * c + rowc;
#pragma unroll
        for (int r = 0; r < NR; r++) v[r] = FV[vix<SOA>(b, d.rowptr + rowc, r0 + r, fvsize, nrhs)];
        if (kb == kP) {  // a full panel: the row's 64 entries in flight at once
            T l[kP];
#pragma unroll
            for (int t = 0; t < kP; t++) l[t] = Lr[int64_t(t) * c];
#pragma unroll
            for (int t = 0; t < kP; t++)
#pragma unroll
                for (int r = 0; r < NR; r++) v[r] -= l[t] * yv[t][r];
        } else {
#pragma unroll 8
            for (int t = 0; t < kb; t++) {
                const T l = T(Lr[int64_t(t) * c]);
#pragma unroll
                for (int r = 0; r < NR; r++) v[r] -= l * yv[t][r];
            }
        }
        if (rok) {
#pragma unroll
            for (int r = 0; r < NR; r++) FV[vix<SOA>(b, d.rowptr + row, r0 + r, fvsize, nrhs)] = v[r];
        }
    }
    const int c1 = c0 + kP;  // next panel
    if (tile != 0 || c1 >= d.w) return;
    const int kb1 = min(kP, d.w - c1);
#pragma unroll
    for (int r = 0; r < NR; r++) vn[lane][r] = lane < kb1 ? v[r] : T(0);
    __syncthreads();
    if (lane < kb1) {
        const T *D = Dinv + int64_t(b) * dsize + d.dinv + int64_t(p + 1) * kP * kP;
        T y[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) y[r] = T(0);
        T dv[kP];  // column `lane` of the block's inverse, all in flight
#pragma unroll
        for (int i = 0; i < kP; i++) dv[i] = D[int64_t(i) * kP + lane];
#pragma unroll
        for (int i = 0; i < kP; i++)
#pragma unroll
            for (int r = 0; r < NR; r++) y[r] += dv[i] * vn[i][r];
#pragma unroll
        for (int r = 0; r < NR; r++) Ys[vix<SOA>(b, d.first + c1 + lane, r0 + r, n, nrhs)] = y[r];
    }
}

// Backward panel p, step 1: partial sums of L[i, c0 + t] x_i over a chunk of
// kSolveChunk rows below the panel, right-hand sides r0 .. r0 + NR - 1.
// Wave g takes rows [64 g, +64) of the chunk in blocks of 16 staged through
// LDS (L read by consecutive lanes along its columns), lane t owns column
// c0 + t; the four waves' sums are added in wave order.
template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(256) void k_bwd_pan_part(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int p, int r0,
    const int32_t *__restrict__ rows, const T *__restrict__ L, int64_t Lsize,
    const T *__restrict__ Ys, int64_t n, T *__restrict__ PART, int64_t psize,
    int nrhs, const int32_t *__restrict__ active) {
    constexpr int RB = 16;
    __shared__ T Ls[4][RB][kP + 1];
    __shared__ T xs[4][RB][NR];
    __shared__ T red[4][kP][NR];
    const int s = list[blockIdx.y];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c0 = p * kP;
    if (c0 >= d.w) return;
    const int kb = min(kP, d.w - c0);
    const int c = d.c;
    const int rbeg = c0 + kb;
    const int chunk = blockIdx.x;
    const int rb = rbeg + chunk * kSolveChunk;
    if (rb >= c) return;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int sr = lane & (RB - 1), sg = lane >> 4;  // staging: row, column group
    const T *Lb = L + int64_t(b) * Lsize + d.loff + int64_t(c0) * c;
    const int32_t *R = rows + d.rowptr;
    T acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = T(0);
    const int w0 = rb + 64 * wv, w1 = min(c, w0 + 64);
    // every row block of this wave's 64 rows in flight at once (entries of
    // L, then the rows' positions and values x)
    constexpr int NB = 64 / RB;
    T lv[NB][16];
    T xq[NB][NR];
#pragma unroll
    for (int k = 0; k < NB; k++) {
        const int i = w0 + k * RB + sr;
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int t = sg + 4 * q;
            lv[k][q] = ldz(Lb, int64_t(t) * c + i, i < w1 && t < kb);
        }
    }
#pragma unroll
    for (int k = 0; k < NB; k++) {
        const int i = w0 + k * RB + sr;
        const bool xo = sg == 0 && i < w1;
        const int64_t pos = i < d.w ? d.first + i : ldz(R, i, xo && i >= d.w);
#pragma unroll
        for (int r = 0; r < NR; r++) xq[k][r] = ldz(Ys, vix<SOA>(b, pos, r0 + r, n, nrhs), xo);
    }
#pragma unroll
    for (int k = 0; k < NB; k++) {
        const int i0 = w0 + k * RB;
        const int i = i0 + sr;
        if (i0 < w1) {
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int t = sg + 4 * q;
                if (i < w1 && t < kb) Ls[wv][sr][t] = lv[k][q];
            }
            if (sg == 0 && i < w1) {
#pragma unroll
                for (int r = 0; r < NR; r++) xs[wv][sr][r] = xq[k][r];
            }
            wave_sync_solve();  // each wave stages and reads its own rows
            const int nr = min(RB, w1 - i0);
            if (lane < kb) {
                for (int q = 0; q < nr; q++) {
                    const T l = T(Ls[wv][q][lane]);
#pragma unroll
                    for (int r = 0; r < NR; r++) acc[r] += l * xs[wv][q][r];
                }
            }
            wave_sync_solve();
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) red[wv][lane][r] = acc[r];
    __syncthreads();
    if (wv == 0 && lane < kb) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const T v = ((red[0][lane][r] + red[1][lane][r]) + red[2][lane][r]) + red[3][lane][r];
            PART[vix<SOA>(b, d.part + int64_t(chunk) * kP + lane, r0 + r, psize, nrhs)] = v;
        }
    }
}

// Backward panel p, step 2: x_p = D_p^T (y_p - sum of the chunks' partial
// sums, in chunk order), right-hand sides r0 .. r0 + NR - 1.  Item =
// (supernode, matrix); one wave, lane t owns column c0 + t.
template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_bwd_pan_fin(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int p, int r0,
    const T *__restrict__ Dinv, int64_t dsize, T *__restrict__ Ys, int64_t n,
    const T *__restrict__ PART, int64_t psize, int nrhs,
    const int32_t *__restrict__ active) {
    __shared__ T Dt[kP * (kP + 1)];
    __shared__ T rhs[kP][NR];
    const int s = list[blockIdx.x];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c0 = p * kP;
    if (c0 >= d.w) return;
    const int kb = min(kP, d.w - c0);
    const int rbeg = c0 + kb;
    const int nch = (d.c - rbeg + kSolveChunk - 1) / kSolveChunk;
    const int t = threadIdx.x;
    // the inverse block, coalesced into LDS: Dt[j][i] = D[j * 64 + i]
    const T *Dp = Dinv + int64_t(b) * dsize + d.dinv + int64_t(p) * kP * kP;
    {
        T v[kP];  // the whole block in flight at once, 64 loads per thread
#pragma unroll
        for (int q = 0; q < kP; q++) v[q] = Dp[q * 64 + t];
#pragma unroll
        for (int q = 0; q < kP; q++) Dt[q * (kP + 1) + t] = v[q];
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        // the chunks' partial sums 16 at a time, all loads of a group in
        // flight before they are added (in chunk order)
        // (clamped in-bounds addresses; only the chunks that exist are added)
        const int tc = t < kb ? t : 0;
        T s0 = T(0);
        for (int q0 = 0; q0 < nch; q0 += 16) {
            T pv[16];
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int q = q0 + u < nch ? q0 + u : nch - 1;
                pv[u] = PART[vix<SOA>(b, d.part + int64_t(q) * kP + tc, r0 + r, psize, nrhs)];
            }
#pragma unroll
            for (int u = 0; u < 16; u++)
                if (q0 + u < nch) s0 += pv[u];
        }
        rhs[t][r] = t < kb ? ldz(Ys, vix<SOA>(b, d.first + c0 + t, r0 + r, n, nrhs), t < kb) - s0
                           : T(0);
    }
    __syncthreads();
    if (t < kb) {
        // x_t = sum_i (L_pp^{-1})[i][t] rhs_i; column t of the inverse is Dt[t][.]
        T xt[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) xt[r] = T(0);
#pragma unroll 8
        for (int i = 0; i < kb; i++) {
            const T dti = Dt[t * (kP + 1) + i];
#pragma unroll
            for (int r = 0; r < NR; r++) xt[r] += dti * rhs[i][r];
        }
#pragma unroll
        for (int r = 0; r < NR; r++) Ys[vix<SOA>(b, d.first + c0 + t, r0 + r, n, nrhs)] = xt[r];
    }
}

// ---------------------------------------------------------------------------
// Panel-solved supernodes with one workgroup per (supernode, matrix): the
// whole front vector lives in LDS and the workgroup walks the 64-column
// panels itself, so a level takes one launch per direction instead of a
// few per panel.  The arithmetic is that of the multi-launch panel kernels
// above, operation for operation (gather with the children in order,
// D_p^{-1} products by ascending index, row updates by ascending column,
// backward partial sums by chunks of kSolveChunk rows split over four
// waves and added in wave order, then in chunk order), so both give the
// same bits.  Used for batches, where (supernodes x matrices) workgroups
// fill the chip; a front of c rows needs c * NR scalars of LDS.
constexpr int kSnThreads = 512;   // backward: eight waves, two row chunks at a time
constexpr int kSnWaves = kSnThreads / 64;
constexpr int kSnRB = 16;         // rows per staging block of the backward sums
// forward: 512 threads in FP32 (more rows of a panel at once), 256 in FP64
// (the row's 64 entries of L in flight take twice the registers)
template <typename T> struct SnThreadsF { static constexpr int value = sizeof(T) == 4 ? 512 : 256; };

// Forward: every thread holds a share of the next panel's inverse block in
// flight while the current panel is processed.
template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(SnThreadsF<T>::value) void k_fwd_sn(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int r0,
    const int32_t *__restrict__ gptr, const int32_t *__restrict__ gidx,
    const T *__restrict__ L, int64_t Lsize, const T *__restrict__ Dinv, int64_t dsize,
    T *__restrict__ Ys, T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs,
    const int32_t *__restrict__ active) {
    constexpr int NTH = SnThreadsF<T>::value;
    constexpr int DPT = kP * kP / NTH;  // inverse-block entries per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *Ds = reinterpret_cast<T *>(smem_raw);               // D_p, as stored
    T(*v)[NR] = reinterpret_cast<T(*)[NR]>(Ds + kP * kP);  // front vector, c rows
    const int s = list[blockIdx.x];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w;
    const int tid = threadIdx.x;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    const T *Db = Dinv + int64_t(b) * dsize + d.dinv;
    T dreg[DPT];
#pragma unroll
    for (int q = 0; q < DPT; q++) dreg[q] = Db[q * NTH + tid];
    for (int i = tid; i < c; i += NTH) {
        const int g0 = gptr[d.rowptr + i], g1 = gptr[d.rowptr + i + 1];
#pragma unroll
        for (int r = 0; r < NR; r++) {
            T a = ldz(Ys, vix<SOA>(b, d.first + i, r0 + r, n, nrhs), i < w);
            for (int g = g0; g < g1; g++) a += FV[vix<SOA>(b, gidx[g], r0 + r, fvsize, nrhs)];
            v[i][r] = a;
        }
    }
    for (int c0 = 0; c0 < w; c0 += kP) {
        const int kb = min(kP, w - c0);
#pragma unroll
        for (int q = 0; q < DPT; q++) Ds[q * NTH + tid] = dreg[q];
        __syncthreads();  // D_p staged, v complete
        if (c0 + kP < w) {
            const T *Dn = Db + int64_t(c0 / kP + 1) * kP * kP;
#pragma unroll
            for (int q = 0; q < DPT; q++) dreg[q] = Dn[q * NTH + tid];
        }
        // y_p = D_p^{-1} v_p (the first panel sums over its kb rows, later
        // ones over all 64 with zeros past kb, as the panel kernels do)
        T y[NR];
        if (tid < kb) {
            const int ni = c0 == 0 ? kb : kP;
#pragma unroll
            for (int r = 0; r < NR; r++) y[r] = T(0);
#pragma unroll 16
            for (int i = 0; i < ni; i++) {
                const T di = Ds[i * kP + tid];
#pragma unroll
                for (int r = 0; r < NR; r++) y[r] += di * (i < kb ? v[c0 + i][r] : T(0));
            }
        }
        __syncthreads();
        if (tid < kb) {
#pragma unroll
            for (int r = 0; r < NR; r++) {
                v[c0 + tid][r] = y[r];
                Ys[vix<SOA>(b, d.first + c0 + tid, r0 + r, n, nrhs)] = y[r];
            }
        }
        __syncthreads();
        // rows below the panel, products by ascending column; a full panel
        // has the row's 64 entries of L in flight before the products
        for (int i = c0 + kb + tid; i < c; i += NTH) {
            const T *Lr = Lb + int64_t(c0) * c + i;
            T a[NR];
#pragma unroll
            for (int r = 0; r < NR; r++) a[r] = v[i][r];
            if (kb == kP) {
                T l[kP];
#pragma unroll
                for (int t = 0; t < kP; t++) l[t] = Lr[int64_t(t) * c];
#pragma unroll
                for (int t = 0; t < kP; t++)
#pragma unroll
                    for (int r = 0; r < NR; r++) a[r] -= l[t] * v[c0 + t][r];
            } else {
#pragma unroll 16
                for (int t = 0; t < kb; t++) {
                    const T l = Lr[int64_t(t) * c];
#pragma unroll
                    for (int r = 0; r < NR; r++) a[r] -= l * v[c0 + t][r];
                }
            }
#pragma unroll
            for (int r = 0; r < NR; r++) v[i][r] = a[r];
        }
        __syncthreads();
    }
    for (int i = w + tid; i < c; i += NTH) {
#pragma unroll
        for (int r = 0; r < NR; r++) FV[vix<SOA>(b, d.rowptr + i, r0 + r, fvsize, nrhs)] = v[i][r];
    }
}

template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(kSnThreads) void k_bwd_sn(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int r0,
    const int32_t *__restrict__ rows, const T *__restrict__ L, int64_t Lsize,
    const T *__restrict__ Dinv, int64_t dsize, T *__restrict__ Ys, int64_t n, int nrhs,
    const int32_t *__restrict__ active) {
    constexpr int RB = kSnRB;
    constexpr int NB = 64 / RB;  // staging blocks per wave's 64 rows
    static_assert(kSnWaves * RB >= kP && kSolveChunk == 4 * 64, "LDS sharing and chunk split");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T stage[kSnWaves * RB * (kP + 1)];  // rows of L while summing, then D_p
    __shared__ T red[kSnWaves][kP][NR];
    __shared__ T rhs[kP][NR];
    T(*Ls)[RB][kP + 1] = reinterpret_cast<T(*)[RB][kP + 1]>(stage);
    T *Dt = stage;
    T(*xs)[NR] = reinterpret_cast<T(*)[NR]>(smem_raw);  // x of the front's rows
    const int s = list[blockIdx.x];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int sr = lane & (RB - 1), sg = lane >> 4;  // staging: row, column group
    const int32_t *R = rows + d.rowptr;
    for (int i = w + tid; i < c; i += kSnThreads) {
        const int ri = R[i];
#pragma unroll
        for (int r = 0; r < NR; r++) xs[i][r] = Ys[vix<SOA>(b, ri, r0 + r, n, nrhs)];
    }
    __syncthreads();
    const T *Lsn = L + int64_t(b) * Lsize + d.loff;
    const T *Db = Dinv + int64_t(b) * dsize + d.dinv;
    for (int c0 = ((w - 1) / kP) * kP; c0 >= 0; c0 -= kP) {
        const int kb = min(kP, w - c0);
        const int rbeg = c0 + kb;
        const T *Lb = Lsn + int64_t(c0) * c;
        // partial sums of L[i, c0 + t] x_i by chunks of kSolveChunk rows:
        // waves 4h .. 4h + 3 take chunk 2k + h, 64 rows each, the four
        // waves' sums are added in wave order and the chunks in order
        // the inverse block and y_p, in flight with the first rows of L
        const T *Dp = Db + int64_t(c0 / kP) * kP * kP;
        constexpr int DPT = kP * kP / kSnThreads;
        T dreg[DPT];
#pragma unroll
        for (int q = 0; q < DPT; q++) dreg[q] = Dp[q * kSnThreads + tid];
        T yp[NR];
#pragma unroll
        for (int r = 0; r < NR; r++)
            yp[r] = ldz(Ys, vix<SOA>(b, d.first + c0 + lane, r0 + r, n, nrhs), wv == 0 && lane < kb);
        T s0[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) s0[r] = T(0);
        for (int rb2 = rbeg; rb2 < c; rb2 += 2 * kSolveChunk) {
            const int h = wv >> 2;
            const int w0 = rb2 + h * kSolveChunk + 64 * (wv & 3), w1 = min(c, w0 + 64);
            T acc[NR];
#pragma unroll
            for (int r = 0; r < NR; r++) acc[r] = T(0);
            // every row block of this wave's 64 rows in flight at once
            T lv[NB][16];
#pragma unroll
            for (int k = 0; k < NB; k++) {
                const int i = w0 + k * RB + sr;
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    const int t = sg + 4 * q;
                    lv[k][q] = ldz(Lb, int64_t(t) * c + i, i < w1 && t < kb);
                }
            }
#pragma unroll
            for (int k = 0; k < NB; k++) {
                const int i0 = w0 + k * RB;
                const int i = i0 + sr;
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    const int t = sg + 4 * q;
                    if (i < w1 && t < kb) Ls[wv][sr][t] = lv[k][q];
                }
                wave_sync_solve();  // each wave stages and reads its own rows
                const int nr = min(RB, w1 - i0);
                if (lane < kb) {
                    for (int q = 0; q < nr; q++) {
                        const T l = Ls[wv][q][lane];
#pragma unroll
                        for (int r = 0; r < NR; r++) acc[r] += l * xs[i0 + q][r];
                    }
                }
                wave_sync_solve();
            }
#pragma unroll
            for (int r = 0; r < NR; r++) red[wv][lane][r] = acc[r];
            __syncthreads();
            if (wv == 0 && lane < kb) {
#pragma unroll
                for (int r = 0; r < NR; r++)
                    s0[r] += ((red[0][lane][r] + red[1][lane][r]) + red[2][lane][r]) + red[3][lane][r];
                if (rb2 + kSolveChunk < c) {
#pragma unroll
                    for (int r = 0; r < NR; r++)
                        s0[r] += ((red[4][lane][r] + red[5][lane][r]) + red[6][lane][r]) + red[7][lane][r];
                }
            }
            __syncthreads();
        }
        // x_p = D_p^{-T} (y_p - partial sums)
#pragma unroll
        for (int q = 0; q < DPT; q++) {
            const int e = q * kSnThreads + tid;
            Dt[(e >> 6) * (kP + 1) + (e & 63)] = dreg[q];
        }
        if (wv == 0) {
#pragma unroll
            for (int r = 0; r < NR; r++) rhs[lane][r] = lane < kb ? yp[r] - s0[r] : T(0);
        }
        __syncthreads();
        if (wv == 0 && lane < kb) {
            T xt[NR];
#pragma unroll
            for (int r = 0; r < NR; r++) xt[r] = T(0);
#pragma unroll 8
            for (int i = 0; i < kb; i++) {
                const T dti = Dt[lane * (kP + 1) + i];
#pragma unroll
                for (int r = 0; r < NR; r++) xt[r] += dti * rhs[i][r];
            }
#pragma unroll
            for (int r = 0; r < NR; r++) {
                xs[c0 + lane][r] = xt[r];
                Ys[vix<SOA>(b, d.first + c0 + lane, r0 + r, n, nrhs)] = xt[r];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Supernodes with whole-block inverses X = L11^{-1} of their diagonal
// blocks (the panel-solved ones of levels whose panel supernodes are all at
// most kXMaxW wide, and the others of levels with at most kXSmallMax of
// them; formed after the factorization; column-major, leading dimension w,
// zero above the diagonal inside the diagonal 64 x 64 blocks, blocks above
// those never read).  Forward, after the gather of the front
// vector v = (v1, v2): y = X v1, then u = v2 - L21 y; backward: rhs = y -
// L21^T x2, then x1 = X^T rhs.  Each is a dense product over the whole
// block, split over 64-row (or 64-column) blocks so that a supernode takes
// many workgroups instead of one chain of 64-column panels.

constexpr int kXChunk = 512;  // vector rows staged in LDS at a time (backward)

// Column sums of the wave's 16 columns j0 .. j0 + 15 (those below jn) of a
// column-major block M (leading dimension ld) over rows [i0, i1), times the
// vector rows staged in vs (row i at vs[i - i0]): acc[k][r] += sum_i
// M[(j0 + k) ld + i] vs[i - i0][r].  Lanes take the rows 64 at a time, so
// every load of M is 64 consecutive entries of one column.
template <typename T, int NR>
__device__ __forceinline__ void wave_colsums(const T *__restrict__ M, int64_t ld, int i0, int i1,
                                             int j0, int jn, const T (*vs)[NR],
                                             T (&acc)[16][NR]) {
    const int lane = threadIdx.x & 63;
#pragma unroll 2
    for (int ib = i0; ib < i1; ib += 64) {
        const int i = ib + lane;
        const bool ok = i < i1;
        T v[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) v[r] = ok ? vs[i - i0][r] : T(0);
        T m[16];
#pragma unroll
        for (int k = 0; k < 16; k++) m[k] = ldz(M, int64_t(j0 + k) * ld + i, ok && j0 + k < jn);
#pragma unroll
        for (int k = 0; k < 16; k++)
#pragma unroll
            for (int r = 0; r < NR; r++) acc[k][r] += m[k] * v[r];
    }
}

// The lanes' column sums meet in a fixed butterfly; lane k (k < 16) returns
// column k's sums (lane 0's rounding), the others garbage.
template <typename T, int NR>
__device__ __forceinline__ void wave_colsums_finish(T (&acc)[16][NR], T (&out)[NR]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 16; k++)
#pragma unroll
        for (int r = 0; r < NR; r++) {
            T a = acc[k][r];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
            a = seg_bcast<64>(a, 0);
            if (lane == k) out[r] = a;
        }
}

// Forward, y = X v1: workgroup (row block R, supernode, matrix); lane = row
// 64 R + lane, the four waves take every fourth column j < 64 (R + 1)
// (X_RJ, J <= R) and their partial sums are added in wave order.
template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(256) void k_fx_y(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int r0,
    const int64_t *__restrict__ xoff, const T *__restrict__ X, int64_t xsize,
    T *__restrict__ Ys, const T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs,
    const int32_t *__restrict__ active) {
    __shared__ T vs[kXMaxW][NR];
    __shared__ T red[3][64][NR];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const int s = list[blockIdx.y];
    const SnDesc d = sn[s];
    const int w = d.w, i0 = 64 * int(blockIdx.x);
    if (i0 >= w) return;
    const int jend = min(w, i0 + 64);
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    for (int j = tid; j < jend; j += 256)
#pragma unroll
        for (int r = 0; r < NR; r++) vs[j][r] = FV[vix<SOA>(b, d.rowptr + j, r0 + r, fvsize, nrhs)];
    __syncthreads();
    const int i = i0 + lane;
    const bool ok = i < w;
    const T *Xb = X + int64_t(b) * xsize + xoff[s];
    T acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = T(0);
#pragma unroll 8
    for (int j = wv; j < jend; j += 4) {
        const T x = ldz(Xb, int64_t(j) * w + i, ok);
#pragma unroll
        for (int r = 0; r < NR; r++) acc[r] += x * vs[j][r];
    }
    if (wv > 0)
#pragma unroll
        for (int r = 0; r < NR; r++) red[wv - 1][lane][r] = acc[r];
    __syncthreads();
    if (wv == 0 && ok)
#pragma unroll
        for (int r = 0; r < NR; r++)
            Ys[vix<SOA>(b, d.first + i, r0 + r, n, nrhs)] =
                ((acc[r] + red[0][lane][r]) + red[1][lane][r]) + red[2][lane][r];
}

// Forward, u = v2 - L21 y into the front vector's rows >= w: workgroup
// (256 kFxRows rows below the diagonal block, supernode, matrix), thread t
// takes rows t + 256 q (q < kFxRows; the rows' loads of one column in flight
// together), every column j < w in ascending order.
constexpr int kFxRows = 4;  // rows per thread of k_fx_u
template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(256) void k_fx_u(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int r0,
    const T *__restrict__ L, int64_t Lsize, const T *__restrict__ Ys, T *__restrict__ FV,
    int64_t n, int64_t fvsize, int nrhs, const int32_t *__restrict__ active) {
    constexpr int RPT = kFxRows;
    __shared__ T ys[kXMaxW][NR];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const SnDesc d = sn[list[blockIdx.y]];
    const int w = d.w, c = d.c, i0 = w + 256 * RPT * int(blockIdx.x);
    if (i0 >= c) return;
    const int tid = threadIdx.x;
    for (int j = tid; j < w; j += 256)
#pragma unroll
        for (int r = 0; r < NR; r++) ys[j][r] = Ys[vix<SOA>(b, d.first + j, r0 + r, n, nrhs)];
    __syncthreads();
    if (i0 + tid >= c) return;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    int ic[RPT];
#pragma unroll
    for (int q = 0; q < RPT; q++) ic[q] = min(i0 + tid + 256 * q, c - 1);
    T acc[RPT][NR];
#pragma unroll
    for (int q = 0; q < RPT; q++)
#pragma unroll
        for (int r = 0; r < NR; r++) acc[q][r] = T(0);
#pragma unroll 8
    for (int j = 0; j < w; j++) {
        T l[RPT];
#pragma unroll
        for (int q = 0; q < RPT; q++) l[q] = Lb[int64_t(j) * c + ic[q]];
#pragma unroll
        for (int q = 0; q < RPT; q++)
#pragma unroll
            for (int r = 0; r < NR; r++) acc[q][r] += l[q] * ys[j][r];
    }
#pragma unroll
    for (int q = 0; q < RPT; q++) {
        const int i = i0 + tid + 256 * q;
        if (i < c)
#pragma unroll
            for (int r = 0; r < NR; r++) {
                const int64_t o = vix<SOA>(b, d.rowptr + i, r0 + r, fvsize, nrhs);
                FV[o] = FV[o] - acc[q][r];
            }
    }
}

// Backward, rhs = y - L21^T x2 into the front vector's rows < w: workgroup
// (column block C, supernode, matrix), wave wv takes columns 64 C + 16 wv
// .. + 15; x2 (read through the supernode's row list) is staged in LDS
// kXChunk rows at a time.
template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(256) void k_bx_t(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int r0,
    const int32_t *__restrict__ rows, const T *__restrict__ L, int64_t Lsize,
    const T *__restrict__ Ys, T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs,
    const int32_t *__restrict__ active) {
    __shared__ T xs[kXChunk][NR];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const SnDesc d = sn[list[blockIdx.y]];
    const int w = d.w, c = d.c;
    if (64 * int(blockIdx.x) >= w) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int j0 = 64 * int(blockIdx.x) + 16 * (tid >> 6);
    const int32_t *R = rows + d.rowptr;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    T acc[16][NR];
#pragma unroll
    for (int k = 0; k < 16; k++)
#pragma unroll
        for (int r = 0; r < NR; r++) acc[k][r] = T(0);
    for (int cb = w; cb < c; cb += kXChunk) {
        const int ce = min(c, cb + kXChunk);
        __syncthreads();  // the previous chunk is read
        for (int i = cb + tid; i < ce; i += 256) {
            const int ri = R[i];
#pragma unroll
            for (int r = 0; r < NR; r++) xs[i - cb][r] = Ys[vix<SOA>(b, ri, r0 + r, n, nrhs)];
        }
        __syncthreads();
        if (j0 < w) wave_colsums<T, NR>(Lb, c, cb, ce, j0, w, xs, acc);
    }
    T t[NR];
    wave_colsums_finish<T, NR>(acc, t);
    const int j = j0 + lane;
    if (lane < 16 && j < w)
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const T y = Ys[vix<SOA>(b, d.first + j, r0 + r, n, nrhs)];
            FV[vix<SOA>(b, d.rowptr + j, r0 + r, fvsize, nrhs)] = y - t[r];
        }
}

// Backward, x1 = X^T rhs: workgroup (column block C, supernode, matrix),
// columns split as in k_bx_t, rows i >= 64 C (X_IC, I >= C) with rhs staged
// in LDS.
template <typename T, int NR, bool SOA>
__global__ __launch_bounds__(256) void k_bx_x(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int r0,
    const int64_t *__restrict__ xoff, const T *__restrict__ X, int64_t xsize,
    T *__restrict__ Ys, const T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs,
    const int32_t *__restrict__ active) {
    __shared__ T rs[kXChunk][NR];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const int s = list[blockIdx.y];
    const SnDesc d = sn[s];
    const int w = d.w;
    const int c0 = 64 * int(blockIdx.x);
    if (c0 >= w) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int j0 = c0 + 16 * (tid >> 6);
    const T *Xb = X + int64_t(b) * xsize + xoff[s];
    T acc[16][NR];
#pragma unroll
    for (int k = 0; k < 16; k++)
#pragma unroll
        for (int r = 0; r < NR; r++) acc[k][r] = T(0);
    for (int cb = c0; cb < w; cb += kXChunk) {
        const int ce = min(w, cb + kXChunk);
        __syncthreads();
        for (int i = cb + tid; i < ce; i += 256)
#pragma unroll
            for (int r = 0; r < NR; r++)
                rs[i - cb][r] = FV[vix<SOA>(b, d.rowptr + i, r0 + r, fvsize, nrhs)];
        __syncthreads();
        if (j0 < w) wave_colsums<T, NR>(Xb, w, cb, ce, j0, w, rs, acc);
    }
    T x[NR];
    wave_colsums_finish<T, NR>(acc, x);
    const int j = j0 + lane;
    if (lane < 16 && j < w)
#pragma unroll
        for (int r = 0; r < NR; r++) Ys[vix<SOA>(b, d.first + j, r0 + r, n, nrhs)] = x[r];
}

// ---------------------------------------------------------------------------
// Batch-interleaved solves.  A group of 64 matrices shares one wave, lane =
// matrix: every lane runs the same sequential substitution on its own
// values, so every load of L or of a vector is 64 consecutive words and no
// value ever crosses lanes.  L (non-panel supernodes) is copied to
// Ls[((b / 64) Lsize + k) 64 + b % 64] once per factorization; the solve
// vectors use vix<true>.

// Ls <- L for kSoaChunk consecutive scalars from `chunks[x]` and the 64
// matrices of group y, through an LDS tile (both sides coalesced).
template <typename T>
__global__ __launch_bounds__(256) void k_to_soa(
    const T *__restrict__ L, int64_t Lsize, const int64_t *__restrict__ chunks, int batch,
    T *__restrict__ Ls) {
    __shared__ T tile[64][kSoaChunk + 1];
    const int64_t k0 = chunks[blockIdx.x];
    const int bg = blockIdx.y;
    const int t = threadIdx.x;
    const int kk = t % kSoaChunk, bh = t / kSoaChunk;  // 256 / kSoaChunk row phases
    constexpr int NPH = 256 / kSoaChunk;
    for (int q0 = 0; q0 < 64; q0 += 16 * NPH) {
        T v[16];
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int bl = q0 + bh + NPH * q;
            const int b = bg * 64 + bl;
            v[q] = ldz(L, int64_t(b) * Lsize + k0 + kk, bl < 64 && b < batch && k0 + kk < Lsize);
        }
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int bl = q0 + bh + NPH * q;
            if (bl < 64) tile[bl][kk] = v[q];
        }
    }
    __syncthreads();
    T *out = Ls + (int64_t(bg) * Lsize + k0) * 64;
#pragma unroll 8
    for (int q = 0; q < kSoaChunk * 64 / 256; q++) {
        const int e = t + 256 * q;
        const int k = e >> 6, bl = e & 63;
        if (k0 + k < Lsize) out[e] = tile[bl][k];
    }
}

// Ys[vix<true>(b, pinv[i], r)] = B[(b nrhs + r) ldb + i] through an LDS
// tile of 64 rows x 64 matrices: read along rows of each right-hand side
// (lanes = rows), written along matrices (lanes = matrices), so both sides
// move whole cache lines.
template <typename T>
__global__ __launch_bounds__(256) void k_perm_in_soa(
    const int32_t *__restrict__ pinv, const double *__restrict__ B, int64_t ldb,
    T *__restrict__ Ys, int64_t n, int nrhs, int batch) {
    __shared__ T tile[64][65];
    const int bg = blockIdx.y;
    const int64_t i0 = int64_t(blockIdx.x) * 64;
    const int t = threadIdx.x, lo = t & 63, hi = t >> 6;
    for (int r = 0; r < nrhs; r++) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int b = bg * 64 + hi + 4 * q;
            v[q] = ldz(B, (int64_t(b) * nrhs + r) * ldb + i0 + lo, b < batch && i0 + lo < n);
        }
#pragma unroll
        for (int q = 0; q < 16; q++) tile[hi + 4 * q][lo] = T(v[q]);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int64_t i = i0 + hi + 4 * q;
            if (i < n) Ys[((int64_t(bg) * n + pinv[i]) * nrhs + r) * 64 + lo] = tile[lo][hi + 4 * q];
        }
        __syncthreads();
    }
}

// X[(b nrhs + r) ldb + i] = Ys[vix<true>(b, pinv[i], r)] for the active
// matrices, through the same kind of tile.
template <typename T>
__global__ __launch_bounds__(256) void k_perm_out_soa(
    const int32_t *__restrict__ pinv, const T *__restrict__ Ys, double *__restrict__ X,
    int64_t ldb, int64_t n, int nrhs, int batch, const int32_t *__restrict__ active) {
    __shared__ T tile[64][65];
    const int bg = blockIdx.y;
    const int64_t i0 = int64_t(blockIdx.x) * 64;
    const int t = threadIdx.x, lo = t & 63, hi = t >> 6;
    for (int r = 0; r < nrhs; r++) {
        T v[16];
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int64_t i = i0 + hi + 4 * q;
            v[q] = ldz(Ys, ((int64_t(bg) * n + ldz(pinv, i, i < n)) * nrhs + r) * 64 + lo, i < n);
        }
#pragma unroll
        for (int q = 0; q < 16; q++) tile[hi + 4 * q][lo] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int b = bg * 64 + hi + 4 * q;
            const bool on = b < batch && i0 + lo < n && (!active || ldz(active, b, b < batch) != 0);
            if (on) X[(int64_t(b) * nrhs + r) * ldb + i0 + lo] = tile[lo][hi + 4 * q];
        }
        __syncthreads();
    }
}

constexpr int kSoaCols = 16;  // columns per chunk of the interleaved kernels
// rows per step of the row loops (their loads in flight together)
template <typename T> struct SoaRows { static constexpr int value = sizeof(T) == 4 ? 4 : 2; };

// Forward, diagonal blocks: one wave per (supernode, group of 64 matrices).
// Columns in chunks of 16: the chunk's rows are solved in registers
// (y_j = (v_j - sum_{k<j} L_jk y_k) / L_jj, ascending), y stored, and the
// later rows of the diagonal block (i < w) updated in FV.
template <typename T, int NR, int JW>
__device__ __forceinline__ void k_fwd_soa_diag_body(
    const SnDesc &d, int bg, const T *__restrict__ Ls, int64_t Lsize, T *__restrict__ Ys,
    T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs, int r0) {
    const unsigned lane = threadIdx.x;
    const int c = d.c, w = d.w;
    const SoaBlk<T> Lb(Ls + (int64_t(bg) * Lsize + d.loff) * 64, lane);
    // the supernode's own rows of y and its rows of the front vectors
    const SoaBlk<T> yb(Ys + ((int64_t(bg) * n + d.first) * nrhs + r0) * 64, lane);
    const SoaBlk<T> fb(FV + ((int64_t(bg) * fvsize + d.rowptr) * nrhs + r0) * 64, lane);
    for (int j0 = 0; j0 < w; j0 += JW) {
        const int jn = min(JW, w - j0);
        T v[JW][NR];
#pragma unroll
        for (int jj = 0; jj < JW; jj++) {
            const int i = j0 + jj;
#pragma unroll
            for (int r = 0; r < NR; r++)
                v[jj][r] = fb.ldz(int64_t(i) * nrhs + r, jj < jn);
        }
#pragma unroll
        for (int jj = 0; jj < JW; jj++) {
            const int i = j0 + jj;
            const bool ok = jj < jn;
            T lrow[JW];  // row i of the chunk's triangle, diagonal included
#pragma unroll
            for (int kk = 0; kk <= jj; kk++) lrow[kk] = Lb.ldz(int64_t(j0 + kk) * c + i, ok);
#pragma unroll
            for (int kk = 0; kk < jj; kk++)
#pragma unroll
                for (int r = 0; r < NR; r++) v[jj][r] -= T(lrow[kk]) * v[kk][r];
            const T rinv = ok ? T(1) / T(lrow[jj]) : T(0);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                v[jj][r] *= rinv;
                if (ok) yb.st(int64_t(i) * nrhs + r, v[jj][r]);
            }
        }
        // rows of the diagonal block below this chunk, RU at a time with
        // every load of the group issued first (v is 0 past jn, so those
        // entries of L are clamped loads without a select)
        constexpr int RU = SoaRows<T>::value;
        for (int i0 = j0 + JW; i0 < w; i0 += RU) {
            T a[RU][NR];
            T l[RU][JW];
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int i = i0 + u;
#pragma unroll
                for (int r = 0; r < NR; r++)
                    a[u][r] = fb.ldc(int64_t(i) * nrhs + r, i < w);
#pragma unroll
                for (int jj = 0; jj < JW; jj++)
                    l[u][jj] = Lb.ldc(int64_t(j0 + jj) * c + i, i < w && jj < jn);
            }
#pragma unroll
            for (int u = 0; u < RU; u++)
#pragma unroll
                for (int jj = 0; jj < JW; jj++)
#pragma unroll
                    for (int r = 0; r < NR; r++) a[u][r] -= T(l[u][jj]) * v[jj][r];
#pragma unroll
            for (int u = 0; u < RU; u++)
                if (i0 + u < w)
#pragma unroll
                    for (int r = 0; r < NR; r++) fb.st(int64_t(i0 + u) * nrhs + r, a[u][r]);
        }
    }
}

// column-chunk width by the supernode's width (uniform per wave), so
// narrow supernodes issue no masked loads for absent columns
template <typename T, int NR>
__device__ __forceinline__ void fwd_soa_diag(const SnDesc &d, int bg, const T *__restrict__ Ls,
                                             int64_t Lsize, T *__restrict__ Ys, T *__restrict__ FV,
                                             int64_t n, int64_t fvsize, int nrhs, int r0) {
    if (d.w <= 4) k_fwd_soa_diag_body<T, NR, 4>(d, bg, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
    else if (d.w <= 8) k_fwd_soa_diag_body<T, NR, 8>(d, bg, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
    else k_fwd_soa_diag_body<T, NR, 16>(d, bg, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
}

template <typename T, int NR>
__global__ __launch_bounds__(64) void k_fwd_soa_diag(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int32_t *__restrict__ gptr, const int32_t *__restrict__ gidx,
    const T *__restrict__ Ls, int64_t Lsize, T *__restrict__ Ys, T *__restrict__ FV,
    int64_t n, int64_t fvsize, int nrhs, int r0) {
    const SnDesc d = sn[list[blockIdx.x]];
    fwd_soa_diag<T, NR>(d, int(blockIdx.y), Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
}

// Forward, rows below the diagonal blocks: one wave per (row block of
// kSoaRows rows, group): u_i = v_i - sum_j L_ij y_j over the supernode's
// columns in chunks of 16 (ascending j), stored in FV as the update vector.
template <typename T, int NR, int JW>
__device__ __forceinline__ void k_fwd_soa_rows_body(
    const SnDesc &d, int rb, int bg, const T *__restrict__ Ls, int64_t Lsize,
    T *__restrict__ Ys, T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs,
    int r0) {
    const unsigned lane = threadIdx.x;
    const int c = d.c, w = d.w;
    const int re = min(c, rb + kSoaRows);
    constexpr int RU = SoaRows<T>::value;
    // global loads here (not buffer loads): with the pointers' no-alias
    // guarantee the next rows' loads of L may be issued before this group's
    // stores to the front vector
    const Soa<const T> Lb{Ls + (int64_t(bg) * Lsize + d.loff) * 64, lane};
    const Soa<const T> yb{Ys + ((int64_t(bg) * n + d.first) * nrhs + r0) * 64, lane};
    const Soa<T> fb{FV + ((int64_t(bg) * fvsize + d.rowptr) * nrhs + r0) * 64, lane};
    if (w > JW) {
        // several column chunks: each row group stays in registers across
        // the chunks (the same operations in the same order per row as the
        // chunk-outer loop below, without storing and reloading the front
        // vector between chunks); y's chunk is reloaded per row group
        for (int i0 = rb; i0 < re; i0 += RU) {
            T a[RU][NR];
#pragma unroll
            for (int u = 0; u < RU; u++)
#pragma unroll
                for (int r = 0; r < NR; r++) a[u][r] = fb.ldc(int64_t(i0 + u) * nrhs + r, i0 + u < re);
            for (int j0 = 0; j0 < w; j0 += JW) {
                const int jn = min(JW, w - j0);
                T y[JW][NR];
                T l[RU][JW];
#pragma unroll
                for (int jj = 0; jj < JW; jj++)
#pragma unroll
                    for (int r = 0; r < NR; r++)
                        y[jj][r] = yb.ldz(int64_t(j0 + jj) * nrhs + r, jj < jn);
#pragma unroll
                for (int u = 0; u < RU; u++)
#pragma unroll
                    for (int jj = 0; jj < JW; jj++)
                        l[u][jj] = Lb.ldc(int64_t(j0 + jj) * c + i0 + u, i0 + u < re && jj < jn);
#pragma unroll
                for (int u = 0; u < RU; u++)
#pragma unroll
                    for (int jj = 0; jj < JW; jj++)
#pragma unroll
                        for (int r = 0; r < NR; r++) a[u][r] -= T(l[u][jj]) * y[jj][r];
            }
#pragma unroll
            for (int u = 0; u < RU; u++)
                if (i0 + u < re)
#pragma unroll
                    for (int r = 0; r < NR; r++) fb[int64_t(i0 + u) * nrhs + r] = a[u][r];
        }
        return;
    }
    for (int j0 = 0; j0 < w; j0 += JW) {
        const int jn = min(JW, w - j0);
        T y[JW][NR];
#pragma unroll
        for (int jj = 0; jj < JW; jj++)
#pragma unroll
            for (int r = 0; r < NR; r++)
                y[jj][r] = yb.ldz(int64_t(j0 + jj) * nrhs + r, jj < jn);
        // RU rows at a time, every load of the group issued before any use
        // (y is 0 past jn and rows past re are not stored, so the loads of
        // L and of the front vector are clamped loads without a select)
        for (int i0 = rb; i0 < re; i0 += RU) {
            T a[RU][NR];
            T l[RU][JW];
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int i = i0 + u;
#pragma unroll
                for (int r = 0; r < NR; r++)
                    a[u][r] = fb.ldc(int64_t(i) * nrhs + r, i < re);
#pragma unroll
                for (int jj = 0; jj < JW; jj++)
                    l[u][jj] = Lb.ldc(int64_t(j0 + jj) * c + i, i < re && jj < jn);
            }
#pragma unroll
            for (int u = 0; u < RU; u++)
#pragma unroll
                for (int jj = 0; jj < JW; jj++)
#pragma unroll
                    for (int r = 0; r < NR; r++) a[u][r] -= T(l[u][jj]) * y[jj][r];
#pragma unroll
            for (int u = 0; u < RU; u++)
                if (i0 + u < re)
#pragma unroll
                    for (int r = 0; r < NR; r++) fb[int64_t(i0 + u) * nrhs + r] = a[u][r];
        }
    }
}

template <typename T, int NR>
__device__ __forceinline__ void fwd_soa_rows(const SnDesc &d, int rb, int bg, const T *__restrict__ Ls,
                                             int64_t Lsize, T *__restrict__ Ys, T *__restrict__ FV,
                                             int64_t n, int64_t fvsize, int nrhs, int r0) {
    if (d.w <= 4) k_fwd_soa_rows_body<T, NR, 4>(d, rb, bg, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
    else if (d.w <= 8) k_fwd_soa_rows_body<T, NR, 8>(d, rb, bg, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
    else k_fwd_soa_rows_body<T, NR, 16>(d, rb, bg, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
}

template <typename T, int NR>
__global__ __launch_bounds__(64) void k_fwd_soa_rows(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ it_s,
    const int32_t *__restrict__ it_r0, const int32_t *__restrict__ gptr,
    const int32_t *__restrict__ gidx, const T *__restrict__ Ls, int64_t Lsize,
    T *__restrict__ Ys, T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs,
    int r0) {
    const SnDesc d = sn[it_s[blockIdx.x]];
    fwd_soa_rows<T, NR>(d, it_r0[blockIdx.x], int(blockIdx.y), Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
}

// Backward, rows below the diagonal blocks: one wave per (row block,
// group): partial sums p_j = sum_i L_ij x_i over the block's rows (x from
// the solved ancestors), columns in chunks of 16, stored at
// part + (block index) w + j.
template <typename T, int NR, int JW>
__device__ __forceinline__ void k_bwd_soa_rows_body(
    const SnDesc &d, int rb, int bg, const int32_t *__restrict__ rows,
    const T *__restrict__ Ls, int64_t Lsize, const T *__restrict__ Ys,
    T *__restrict__ PS, int64_t psize, int64_t n, int nrhs, int r0) {
    const unsigned lane = threadIdx.x;
    const int c = d.c, w = d.w;
    const int re = min(c, rb + kSoaRows);
    const int kblk = (rb - w) / kSoaRows;
    constexpr int RU = SoaRows<T>::value;
    const int32_t *R = rows + d.rowptr;
    // the block's row indices, one per lane, broadcast with readlane below
    const int rmine = rb + int(lane) < re ? R[rb + lane] : 0;
    const SoaBlk<T> Lb(Ls + (int64_t(bg) * Lsize + d.loff) * 64, lane);
    const Soa<const T> yb{Ys + (int64_t(bg) * n * nrhs + r0) * 64, lane};
    const SoaBlk<T> pb(PS + ((int64_t(bg) * psize + d.part + int64_t(kblk) * w) * nrhs + r0) * 64, lane);
    for (int j0 = 0; j0 < w; j0 += JW) {
        const int jn = min(JW, w - j0);
        T acc[JW][NR];
#pragma unroll
        for (int jj = 0; jj < JW; jj++)
#pragma unroll
            for (int r = 0; r < NR; r++) acc[jj][r] = T(0);
        // x is 0 past re and the sums of columns past jn are not stored, so
        // the loads of L are clamped loads without a select
        for (int i0 = rb; i0 < re; i0 += RU) {
            T x[RU][NR];
            T l[RU][JW];
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int i = i0 + u;
                const int ri = i < re ? __builtin_amdgcn_readlane(rmine, i - rb) : 0;
#pragma unroll
                for (int r = 0; r < NR; r++) x[u][r] = yb.ldz(int64_t(ri) * nrhs + r, i < re);
#pragma unroll
                for (int jj = 0; jj < JW; jj++)
                    l[u][jj] = Lb.ldc(int64_t(j0 + jj) * c + i, i < re && jj < jn);
            }
#pragma unroll
            for (int u = 0; u < RU; u++)
#pragma unroll
                for (int jj = 0; jj < JW; jj++)
#pragma unroll
                    for (int r = 0; r < NR; r++) acc[jj][r] += T(l[u][jj]) * x[u][r];
        }
#pragma unroll
        for (int jj = 0; jj < JW; jj++)
            if (jj < jn)
#pragma unroll
                for (int r = 0; r < NR; r++) pb.st(int64_t(j0 + jj) * nrhs + r, acc[jj][r]);
    }
}

template <typename T, int NR>
__device__ __forceinline__ void bwd_soa_rows(const SnDesc &d, int rb, int bg,
                                             const int32_t *__restrict__ rows,
                                             const T *__restrict__ Ls, int64_t Lsize,
                                             const T *__restrict__ Ys, T *__restrict__ PS,
                                             int64_t psize, int64_t n, int nrhs, int r0) {
    if (d.w <= 4) k_bwd_soa_rows_body<T, NR, 4>(d, rb, bg, rows, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
    else if (d.w <= 8) k_bwd_soa_rows_body<T, NR, 8>(d, rb, bg, rows, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
    else k_bwd_soa_rows_body<T, NR, 16>(d, rb, bg, rows, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
}

template <typename T, int NR>
__global__ __launch_bounds__(64) void k_bwd_soa_rows(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ it_s,
    const int32_t *__restrict__ it_r0, const int32_t *__restrict__ rows,
    const T *__restrict__ Ls, int64_t Lsize, const T *__restrict__ Ys,
    T *__restrict__ PS, int64_t psize, int64_t n, int nrhs, int r0) {
    const SnDesc d = sn[it_s[blockIdx.x]];
    bwd_soa_rows<T, NR>(d, it_r0[blockIdx.x], int(blockIdx.y), rows, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
}

// Backward, diagonal blocks: one wave per (supernode, group).  Column
// chunks of 16 from the last: rhs_j = y_j - (row-block partial sums, in
// block order) - (the supernode's own later rows, descending), then the
// chunk's triangle from its last column (x_j = rhs_j / L_jj, subtracted
// from the earlier columns of the chunk).  Every column sees the same
// sequence of operations as in the row-major kernels.
template <typename T, int NR, int JW>
__device__ __forceinline__ void k_bwd_soa_diag_body(
    const SnDesc &d, int bg, const T *__restrict__ Ls, int64_t Lsize, T *__restrict__ Ys,
    const T *__restrict__ PS, int64_t psize, int64_t n, int nrhs, int r0) {
    const unsigned lane = threadIdx.x;
    const int c = d.c, w = d.w;
    const int nblk = (c - w + kSoaRows - 1) / kSoaRows;
    const SoaBlk<T> Lb(Ls + (int64_t(bg) * Lsize + d.loff) * 64, lane);
    const SoaBlk<T> yb(Ys + ((int64_t(bg) * n + d.first) * nrhs + r0) * 64, lane);
    const SoaBlk<T> pb(PS + ((int64_t(bg) * psize + d.part) * nrhs + r0) * 64, lane);
    constexpr int RU = SoaRows<T>::value;
    for (int j0 = ((w - 1) / JW) * JW; j0 >= 0; j0 -= JW) {
        const int jn = min(JW, w - j0);
        T acc[JW][NR];
#pragma unroll
        for (int jj = 0; jj < JW; jj++)
#pragma unroll
            for (int r = 0; r < NR; r++)
                acc[jj][r] = yb.ldz(int64_t(j0 + jj) * nrhs + r, jj < jn);
        for (int k = 0; k < nblk; k++) {  // row-block partial sums, in block order
            T p[JW][NR];
#pragma unroll
            for (int jj = 0; jj < JW; jj++)
#pragma unroll
                for (int r = 0; r < NR; r++)
                    p[jj][r] = pb.ldz((int64_t(k) * w + j0 + jj) * nrhs + r, jj < jn);
#pragma unroll
            for (int jj = 0; jj < JW; jj++)
#pragma unroll
                for (int r = 0; r < NR; r++) acc[jj][r] -= p[jj][r];
        }
        // the supernode's own later rows, descending as in the other layout,
        // RU rows with their loads in flight together
        for (int i1 = w - 1; i1 >= j0 + JW; i1 -= RU) {
            T x[RU][NR];
            T l[RU][JW];
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int i = i1 - u;
                const bool ok = i >= j0 + JW;
#pragma unroll
                for (int r = 0; r < NR; r++) x[u][r] = yb.ldz(int64_t(i) * nrhs + r, ok);
#pragma unroll
                for (int jj = 0; jj < JW; jj++)  // x is 0 when !ok; columns past jn unused
                    l[u][jj] = Lb.ldc(int64_t(j0 + jj) * c + i, ok && jj < jn);
            }
#pragma unroll
            for (int u = 0; u < RU; u++)
#pragma unroll
                for (int jj = 0; jj < JW; jj++)
#pragma unroll
                    for (int r = 0; r < NR; r++) acc[jj][r] -= T(l[u][jj]) * x[u][r];
        }
#pragma unroll
        for (int jj = JW - 1; jj >= 0; jj--) {
            const int j = j0 + jj;
            const bool ok = jj < jn;
            T lrow[JW];  // row j of the chunk's triangle, diagonal included
#pragma unroll
            for (int kk = 0; kk <= jj; kk++) lrow[kk] = Lb.ldz(int64_t(j0 + kk) * c + j, ok);
            const T rinv = ok ? T(1) / T(lrow[jj]) : T(0);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                acc[jj][r] *= rinv;
                if (ok) yb.st(int64_t(j) * nrhs + r, acc[jj][r]);
            }
#pragma unroll
            for (int kk = 0; kk < jj; kk++)
#pragma unroll
                for (int r = 0; r < NR; r++) acc[kk][r] -= T(lrow[kk]) * acc[jj][r];
        }
    }
}

template <typename T, int NR>
__device__ __forceinline__ void bwd_soa_diag(const SnDesc &d, int bg, const T *__restrict__ Ls,
                                             int64_t Lsize, T *__restrict__ Ys,
                                             const T *__restrict__ PS, int64_t psize, int64_t n,
                                             int nrhs, int r0) {
    if (d.w <= 4) k_bwd_soa_diag_body<T, NR, 4>(d, bg, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
    else if (d.w <= 8) k_bwd_soa_diag_body<T, NR, 8>(d, bg, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
    else k_bwd_soa_diag_body<T, NR, 16>(d, bg, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
}

template <typename T, int NR>
__global__ __launch_bounds__(64) void k_bwd_soa_diag(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const T *__restrict__ Ls, int64_t Lsize, T *__restrict__ Ys,
    const T *__restrict__ PS, int64_t psize, int64_t n, int nrhs, int r0) {
    const SnDesc d = sn[list[blockIdx.x]];
    bwd_soa_diag<T, NR>(d, int(blockIdx.y), Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
}

// Bottom subtrees in one launch (batch-interleaved layout).  The lowest
// levels of the tree hold many small supernodes; solving them level by
// level costs three launches per level and passes every update vector
// through memory between launches.  Here one wave per (subtree, group of 64
// matrices) walks a whole subtree: forward in postorder (children first),
// backward in reverse postorder.  Each supernode goes through the same
// three steps as in the level kernels (gather of its front vector, the
// diagonal block, the rows below; backward: the row blocks' partial sums,
// then the diagonal block) with the same arithmetic in the same order, so
// the bits are those of the level-by-level solve; forward, a supernode of
// width <= 16 takes the three steps in one pass (fwd_soa_fused_body).  A lane only ever reads entries of
// its own matrix that it wrote earlier in the same wave or that earlier
// launches wrote, so the wave needs no synchronization.

// Gathered front-vector rows i0 .. i0 + GR - 1 of supernode d: y_{first + i}
// for i < w (0 below), plus the children's update entries of the row in map
// order; rows at or past `lim` give 0 and load nothing.  The chunk's gather
// indices come in with one vector load (lane l holds entry g0 + l) and are
// broadcast from there, so the first GK entries of every row are loaded
// before any is added; later entries of a row, if any, follow one by one.
template <typename T, int NR, int GR, int GK>
__device__ __forceinline__ void soa_gather_chunk(const SnDesc &d, int i0, int lim,
                                                 const int32_t *__restrict__ gptr,
                                                 const int32_t *__restrict__ gidx,
                                                 const Soa<const T> &yg, const Soa<T> &fg,
                                                 int nrhs, T (&a)[GR][NR]) {
    const int64_t q0 = d.rowptr + i0;
    const int nr = min(GR, lim - i0);
    int gb[GR + 1];
#pragma unroll
    for (int u = 0; u <= GR; u++) gb[u] = gptr[q0 + min(u, nr)];
    const int gcnt = gb[GR] - gb[0];
    const int gl = fg.lane < unsigned(gcnt) ? gidx[gb[0] + int(fg.lane)] : 0;
#pragma unroll
    for (int u = 0; u < GR; u++) {
        const int i = i0 + u;
        const bool own = i < d.w && u < nr;
#pragma unroll
        for (int r = 0; r < NR; r++) a[u][r] = yg.ldz(int64_t(d.first + i) * nrhs + r, own);
    }
    T t[GR][GK][NR];
#pragma unroll
    for (int u = 0; u < GR; u++)
#pragma unroll
        for (int k = 0; k < GK; k++) {
            const int g = gb[u] + k;
            const bool ok = g < gb[u + 1] && g - gb[0] < 64;
            const int64_t src = __builtin_amdgcn_readlane(gl, ok ? g - gb[0] : 0);
#pragma unroll
            for (int r = 0; r < NR; r++) t[u][k][r] = fg.ldc(src * nrhs + r, ok);
        }
#pragma unroll
    for (int u = 0; u < GR; u++) {
        if (u >= nr) break;
        int g = gb[u];
#pragma unroll
        for (int k = 0; k < GK; k++) {
            if (g < gb[u + 1] && g - gb[0] < 64) {
#pragma unroll
                for (int r = 0; r < NR; r++) a[u][r] += t[u][k][r];
                g++;
            }
        }
        for (; g < gb[u + 1]; g++) {
            const int64_t src = gidx[g];
#pragma unroll
            for (int r = 0; r < NR; r++) a[u][r] += fg[src * nrhs + r];
        }
    }
}

// Front vector of supernode d (forward) into FV, as k_gather.
template <typename T, int NR>
__device__ __forceinline__ void fwd_soa_gather(const SnDesc &d, int bg,
                                               const int32_t *__restrict__ gptr,
                                               const int32_t *__restrict__ gidx,
                                               const T *__restrict__ Ys, T *__restrict__ FV,
                                               int64_t n, int64_t fvsize, int nrhs, int r0) {
    const unsigned lane = threadIdx.x & 63;
    const Soa<const T> yg{Ys + (int64_t(bg) * n * nrhs + r0) * 64, lane};
    const Soa<T> fg{FV + (int64_t(bg) * fvsize * nrhs + r0) * 64, lane};
    constexpr int GR = 8, GK = sizeof(T) == 4 ? 4 : 2;
    for (int i0 = 0; i0 < d.c; i0 += GR) {
        T a[GR][NR];
        soa_gather_chunk<T, NR, GR, GK>(d, i0, d.c, gptr, gidx, yg, fg, nrhs, a);
#pragma unroll
        for (int u = 0; u < GR; u++)
            if (i0 + u < d.c)
#pragma unroll
                for (int r = 0; r < NR; r++) fg[(d.rowptr + i0 + u) * nrhs + r] = a[u][r];
    }
}

// Gather, diagonal block and rows below of one supernode with w <= JW (one
// column chunk), in one pass: the diagonal block's front rows stay in
// registers and the update rows are gathered, reduced and stored once.  The
// arithmetic is that of fwd_soa_gather + fwd_soa_diag + fwd_soa_rows with
// the same JW, operation for operation, so the bits are the same.
template <typename T, int NR, int JW>
__device__ __forceinline__ void fwd_soa_fused_body(
    const SnDesc &d, int bg, const int32_t *__restrict__ gptr, const int32_t *__restrict__ gidx,
    const T *__restrict__ Ls, int64_t Lsize, T *__restrict__ Ys, T *__restrict__ FV, int64_t n,
    int64_t fvsize, int nrhs, int r0) {
    const unsigned lane = threadIdx.x & 63;
    const int c = d.c, w = d.w;
    // four update rows per step and two child entries per row in flight:
    // larger steps take more registers than three waves per SIMD allow
    constexpr int GK = 2, GR = 4;
    constexpr int TR = JW < GR ? JW : GR;  // diagonal-block rows per gather chunk
    const Soa<const T> yg{Ys + (int64_t(bg) * n * nrhs + r0) * 64, lane};
    const Soa<T> fg{FV + (int64_t(bg) * fvsize * nrhs + r0) * 64, lane};
    const SoaBlk<T> Lb(Ls + (int64_t(bg) * Lsize + d.loff) * 64, lane);
    const SoaBlk<T> yb(Ys + ((int64_t(bg) * n + d.first) * nrhs + r0) * 64, lane);
    T v[JW][NR];
#pragma unroll
    for (int k = 0; k < JW / TR; k++) {
        T a[TR][NR];
        if (k * TR < w) {
            soa_gather_chunk<T, NR, TR, GK>(d, k * TR, w, gptr, gidx, yg, fg, nrhs, a);
        } else {
#pragma unroll
            for (int u = 0; u < TR; u++)
#pragma unroll
                for (int r = 0; r < NR; r++) a[u][r] = T(0);
        }
#pragma unroll
        for (int u = 0; u < TR; u++)
#pragma unroll
            for (int r = 0; r < NR; r++) v[k * TR + u][r] = a[u][r];
    }
#pragma unroll
    for (int jj = 0; jj < JW; jj++) {
        const bool ok = jj < w;
        T lrow[JW];
#pragma unroll
        for (int kk = 0; kk <= jj; kk++) lrow[kk] = Lb.ldz(int64_t(kk) * c + jj, ok);
#pragma unroll
        for (int kk = 0; kk < jj; kk++)
#pragma unroll
            for (int r = 0; r < NR; r++) v[jj][r] -= T(lrow[kk]) * v[kk][r];
        const T rinv = ok ? T(1) / T(lrow[jj]) : T(0);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            v[jj][r] *= rinv;
            if (ok) yb.st(int64_t(jj) * nrhs + r, v[jj][r]);
        }
    }
    for (int i0 = w; i0 < c; i0 += GR) {
        T a[GR][NR];
        soa_gather_chunk<T, NR, GR, GK>(d, i0, c, gptr, gidx, yg, fg, nrhs, a);
        T l[GR][JW];
#pragma unroll
        for (int u = 0; u < GR; u++)
#pragma unroll
            for (int jj = 0; jj < JW; jj++)
                l[u][jj] = Lb.ldc(int64_t(jj) * c + i0 + u, i0 + u < c && jj < w);
#pragma unroll
        for (int u = 0; u < GR; u++)
#pragma unroll
            for (int jj = 0; jj < JW; jj++)
#pragma unroll
                for (int r = 0; r < NR; r++) a[u][r] -= T(l[u][jj]) * v[jj][r];
#pragma unroll
        for (int u = 0; u < GR; u++)
            if (i0 + u < c)
#pragma unroll
                for (int r = 0; r < NR; r++) fg[(d.rowptr + i0 + u) * nrhs + r] = a[u][r];
    }
}

template <typename T, int NR>
__global__ __launch_bounds__(64) void k_fwd_soa_subtree(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ sub_ptr,
    const int32_t *__restrict__ sub_sn, const int32_t *__restrict__ gptr,
    const int32_t *__restrict__ gidx, const T *__restrict__ Ls, int64_t Lsize,
    T *__restrict__ Ys, T *__restrict__ FV, int64_t n, int64_t fvsize, int nrhs, int r0) {
    const int bg = blockIdx.y;
    const int e0 = sub_ptr[blockIdx.x], e1 = sub_ptr[blockIdx.x + 1];
    for (int e = e0; e < e1; e++) {
        const SnDesc d = sn[sub_sn[e]];
        if (d.w <= 4) {
            fwd_soa_fused_body<T, NR, 4>(d, bg, gptr, gidx, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
        } else if (d.w <= 8) {
            fwd_soa_fused_body<T, NR, 8>(d, bg, gptr, gidx, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
        } else if (d.w <= 16) {
            fwd_soa_fused_body<T, NR, 16>(d, bg, gptr, gidx, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
        } else {
            fwd_soa_gather<T, NR>(d, bg, gptr, gidx, Ys, FV, n, fvsize, nrhs, r0);
            fwd_soa_diag<T, NR>(d, bg, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
            for (int rb = d.w; rb < d.c; rb += kSoaRows)
                fwd_soa_rows<T, NR>(d, rb, bg, Ls, Lsize, Ys, FV, n, fvsize, nrhs, r0);
        }
    }
}

template <typename T, int NR>
__global__ __launch_bounds__(64) void k_bwd_soa_subtree(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ sub_ptr,
    const int32_t *__restrict__ sub_sn, const int32_t *__restrict__ rows,
    const T *__restrict__ Ls, int64_t Lsize, T *__restrict__ Ys, T *__restrict__ PS,
    int64_t psize, int64_t n, int nrhs, int r0) {
    const int bg = blockIdx.y;
    const int e0 = sub_ptr[blockIdx.x], e1 = sub_ptr[blockIdx.x + 1];
    for (int e = e1 - 1; e >= e0; e--) {
        const SnDesc d = sn[sub_sn[e]];
        for (int rb = d.w; rb < d.c; rb += kSoaRows)
            bwd_soa_rows<T, NR>(d, rb, bg, rows, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
        bwd_soa_diag<T, NR>(d, bg, Ls, Lsize, Ys, PS, psize, n, nrhs, r0);
    }
}

// Solve workspaces hold vectors in the factor's precision (allocated as
// doubles, large enough for either).
template <typename T>
T *as(double *p) { return reinterpret_cast<T *>(p); }

template <typename T>
hipError_t dinv_impl(const sc_plan *P, sc_numeric *N, hipStream_t st, int parts) {
    DevPlan *D = P->dev;
    const T *L = static_cast<const T *>(N->L);
    if ((parts & 1) && N->xinv && !P->xs_list.empty()) {
        N->prof.begin(KK_Dinv, 0.0, 0.0, st);
        hipLaunchKernelGGL(k_xsmall<T>, dim3(unsigned(N->batch), unsigned(P->xs_list.size())),
                           dim3(64), 0, st, D->sn, D->xs_list, D->xoff, L, P->Lsize,
                           static_cast<T *>(N->xinv), P->xsize);
        N->prof.end(st);
    }
    if (!(parts & 2) || P->dinv_list.empty()) return hipGetLastError();
    const int64_t maxp = (P->max_width + kP - 1) / kP;
    N->prof.begin(KK_Dinv, 0.0, 0.0, st);
    hipLaunchKernelGGL(k_dinv<T>,
                       dim3(unsigned(maxp), unsigned(P->dinv_list.size()), unsigned(N->batch)),
                       dim3(64), 0, st, D->sn, D->dinv_list, L, P->Lsize, as<T>(N->dinv),
                       P->dinv_size);
    N->prof.end(st);
    return hipGetLastError();
}

template <typename T, bool SOA>
void launch_gather_rows(const int32_t *gq, const int32_t *gy, int32_t nrow, double vw, double ib,
                        const sc_plan *P, sc_numeric *N, int nrhs, const int32_t *active,
                        hipStream_t st) {
    if (nrow == 0) return;
    const DevPlan *D = P->dev;
    const int B = N->batch;
    const int64_t fvsize = int64_t(P->rows.size());
    N->prof.begin(KK_Gather, 0.0, (vw * double(sizeof(T)) + ib) * double(nrhs) * double(B), st);
    const dim3 g = SOA ? dim3(unsigned((nrow + 3) / 4), unsigned((B + 63) / 64))
                       : dim3(unsigned((int64_t(nrow) * B + 255) / 256));
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
        const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_GATHER(NRV)                                                                     \
    hipLaunchKernelGGL((k_gather<T, SOA, NRV>), g, dim3(256), 0, st, gq, gy, nrow, D->gptr,       \
                       D->gidx, as<T>(N->wsc->y), as<T>(N->wsc->u), P->n, fvsize, nrhs, r0, B,  \
                       active)
        if (nrr == 1) SPCHOL_GATHER(1);
        else if (nrr == 2) SPCHOL_GATHER(2);
        else if (nrr == 3) SPCHOL_GATHER(3);
        else SPCHOL_GATHER(4);
#undef SPCHOL_GATHER
    }
    N->prof.end(st);
}

// Gather of the front vectors of one level (rows of the supernodes not
// solved by panels), every right-hand side.
template <typename T, bool SOA>
void launch_gather(const SLaunch &l, const sc_plan *P, sc_numeric *N, int nrhs,
                   const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    launch_gather_rows<T, SOA>(D->grow_q + l.grow0, D->grow_y + l.grow0, l.ngrow, l.vw_gather,
                               l.ib_gather, P, N, nrhs, active, st);
}

// One launch of the segment kernels for row class k.
template <typename T, int NR, bool SOA>
void launch_fwd_class(int k, dim3 g, hipStream_t st, const DevPlan *D, const sc_plan *P,
                      const sc_numeric *N, const SClass &cl, int nitems, int r0, int nrhs,
                      int64_t fvsize, const int32_t *active) {
    const T *L = static_cast<const T *>(N->L);
    const int32_t *lst = D->slv_small + cl.list0;
#define SPCHOL_FWDS(G, SL)                                                                   \
    hipLaunchKernelGGL((k_fwd_seg<T, G, SL, NR, SOA>), g, dim3(256), 0, st, D->sn, lst, cl.n, \
                       nitems, r0, D->gptr, D->gidx, L, P->Lsize, as<T>(N->wsc->y), as<T>(N->wsc->u), P->n,     \
                       fvsize, nrhs, active)
    switch (k) {
    case 0: SPCHOL_FWDS(16, 1); break;
    case 1: SPCHOL_FWDS(32, 1); break;
    case 2: SPCHOL_FWDS(64, 1); break;
    case 3: SPCHOL_FWDS(64, 2); break;
    case 4: SPCHOL_FWDS(64, 4); break;
    default: SPCHOL_FWDS(64, 8); break;
    }
#undef SPCHOL_FWDS
}

template <typename T, int NR, bool SOA>
void launch_bwd_class(int k, dim3 g, hipStream_t st, const DevPlan *D, const sc_plan *P,
                      const sc_numeric *N, const SClass &cl, int nitems, int r0, int nrhs,
                      const int32_t *active) {
    const T *L = static_cast<const T *>(N->L);
    const int32_t *lst = D->slv_small + cl.list0;
#define SPCHOL_BWDS(G)                                                                       \
    hipLaunchKernelGGL((k_bwd_seg<T, G, NR, SOA>), g, dim3(256), 0, st, D->sn, lst, cl.n,     \
                       nitems, r0, D->rows, L, P->Lsize, as<T>(N->wsc->y), P->n, nrhs, active)
    if (k == 0) SPCHOL_BWDS(16);
    else if (k == 1) SPCHOL_BWDS(32);
    else SPCHOL_BWDS(64);
#undef SPCHOL_BWDS
}

inline int class_lanes(int k) { return k == 0 ? 16 : k == 1 ? 32 : 64; }

// Forward and backward steps of one level's supernodes not solved by
// panels, with the segment kernels (one launch per row class).
template <typename T, bool SOA>
void classes_forward(const SLaunch &l, const sc_plan *P, sc_numeric *N, int nrhs,
                     const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    const int B = N->batch;
    const int64_t fvsize = int64_t(P->rows.size());
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    for (int k = 0; k < kSolveClasses; k++) {
        const SClass &cl = l.cls[k];
        if (cl.n == 0) continue;
        N->prof.begin(KK_Fwd, cl.flops * nr * nb,
                      (cl.words * sz + (cl.vwords * sz + cl.ibytes) * nr) * nb, st,
                      cl.lx * sz * nb);
        const int nitems = cl.n * B;
        const int nseg = 256 / class_lanes(k);
        const dim3 g(unsigned((nitems + nseg - 1) / nseg));
        for (int r0 = 0; r0 < nrhs; r0 += 4) {
            const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_FWDC(NRV) \
    launch_fwd_class<T, NRV, SOA>(k, g, st, D, P, N, cl, nitems, r0, nrhs, fvsize, active)
            if (nrr == 1) SPCHOL_FWDC(1);
            else if (nrr == 2) SPCHOL_FWDC(2);
            else if (nrr == 3) SPCHOL_FWDC(3);
            else SPCHOL_FWDC(4);
#undef SPCHOL_FWDC
        }
        N->prof.end(st);
    }
}

template <typename T, bool SOA>
void classes_backward(const SLaunch &l, const sc_plan *P, sc_numeric *N, int nrhs,
                      const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    const int B = N->batch;
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    for (int k = kSolveClasses - 1; k >= 0; k--) {
        const SClass &cl = l.cls[k];
        if (cl.n == 0) continue;
        N->prof.begin(KK_Bwd, cl.flops * nr * nb,
                      (cl.words * sz + (cl.vwords * sz + cl.ibytes) * nr) * nb, st,
                      cl.lx * sz * nb);
        const int nitems = cl.n * B;
        const int nseg = 256 / class_lanes(k);
        const dim3 g(unsigned((nitems + nseg - 1) / nseg));
        for (int r0 = 0; r0 < nrhs; r0 += 4) {
            const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_BWDC(NRV) \
    launch_bwd_class<T, NRV, SOA>(k, g, st, D, P, N, cl, nitems, r0, nrhs, active)
            if (nrr == 1) SPCHOL_BWDC(1);
            else if (nrr == 2) SPCHOL_BWDC(2);
            else if (nrr == 3) SPCHOL_BWDC(3);
            else SPCHOL_BWDC(4);
#undef SPCHOL_BWDC
        }
        N->prof.end(st);
    }
}

// Panel-solved supernodes of one level, forward (gather with y_0, then one
// launch per panel) and backward (per panel from the last: partial sums
// below the panel, then the panel's own solve), in either vector layout.
template <typename T, bool SOA>
void panels_forward(const SLaunch &l, const sc_plan *P, sc_numeric *N, int nrhs,
                    const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    const T *L = static_cast<const T *>(N->L);
    const int B = N->batch;
    const int64_t fvsize = int64_t(P->rows.size());
    Profiler &prof = N->prof;
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    prof.begin(KK_FwdPanel, 0.0, (l.vw_pan * sz + l.ib_pan) * nr * nb, st);
    hipLaunchKernelGGL((k_pan_gather<T, SOA>), dim3(unsigned(l.npan), unsigned(B)), dim3(256), 0, st,
                       D->sn, D->slv_pan + l.pan0, D->gptr, D->gidx, as<T>(N->dinv), P->dinv_size,
                       as<T>(N->wsc->y), as<T>(N->wsc->u), P->n, fvsize, nrhs, active);
    prof.end(st);
    for (size_t q = 0; q < l.panels.size(); q++) {
        const SPanel &pp = l.panels[q];
        if (pp.fwd_tiles == 0) continue;
        prof.begin(KK_FwdPanel, pp.flops * nr * nb,
                   (pp.words * sz + pp.dwords * sz + pp.vwords * sz * nr) * nb, st,
                   pp.lx * sz * nb);
        const dim3 g(unsigned(pp.fwd_tiles), unsigned(l.npan), unsigned(B));
        for (int r0 = 0; r0 < nrhs; r0 += 4) {
            const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_FWDP(NRV)                                                                       \
    hipLaunchKernelGGL((k_fwd_panel<T, NRV, SOA>), g, dim3(64), 0, st, D->sn,                  \
                       D->slv_pan + l.pan0, int(q), r0, L, P->Lsize, as<T>(N->dinv), P->dinv_size,     \
                       as<T>(N->wsc->y), as<T>(N->wsc->u), P->n, fvsize, nrhs, active)
            if (nrr == 1) SPCHOL_FWDP(1);
            else if (nrr == 2) SPCHOL_FWDP(2);
            else if (nrr == 3) SPCHOL_FWDP(3);
            else SPCHOL_FWDP(4);
#undef SPCHOL_FWDP
        }
        prof.end(st);
    }
}

template <typename T, bool SOA>
void panels_backward(const SLaunch &l, const sc_plan *P, sc_numeric *N, int nrhs,
                     const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    const T *L = static_cast<const T *>(N->L);
    const int B = N->batch;
    Profiler &prof = N->prof;
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    for (size_t q = l.panels.size(); q-- > 0;) {
        const SPanel &pp = l.panels[q];
        prof.begin(KK_BwdPanel, pp.flops * nr * nb,
                   (pp.words * sz + pp.dwords * sz + pp.vwords * sz * nr) * nb, st,
                   pp.lx * sz * nb);
        for (int r0 = 0; r0 < nrhs; r0 += 4) {
            const int nrr = std::min(4, nrhs - r0);
            const dim3 gp(unsigned(pp.bwd_chunks), unsigned(l.npan), unsigned(B));
            const dim3 gf(unsigned(l.npan), unsigned(B));
#define SPCHOL_BWDP(NRV)                                                                         \
    do {                                                                                         \
        if (pp.bwd_chunks > 0)                                                                   \
            hipLaunchKernelGGL((k_bwd_pan_part<T, NRV, SOA>), gp, dim3(256), 0, st, D->sn,       \
                               D->slv_pan + l.pan0, int(q), r0, D->rows, L, P->Lsize, as<T>(N->wsc->y),   \
                               P->n, as<T>(N->wsc->part), P->part_size, nrhs, active);                    \
        hipLaunchKernelGGL((k_bwd_pan_fin<T, NRV, SOA>), gf, dim3(64), 0, st, D->sn,                \
                           D->slv_pan + l.pan0, int(q), r0, as<T>(N->dinv), P->dinv_size, as<T>(N->wsc->y),      \
                           P->n, as<T>(N->wsc->part), P->part_size, nrhs, active);                        \
    } while (0)
            if (nrr == 1) SPCHOL_BWDP(1);
            else if (nrr == 2) SPCHOL_BWDP(2);
            else if (nrr == 3) SPCHOL_BWDP(3);
            else SPCHOL_BWDP(4);
#undef SPCHOL_BWDP
        }
        prof.end(st);
    }
}

// Panel-solved supernodes of a level with one workgroup per (supernode,
// matrix), when the batch fills the chip and the front vector fits in LDS:
// at least kSnMinBatch matrices and kSnMinGroups workgroups, fronts of at
// most kSnMaxRows rows (a taller front is a long chain for one workgroup;
// the multi-launch panel kernels spread it over the chip instead).
constexpr int kSnMinBatch = 16;
constexpr int kSnMinGroups = 64;
constexpr int kSnMaxRows = 1024;
template <typename T>
size_t sn_static_lds(int nr) {
    return sizeof(T) * (size_t(kSnWaves) * kSnRB * (kP + 1) + (kSnWaves + 1) * size_t(kP) * nr);
}
template <typename T>
bool sn_fits(const SLaunch &l, const sc_numeric *N, int nrhs) {
    const int nr = std::min(kMaxRhsPanel, nrhs);
    const size_t front = size_t(l.maxc_pan) * nr * sizeof(T);
    return N->batch >= kSnMinBatch && int64_t(l.npan) * N->batch >= kSnMinGroups &&
           l.maxc_pan <= kSnMaxRows && front + sn_static_lds<T>(nr) <= size_t(g_max_lds) &&
           front + kP * kP * sizeof(T) <= size_t(g_max_lds);
}

template <typename T, bool SOA>
void sn_forward(const SLaunch &l, const sc_plan *P, sc_numeric *N, int nrhs,
                const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    const T *L = static_cast<const T *>(N->L);
    const int B = N->batch;
    const int64_t fvsize = int64_t(P->rows.size());
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    double f = 0.0, wds = 0.0, dw = 0.0, vw = 0.0, lx = 0.0;
    for (const SPanel &pp : l.panels) {
        f += pp.flops;
        wds += pp.words;
        dw += pp.dwords;
        vw += pp.vwords;
        lx += pp.lx;
    }
    N->prof.begin(KK_FwdPanel, f * nr * nb,
                  ((wds + dw) * sz + (vw * sz + l.vw_pan * sz + l.ib_pan) * nr) * nb, st,
                  lx * sz * nb);
    const dim3 g(unsigned(l.npan), unsigned(B));
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPanel) {
        const int nrr = std::min(kMaxRhsPanel, nrhs - r0);
        const size_t lds = (size_t(l.maxc_pan) * nrr + kP * kP) * sizeof(T);
#define SPCHOL_FWDSN(NRV)                                                                      \
    hipLaunchKernelGGL((k_fwd_sn<T, NRV, SOA>), g, dim3(SnThreadsF<T>::value), lds, st, D->sn,   \
                       D->slv_pan + l.pan0, r0, D->gptr, D->gidx, L, P->Lsize, as<T>(N->dinv),   \
                       P->dinv_size, as<T>(N->wsc->y), as<T>(N->wsc->u), P->n, fvsize, nrhs, active)
        if (nrr == 1) SPCHOL_FWDSN(1);
        else if (nrr == 2) SPCHOL_FWDSN(2);
        else if (nrr == 3) SPCHOL_FWDSN(3);
        else SPCHOL_FWDSN(4);
#undef SPCHOL_FWDSN
    }
    N->prof.end(st);
}

template <typename T, bool SOA>
void sn_backward(const SLaunch &l, const sc_plan *P, sc_numeric *N, int nrhs,
                 const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    const T *L = static_cast<const T *>(N->L);
    const int B = N->batch;
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    double f = 0.0, wds = 0.0, dw = 0.0, vw = 0.0, lx = 0.0;
    for (const SPanel &pp : l.panels) {
        f += pp.flops;
        wds += pp.words;
        dw += pp.dwords;
        vw += pp.vwords;
        lx += pp.lx;
    }
    N->prof.begin(KK_BwdPanel, f * nr * nb, ((wds + dw) * sz + vw * sz * nr) * nb, st,
                  lx * sz * nb);
    const dim3 g(unsigned(l.npan), unsigned(B));
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPanel) {
        const int nrr = std::min(kMaxRhsPanel, nrhs - r0);
        const size_t lds = size_t(l.maxc_pan) * nrr * sizeof(T);
#define SPCHOL_BWDSN(NRV)                                                                      \
    hipLaunchKernelGGL((k_bwd_sn<T, NRV, SOA>), g, dim3(kSnThreads), lds, st, D->sn,             \
                       D->slv_pan + l.pan0, r0, D->rows, L, P->Lsize, as<T>(N->dinv),            \
                       P->dinv_size, as<T>(N->wsc->y), P->n, nrhs, active)
        if (nrr == 1) SPCHOL_BWDSN(1);
        else if (nrr == 2) SPCHOL_BWDSN(2);
        else if (nrr == 3) SPCHOL_BWDSN(3);
        else SPCHOL_BWDSN(4);
#undef SPCHOL_BWDSN
    }
    N->prof.end(st);
}

// Supernodes of a level with whole-block inverses: the panel-solved ones
// (all at most kXMaxW wide) or the others of a level with few of them; the
// front vectors are gathered beforehand.  `list` holds cnt supernodes at
// most maxw wide with at most maxc rows; xw and lx are the scalars of X and
// L21 read per sweep and the exact entries of L (per matrix).
struct XSet {
    const int32_t *list;
    int32_t cnt, maxw, maxc;
    double xw, lx;
};
inline XSet xset_panels(const SLaunch &l, const DevPlan *D) {
    return XSet{D->slv_pan + l.pan0, l.npan, l.maxw_pan, l.maxc_pan, l.x_words, l.x_lx};
}
inline XSet xset_small(const SLaunch &l, const DevPlan *D) {
    return XSet{D->slv_small + l.all0, l.nall, l.maxw_small, l.maxc_small, l.xs_words, l.xs_lx};
}

template <typename T, bool SOA>
void x_forward(const XSet &xs, const sc_plan *P, sc_numeric *N, int nrhs,
               const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    const T *L = static_cast<const T *>(N->L);
    const T *X = static_cast<const T *>(N->xinv);
    const int B = N->batch;
    const int64_t fvsize = int64_t(P->rows.size());
    Profiler &prof = N->prof;
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    prof.begin(KK_FwdPanel, 2.0 * xs.xw * nr * nb, xs.xw * sz * nb, st, xs.lx * sz * nb);
    const dim3 gy(unsigned((xs.maxw + 63) / 64), unsigned(xs.cnt), unsigned(B));
    const dim3 gu(unsigned((xs.maxc + 256 * kFxRows - 1) / (256 * kFxRows)), unsigned(xs.cnt), unsigned(B));
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
        const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_FX(NRV)                                                                          \
    do {                                                                                        \
        hipLaunchKernelGGL((k_fx_y<T, NRV, SOA>), gy, dim3(256), 0, st, D->sn, xs.list, r0,      \
                           D->xoff, X, P->xsize, as<T>(N->wsc->y), as<T>(N->wsc->u), P->n,      \
                           fvsize, nrhs, active);                                               \
        hipLaunchKernelGGL((k_fx_u<T, NRV, SOA>), gu, dim3(256), 0, st, D->sn, xs.list, r0, L,   \
                           P->Lsize, as<T>(N->wsc->y), as<T>(N->wsc->u), P->n, fvsize, nrhs,    \
                           active);                                                             \
    } while (0)
        if (nrr == 1) SPCHOL_FX(1);
        else if (nrr == 2) SPCHOL_FX(2);
        else if (nrr == 3) SPCHOL_FX(3);
        else SPCHOL_FX(4);
#undef SPCHOL_FX
    }
    prof.end(st);
}

template <typename T, bool SOA>
void x_backward(const XSet &xs, const sc_plan *P, sc_numeric *N, int nrhs,
                const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    const T *L = static_cast<const T *>(N->L);
    const T *X = static_cast<const T *>(N->xinv);
    const int B = N->batch;
    const int64_t fvsize = int64_t(P->rows.size());
    Profiler &prof = N->prof;
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    prof.begin(KK_BwdPanel, 2.0 * xs.xw * nr * nb, xs.xw * sz * nb, st, xs.lx * sz * nb);
    const dim3 g(unsigned((xs.maxw + 63) / 64), unsigned(xs.cnt), unsigned(B));
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
        const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_BX(NRV)                                                                          \
    do {                                                                                        \
        hipLaunchKernelGGL((k_bx_t<T, NRV, SOA>), g, dim3(256), 0, st, D->sn, xs.list, r0,       \
                           D->rows, L, P->Lsize, as<T>(N->wsc->y), as<T>(N->wsc->u), P->n,      \
                           fvsize, nrhs, active);                                               \
        hipLaunchKernelGGL((k_bx_x<T, NRV, SOA>), g, dim3(256), 0, st, D->sn, xs.list, r0,       \
                           D->xoff, X, P->xsize, as<T>(N->wsc->y), as<T>(N->wsc->u), P->n,      \
                           fvsize, nrhs, active);                                               \
    } while (0)
        if (nrr == 1) SPCHOL_BX(1);
        else if (nrr == 2) SPCHOL_BX(2);
        else if (nrr == 3) SPCHOL_BX(3);
        else SPCHOL_BX(4);
#undef SPCHOL_BX
    }
    prof.end(st);
}

// Panel-solved supernodes of a level with whole-block inverses: the gather
// of their front vectors, then the products.
template <typename T, bool SOA>
void x_forward_panels(const SLaunch &l, const sc_plan *P, sc_numeric *N, int nrhs,
                      const int32_t *active, hipStream_t st) {
    const DevPlan *D = P->dev;
    launch_gather_rows<T, SOA>(D->xg_q + l.xg0, D->xg_y + l.xg0, l.nxg, l.vw_xg, l.ib_xg, P, N,
                               nrhs, active, st);
    x_forward<T, SOA>(xset_panels(l, D), P, N, nrhs, active, st);
}

// Batch-interleaved solve (groups of 64 matrices, lane = matrix).
template <typename T>
hipError_t solve_soa(const sc_plan *P, sc_numeric *N, const double *bin, double *b,
                     int32_t nrhs, int64_t ldb, hipStream_t st, const int32_t *active) {
    DevPlan *D = P->dev;
    const int B = N->batch;
    const unsigned G = unsigned((B + 63) / 64);
    const int64_t fvsize = int64_t(P->rows.size());
    const T *Ls = static_cast<const T *>(N->Ls);
    Profiler &prof = N->prof;
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    if (!N->ls_ok) {  // normally made during the factorization
        const hipError_t e = spchol_to_soa_run(P, N, st);
        if (e != hipSuccess) return e;
    }
    const dim3 pgrid(unsigned((P->n + 63) / 64), G);
    prof.begin(KK_Perm, 0.0, nb * nr * (8.0 + sz) * double(P->n) + 4.0 * double(P->n), st);
    hipLaunchKernelGGL(k_perm_in_soa<T>, pgrid, dim3(256), 0, st, D->pinv, bin, ldb, as<T>(N->wsc->y), P->n,
                       nrhs, B);
    prof.end(st);
    // top levels with few supernodes: one lane per row (segment kernels)
    const int32_t segmax = P->opt.soa_seg_max == 0 ? kSoaSegMax : P->opt.soa_seg_max;
    auto by_rows = [&](const SLaunch &l) { return segmax > 0 && int64_t(l.nall) * G <= segmax; };
    // bottom levels as whole subtrees: up to the highest level K such that
    // every level up to K runs the interleaved level kernels and the
    // subtrees closed at K still give enough (subtree, group) waves
    const int32_t fmin = P->opt.soa_subtree_min == 0 ? kSoaSubtreeMin : P->opt.soa_subtree_min;
    int32_t K = -1;
    if (fmin > 0)
        for (int32_t k = 0; k < int32_t(D->fz_roots.size()); k++) {
            const SLaunch &l = D->ssched[k];
            if (by_rows(l) || l.npan > 0 || (N->xinv && l.xsmall) ||
                int64_t(D->fz_roots[k]) * G < fmin)
                break;
            K = k;
        }
    // algorithmic work of the fused launches (the levels they cover)
    double ff = 0.0, fw = 0.0, fv = 0.0, fi = 0.0, fx = 0.0;
    for (int32_t k = 0; k <= K; k++) {
        const SLaunch &l = D->ssched[k];
        ff += l.f_diag + l.f_rows;
        fw += l.w_diag + l.w_rows;
        fv += l.vw_diag + l.vw_rows + l.vw_gather;
        fi += l.ib_diag + l.ib_rows + l.ib_gather;
        fx += l.lx_diag + l.lx_rows;
    }
    if (K >= 0) {
        prof.begin(KK_Fwd, ff * nr * nb, (fw * sz + (fv * sz + fi) * nr) * nb, st, fx * sz * nb);
        for (int r0 = 0; r0 < nrhs; r0 += 4) {
            const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_SUBF(NRV)                                                                         \
    hipLaunchKernelGGL((k_fwd_soa_subtree<T, NRV>), dim3(unsigned(D->fz_roots[K]), G), dim3(64), \
                       0, st, D->sn, D->fz_ptr[K], D->fz_sn[K], D->gptr, D->gidx, Ls, P->Lsize,  \
                       as<T>(N->wsc->y), as<T>(N->wsc->u), P->n, fvsize, nrhs, r0)
            if (nrr == 1) SPCHOL_SUBF(1);
            else if (nrr == 2) SPCHOL_SUBF(2);
            else if (nrr == 3) SPCHOL_SUBF(3);
            else SPCHOL_SUBF(4);
#undef SPCHOL_SUBF
        }
        prof.end(st);
    }
    for (const SLaunch &l : D->ssched) {
        if (l.level <= K) continue;  // in the subtrees above
        launch_gather<T, true>(l, P, N, nrhs, nullptr, st);
        const bool xsm = N->xinv && l.xsmall;
        if (xsm) {
            x_forward<T, true>(xset_small(l, D), P, N, nrhs, nullptr, st);
        } else if (by_rows(l)) {
            classes_forward<T, true>(l, P, N, nrhs, nullptr, st);
        } else if (l.nall > 0) {
            prof.begin(KK_Fwd, l.f_diag * nr * nb, (l.w_diag * sz + (l.vw_diag * sz + l.ib_diag) * nr) * nb, st, l.lx_diag * sz * nb);
            for (int r0 = 0; r0 < nrhs; r0 += 4) {
                const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_SOAF(NRV)                                                                        \
    hipLaunchKernelGGL((k_fwd_soa_diag<T, NRV>), dim3(unsigned(l.nall), G), dim3(64), 0, st,     \
                       D->sn, D->slv_small + l.all0, D->gptr, D->gidx, Ls, P->Lsize, as<T>(N->wsc->y),   \
                       as<T>(N->wsc->u), P->n, fvsize, nrhs, r0)
                if (nrr == 1) SPCHOL_SOAF(1);
                else if (nrr == 2) SPCHOL_SOAF(2);
                else if (nrr == 3) SPCHOL_SOAF(3);
                else SPCHOL_SOAF(4);
#undef SPCHOL_SOAF
            }
            prof.end(st);
        }
        if (l.nit > 0 && !by_rows(l) && !xsm) {
            prof.begin(KK_FwdRows, l.f_rows * nr * nb, (l.w_rows * sz + (l.vw_rows * sz + l.ib_rows) * nr) * nb, st, l.lx_rows * sz * nb);
            for (int r0 = 0; r0 < nrhs; r0 += 4) {
                const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_SOAF(NRV)                                                                        \
    hipLaunchKernelGGL((k_fwd_soa_rows<T, NRV>), dim3(unsigned(l.nit), G), dim3(64), 0, st,      \
                       D->sn, D->soa_it_s + l.it0, D->soa_it_r0 + l.it0, D->gptr, D->gidx, Ls,  \
                       P->Lsize, as<T>(N->wsc->y), as<T>(N->wsc->u), P->n, fvsize, nrhs, r0)
                if (nrr == 1) SPCHOL_SOAF(1);
                else if (nrr == 2) SPCHOL_SOAF(2);
                else if (nrr == 3) SPCHOL_SOAF(3);
                else SPCHOL_SOAF(4);
#undef SPCHOL_SOAF
            }
            prof.end(st);
        }
        if (l.npan > 0) {
            if (N->xinv && l.xpan) x_forward_panels<T, true>(l, P, N, nrhs, nullptr, st);
            else if (sn_fits<T>(l, N, nrhs)) sn_forward<T, true>(l, P, N, nrhs, nullptr, st);
            else panels_forward<T, true>(l, P, N, nrhs, nullptr, st);
        }
    }
    for (auto it = D->ssched.rbegin(); it != D->ssched.rend(); ++it) {
        const SLaunch &l = *it;
        if (l.level <= K) {  // the subtrees, once, after the levels above them
            if (l.level == K) {
                prof.begin(KK_Bwd, ff * nr * nb, (fw * sz + (fv * sz + fi) * nr) * nb, st, fx * sz * nb);
                for (int r0 = 0; r0 < nrhs; r0 += 4) {
                    const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_SUBB(NRV)                                                                         \
    hipLaunchKernelGGL((k_bwd_soa_subtree<T, NRV>), dim3(unsigned(D->fz_roots[K]), G), dim3(64), \
                       0, st, D->sn, D->fz_ptr[K], D->fz_sn[K], D->rows, Ls, P->Lsize,           \
                       as<T>(N->wsc->y), as<T>(N->wsc->ps), P->soa_psize, P->n, nrhs, r0)
                    if (nrr == 1) SPCHOL_SUBB(1);
                    else if (nrr == 2) SPCHOL_SUBB(2);
                    else if (nrr == 3) SPCHOL_SUBB(3);
                    else SPCHOL_SUBB(4);
#undef SPCHOL_SUBB
                }
                prof.end(st);
            }
            continue;
        }
        if (l.npan > 0) {
            if (N->xinv && l.xpan) x_backward<T, true>(xset_panels(l, D), P, N, nrhs, nullptr, st);
            else if (sn_fits<T>(l, N, nrhs)) sn_backward<T, true>(l, P, N, nrhs, nullptr, st);
            else panels_backward<T, true>(l, P, N, nrhs, nullptr, st);
        }
        if (N->xinv && l.xsmall) {
            x_backward<T, true>(xset_small(l, D), P, N, nrhs, nullptr, st);
            continue;
        }
        if (by_rows(l)) {
            classes_backward<T, true>(l, P, N, nrhs, nullptr, st);
            continue;
        }
        if (l.nit > 0) {
            prof.begin(KK_BwdRows, l.f_rows * nr * nb, (l.w_rows * sz + (l.vw_rows * sz + l.ib_rows) * nr) * nb, st, l.lx_rows * sz * nb);
            for (int r0 = 0; r0 < nrhs; r0 += 4) {
                const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_SOAB(NRV)                                                                        \
    hipLaunchKernelGGL((k_bwd_soa_rows<T, NRV>), dim3(unsigned(l.nit), G), dim3(64), 0, st,      \
                       D->sn, D->soa_it_s + l.it0, D->soa_it_r0 + l.it0, D->rows, Ls, P->Lsize, \
                       as<T>(N->wsc->y), as<T>(N->wsc->ps), P->soa_psize, P->n, nrhs, r0)
                if (nrr == 1) SPCHOL_SOAB(1);
                else if (nrr == 2) SPCHOL_SOAB(2);
                else if (nrr == 3) SPCHOL_SOAB(3);
                else SPCHOL_SOAB(4);
#undef SPCHOL_SOAB
            }
            prof.end(st);
        }
        if (l.nall > 0) {
            prof.begin(KK_Bwd, l.f_diag * nr * nb, (l.w_diag * sz + (l.vw_diag * sz + l.ib_diag) * nr) * nb, st, l.lx_diag * sz * nb);
            for (int r0 = 0; r0 < nrhs; r0 += 4) {
                const int nrr = std::min(4, nrhs - r0);
#define SPCHOL_SOAB(NRV)                                                                        \
    hipLaunchKernelGGL((k_bwd_soa_diag<T, NRV>), dim3(unsigned(l.nall), G), dim3(64), 0, st,     \
                       D->sn, D->slv_small + l.all0, Ls, P->Lsize, as<T>(N->wsc->y), as<T>(N->wsc->ps),           \
                       P->soa_psize, P->n, nrhs, r0)
                if (nrr == 1) SPCHOL_SOAB(1);
                else if (nrr == 2) SPCHOL_SOAB(2);
                else if (nrr == 3) SPCHOL_SOAB(3);
                else SPCHOL_SOAB(4);
#undef SPCHOL_SOAB
            }
            prof.end(st);
        }
    }
    prof.begin(KK_Perm, 0.0, nb * nr * (8.0 + sz) * double(P->n) + 4.0 * double(P->n), st);
    hipLaunchKernelGGL(k_perm_out_soa<T>, pgrid, dim3(256), 0, st, D->pinv, as<T>(N->wsc->y), b, ldb, P->n,
                       nrhs, B, active);
    prof.end(st);
    return hipGetLastError();
}

template <typename T>
hipError_t solve_impl(const sc_plan *P, sc_numeric *N, const double *bin, double *b,
                      int32_t nrhs, int64_t ldb, hipStream_t st, const int32_t *active) {
    DevPlan *D = P->dev;
    const int B = N->batch;
    Profiler &prof = N->prof;
    const double sz = double(sizeof(T)), nr = double(nrhs), nb = double(B);
    const dim3 pgrid(unsigned((P->n + 255) / 256), unsigned(B));
    prof.begin(KK_Perm, 0.0, nb * nr * (8.0 + sz) * double(P->n) + 4.0 * double(P->n), st);
    hipLaunchKernelGGL(k_perm_in<T>, pgrid, dim3(256), 0, st, D->perm, bin, ldb, as<T>(N->wsc->y), P->n, nrhs,
                       active);
    prof.end(st);
    // forward: levels ascending
    for (const SLaunch &l : D->ssched) {
        launch_gather<T, false>(l, P, N, nrhs, active, st);
        if (N->xinv && l.xsmall) x_forward<T, false>(xset_small(l, D), P, N, nrhs, active, st);
        else classes_forward<T, false>(l, P, N, nrhs, active, st);
        if (l.npan > 0) {
            if (N->xinv && l.xpan) x_forward_panels<T, false>(l, P, N, nrhs, active, st);
            else if (sn_fits<T>(l, N, nrhs)) sn_forward<T, false>(l, P, N, nrhs, active, st);
            else panels_forward<T, false>(l, P, N, nrhs, active, st);
        }
    }
    // backward: levels descending
    for (auto it = D->ssched.rbegin(); it != D->ssched.rend(); ++it) {
        const SLaunch &l = *it;
        if (l.npan > 0) {
            if (N->xinv && l.xpan) x_backward<T, false>(xset_panels(l, D), P, N, nrhs, active, st);
            else if (sn_fits<T>(l, N, nrhs)) sn_backward<T, false>(l, P, N, nrhs, active, st);
            else panels_backward<T, false>(l, P, N, nrhs, active, st);
        }
        if (N->xinv && l.xsmall) x_backward<T, false>(xset_small(l, D), P, N, nrhs, active, st);
        else classes_backward<T, false>(l, P, N, nrhs, active, st);
    }
    prof.begin(KK_Perm, 0.0, nb * nr * (8.0 + sz) * double(P->n) + 4.0 * double(P->n), st);
    hipLaunchKernelGGL(k_perm_out<T>, pgrid, dim3(256), 0, st, D->pinv, as<T>(N->wsc->y), b, ldb, P->n, nrhs,
                       active);
    prof.end(st);
    return hipGetLastError();
}

}  // namespace

// Exact entries of L (amalgamation padding excluded) in column j with row
// index below rlim.
static double exact_rows_below(const sc_plan *P, int32_t j, int64_t rlim) {
    const int64_t t = int64_t(std::upper_bound(P->ffirst.begin(), P->ffirst.end(), j) -
                              P->ffirst.begin()) - 1;
    const int32_t *a = P->frows.data() + P->frowptr[t] + (j - P->ffirst[t]);
    const int32_t *b = P->frows.data() + P->frowptr[t + 1];
    return double(std::lower_bound(a, b, rlim) - a);
}

// Solve schedule per level, with the algorithmic work of each launch (per
// matrix; vector bytes per right-hand side).
void spchol_build_solve_schedule(const sc_plan *P, DevPlan *D) {
    D->ssched.clear();
    auto l_exact = [&](const SnDesc &d, int32_t j0, int32_t j1) {
        double c = 0.0;
        for (int32_t j = d.first + j0; j < d.first + j1; j++) c += double(P->colcount[j]);
        return c;
    };
    for (int32_t l = 0; l < P->nlevels; l++) {
        SLaunch s{};
        s.level = l;
        for (int k = 0; k < kSolveClasses; k++) {
            SClass &cl = s.cls[k];
            cl.list0 = P->slv_cls_ptr[size_t(l) * kSolveClasses + k];
            cl.n = P->slv_cls_ptr[size_t(l) * kSolveClasses + k + 1] - cl.list0;
            for (int32_t e = cl.list0; e < cl.list0 + cl.n; e++) {
                const SnDesc &d = P->sn[P->slv_small[e]];
                const double lw = double(d.c) * d.w - double(d.w) * (d.w - 1) / 2;
                cl.flops += 2.0 * lw;
                cl.words += lw;
                // the front vector in and out and its row indices
                cl.vwords += 2.0 * d.c;
                cl.ibytes += 4.0 * d.c;
                cl.lx += l_exact(d, 0, d.w);
            }
        }
        s.all0 = P->slv_cls_ptr[size_t(l) * kSolveClasses];
        s.nall = P->slv_cls_ptr[size_t(l + 1) * kSolveClasses] - s.all0;
        s.it0 = P->soa_it_ptr[l];
        s.nit = P->soa_it_ptr[l + 1] - s.it0;
        s.grow0 = P->grow_ptr[l];
        s.ngrow = P->grow_ptr[l + 1] - s.grow0;
        for (int32_t q = s.grow0; q < s.grow0 + s.ngrow; q++) {
            const int32_t row = P->grow_q[q];
            s.vw_gather += 1.0 + (P->grow_y[q] >= 0 ? 1.0 : 0.0) +
                           double(P->gptr[row + 1] - P->gptr[row]);
            s.ib_gather += 12.0 + 4.0 * double(P->gptr[row + 1] - P->gptr[row]);
        }
        for (int32_t e = s.all0; e < s.all0 + s.nall; e++) {
            const SnDesc &d = P->sn[P->slv_small[e]];
            const double tri = double(d.w) * (d.w + 1) / 2, rect = double(d.m) * d.w;
            s.f_diag += 2.0 * tri;
            s.w_diag += tri;
            s.vw_diag += 2.0 * d.w;
            s.ib_diag += 4.0 * d.w;
            s.f_rows += 2.0 * rect;
            s.w_rows += rect;
            s.vw_rows += 2.0 * d.m;
            s.ib_rows += 4.0 * d.m;
            double dg = 0.0;
            for (int32_t j = d.first; j < d.first + d.w; j++)
                dg += exact_rows_below(P, j, int64_t(d.first) + d.w);
            s.lx_diag += dg;
            s.lx_rows += l_exact(d, 0, d.w) - dg;
        }
        s.pan0 = P->slv_pan_ptr[l];
        s.npan = P->slv_pan_ptr[l + 1] - s.pan0;
        s.maxc_pan = P->slv_pan_maxc[l];
        s.maxw_pan = P->slv_pan_maxw[l];
        s.xpan = P->slv_pan_x[l] != 0;
        s.xsmall = P->slv_small_x[l] != 0;
        for (int32_t e = s.all0; s.xsmall && e < s.all0 + s.nall; e++) {
            const SnDesc &d = P->sn[P->slv_small[e]];
            s.maxw_small = std::max(s.maxw_small, d.w);
            s.maxc_small = std::max(s.maxc_small, d.c);
            s.xs_words += double(d.w) * (d.w + 1) / 2 + double(d.c - d.w) * d.w;
            s.xs_lx += l_exact(d, 0, d.w);
        }
        s.xg0 = P->xg_ptr[l];
        s.nxg = P->xg_ptr[l + 1] - s.xg0;
        for (int32_t q = s.xg0; q < s.xg0 + s.nxg; q++) {
            const int32_t row = P->xg_q[q];
            s.vw_xg += 1.0 + (P->xg_y[q] >= 0 ? 1.0 : 0.0) + double(P->gptr[row + 1] - P->gptr[row]);
            s.ib_xg += 12.0 + 4.0 * double(P->gptr[row + 1] - P->gptr[row]);
        }
        for (int32_t e = s.pan0; e < s.pan0 + s.npan; e++) {
            const SnDesc &d = P->sn[P->slv_pan[e]];
            s.vw_pan += 2.0 * d.c;
            s.ib_pan += 4.0 * d.c;
            s.x_words += double(d.w) * (d.w + 1) / 2 + double(d.c - d.w) * d.w;
            s.x_lx += l_exact(d, 0, d.w);
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
                pp.bwd_chunks = std::max<int64_t>(pp.bwd_chunks, (below + kSolveChunk - 1) / kSolveChunk);
                const double lw = double(below) * kb;
                pp.flops += 2.0 * lw + 2.0 * kb * kb;
                pp.words += lw;
                pp.vwords += below + 2.0 * kb;
                pp.dwords += double(kb) * kb;
                pp.lx += l_exact(d, c0, c0 + kb);
            }
            s.panels.push_back(pp);
        }
        D->ssched.push_back(s);
    }
}

// Subtree lists of the fused bottom-level solve, for every level K up to
// which no level has panel-solved supernodes (host work once per plan, then
// uploaded).
hipError_t spchol_build_subtrees(const sc_plan *P, DevPlan *D) {
    int32_t kmax = -1;
    for (const SLaunch &l : D->ssched) {
        if (l.npan > 0) break;
        kmax = l.level;
    }
    D->fz_ptr.assign(size_t(kmax + 1), nullptr);
    D->fz_sn.assign(size_t(kmax + 1), nullptr);
    D->fz_roots.assign(size_t(kmax + 1), 0);
    std::vector<int32_t> ptr, order;
    for (int32_t K = 0; K <= kmax; K++) {
        ptr.assign(1, 0);
        order.clear();
        for (int32_t s = 0; s < P->ns; s++) {
            const SnDesc &d = P->sn[s];
            if (d.level > K || (d.parent >= 0 && P->sn[d.parent].level <= K)) continue;
            // postorder of the subtree of s: children (in list order) first
            std::vector<std::pair<int32_t, int32_t>> st{{s, P->sn[s].chbeg}};
            while (!st.empty()) {
                auto &top = st.back();
                const SnDesc &t = P->sn[top.first];
                if (top.second < t.chend) {
                    const int32_t ch = P->chlist[top.second++];
                    st.push_back({ch, P->sn[ch].chbeg});
                } else {
                    order.push_back(top.first);
                    st.pop_back();
                }
            }
            ptr.push_back(int32_t(order.size()));
        }
        D->fz_roots[K] = int32_t(ptr.size() - 1);
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&D->fz_ptr[K]), ptr.size() * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void **>(&D->fz_sn[K]),
                          std::max<size_t>(order.size(), 1) * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(D->fz_ptr[K], ptr.data(), ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess && !order.empty())
            e = hipMemcpy(D->fz_sn[K], order.data(), order.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int NR>
void sn_lds_limits() {
    const int dyn = g_max_lds - int(sn_static_lds<T>(NR));
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_sn<T, NR, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, g_max_lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_sn<T, NR, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, g_max_lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bwd_sn<T, NR, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bwd_sn<T, NR, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

hipError_t spchol_solve_init() {
    sn_lds_limits<double, 1>();
    sn_lds_limits<double, 2>();
    sn_lds_limits<double, 3>();
    sn_lds_limits<double, 4>();
    sn_lds_limits<float, 1>();
    sn_lds_limits<float, 2>();
    sn_lds_limits<float, 3>();
    sn_lds_limits<float, 4>();
    (void)hipGetLastError();  // an attribute the runtime refuses keeps the default
    return hipSuccess;
}

template <typename T>
hipError_t to_soa_impl(const sc_plan *P, sc_numeric *N, hipStream_t st) {
    const DevPlan *D = P->dev;
    const int B = N->batch;
    const unsigned G = unsigned((B + 63) / 64);
    // the levels solved with whole-block inverses read L, not the copy
    const size_t nch = (N->xinv ? P->soa_chunks_x : P->soa_chunks).size();
    N->prof.begin(KK_ToSoa, 0.0, 2.0 * double(sizeof(T)) * double(B) * double(nch) * kSoaChunk, st);
    if (nch > 0)
        hipLaunchKernelGGL(k_to_soa<T>, dim3(unsigned(nch), G), dim3(256), 0, st,
                           static_cast<const T *>(N->L), P->Lsize,
                           N->xinv ? D->soa_chunks_x : D->soa_chunks, B, static_cast<T *>(N->Ls));
    N->prof.end(st);
    N->ls_ok = true;
    return hipGetLastError();
}

hipError_t spchol_to_soa_run(const sc_plan *P, sc_numeric *N, hipStream_t st) {
    if (N->dtype == SC_F64) return to_soa_impl<double>(P, N, st);
    return to_soa_impl<float>(P, N, st);
}

hipError_t spchol_dinv_run(const sc_plan *P, sc_numeric *N, hipStream_t st, int parts) {
    if (N->dtype == SC_F64) return dinv_impl<double>(P, N, st, parts);
    return dinv_impl<float>(P, N, st, parts);
}

hipError_t spchol_solve_run(const sc_plan *P, sc_numeric *N, double *b, int32_t nrhs,
                            int64_t ldb, hipStream_t st, const int32_t *active,
                            const double *bin) {
    if (!bin) bin = b;
    if (N->soa) {
        if (N->dtype == SC_F64) return solve_soa<double>(P, N, bin, b, nrhs, ldb, st, active);
        return solve_soa<float>(P, N, bin, b, nrhs, ldb, st, active);
    }
    if (N->dtype == SC_F64) return solve_impl<double>(P, N, bin, b, nrhs, ldb, st, active);
    return solve_impl<float>(P, N, bin, b, nrhs, ldb, st, active);
}
