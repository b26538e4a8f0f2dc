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

// Column j of a front: L columns live in the c x w block, update columns in
// the m x m block.  Returns a pointer p with the front entry (i, j) at p[i]
// (only rows i >= j are ever touched for update columns).
template <typename T>
__device__ inline T *front_col(T *Lb, T *Ub, int c, int w, int m, int j) {
    return j < w ? Lb + int64_t(j) * c : Ub + int64_t(j - w) * m - w;
}

// Right-looking Cholesky of the first w columns of a c x c front held in
// LDS (column-major, leading dimension ld), including the Schur update of
// the trailing block.  A pivot that fails d > 0 is recorded (1-based step,
// smallest wins) and replaced by 1 so no NaN spreads.
template <typename T>
__device__ void lds_partial_chol(T *F, int ld, int c, int w, int col0,
                                 int32_t *info_b) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int j = 0; j < w; j++) {
        T djj = F[j * ld + j];
        __syncthreads();
        const bool bad = !(djj > T(0));
        if (bad) djj = T(1);
        const T ljj = dsqrt(djj);
        if (tid == 0) {
            F[j * ld + j] = ljj;
            if (bad) atomicMin(info_b, col0 + j + 1);
        }
        for (int i = j + 1 + tid; i < c; i += nt) F[j * ld + i] /= ljj;
        __syncthreads();
        const int r = c - j - 1;
        const T *cj = F + j * ld + j + 1;
        for (int e = tid; e < r * r; e += nt) {
            const int tt = e / r, ii = e - tt * r;
            if (ii >= tt) F[(j + 1 + tt) * ld + j + 1 + ii] -= cj[ii] * cj[tt];
        }
        __syncthreads();
    }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// small fronts: the whole front in LDS, one workgroup per supernode
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_front_small(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int32_t *__restrict__ relmap, const int32_t *__restrict__ chlist,
    const int64_t *__restrict__ acolptr, const int32_t *__restrict__ aoff,
    const int64_t *__restrict__ avidx, const double *__restrict__ vals,
    int64_t ldv, T *__restrict__ L, int64_t Lsize, T *__restrict__ U,
    int64_t Usize, int32_t *__restrict__ info) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *F = reinterpret_cast<T *>(smem_raw);
    const int s = list[blockIdx.x];
    const int b = blockIdx.y;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w, m = d.m;
    const int tid = threadIdx.x, nt = blockDim.x;
    L += int64_t(b) * Lsize;
    U += int64_t(b) * Usize;
    vals += int64_t(b) * ldv;

    for (int e = tid; e < c * c; e += nt) F[e] = T(0);
    __syncthreads();
    const int64_t a0 = acolptr[d.first], a1 = acolptr[d.first + w];
    for (int64_t e = a0 + tid; e < a1; e += nt) F[aoff[e]] = T(vals[avidx[e]]);
    for (int q = d.chbeg; q < d.chend; q++) {
        const SnDesc cd = sn[chlist[q]];
        const int32_t *rm = relmap + cd.relptr;
        const T *Uc = U + cd.uoff;
        const int mc = cd.m;
        __syncthreads();
        for (int e = tid; e < mc * mc; e += nt) {
            const int j = e / mc, i = e - j * mc;
            if (i >= j) F[rm[j] * c + rm[i]] += Uc[e];
        }
    }
    __syncthreads();
    lds_partial_chol(F, c, c, w, d.first, info + b);
    T *Ls = L + d.loff;
    for (int e = tid; e < c * w; e += nt) {
        const int j = e / c, i = e - j * c;
        Ls[e] = i >= j ? F[e] : T(0);
    }
    T *Us = U + d.uoff;
    for (int e = tid; e < m * m; e += nt) {
        const int j = e / m, i = e - j * m;
        if (i >= j) Us[e] = F[(w + j) * c + w + i];
    }
}

// ---------------------------------------------------------------------------
// large fronts: assembly, one workgroup per target column
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_assemble(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int64_t *__restrict__ colstart, int nlist,
    const int32_t *__restrict__ relmap, const int32_t *__restrict__ chlist,
    const int64_t *__restrict__ acolptr, const int32_t *__restrict__ aoff,
    const int64_t *__restrict__ avidx, const double *__restrict__ vals,
    int64_t ldv, T *__restrict__ L, int64_t Lsize, T *__restrict__ U,
    int64_t Usize) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *col = reinterpret_cast<T *>(smem_raw);
    const int64_t g = blockIdx.x;
    int lo = 0, hi = nlist - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (colstart[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const int s = list[lo];
    const int tj = int(g - colstart[lo]);
    const int b = blockIdx.y;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w, m = d.m;
    const int tid = threadIdx.x, nt = blockDim.x;
    L += int64_t(b) * Lsize;
    U += int64_t(b) * Usize;
    vals += int64_t(b) * ldv;

    for (int i = tid; i < c; i += nt) col[i] = T(0);
    __syncthreads();
    if (tj < w) {
        const int j = d.first + tj;
        const int64_t base = int64_t(tj) * c;
        for (int64_t e = acolptr[j] + tid; e < acolptr[j + 1]; e += nt)
            col[aoff[e] - base] = T(vals[avidx[e]]);
    }
    for (int q = d.chbeg; q < d.chend; q++) {
        const SnDesc cd = sn[chlist[q]];
        const int32_t *rm = relmap + cd.relptr;
        const int mc = cd.m;
        int l2 = 0, h2 = mc;  // first child row mapped at or below tj
        while (l2 < h2) {
            const int mid = (l2 + h2) >> 1;
            if (rm[mid] < tj) l2 = mid + 1; else h2 = mid;
        }
        __syncthreads();
        if (l2 < mc && rm[l2] == tj) {
            const T *uc = U + cd.uoff + int64_t(l2) * mc;
            for (int i = l2 + tid; i < mc; i += nt) col[rm[i]] += uc[i];
        }
    }
    __syncthreads();
    if (tj < w) {
        T *dst = L + d.loff + int64_t(tj) * c;
        for (int i = tid; i < c; i += nt) dst[i] = i >= tj ? col[i] : T(0);
    } else {
        T *dst = U + d.uoff + int64_t(tj - w) * m - w;
        for (int i = tj + tid; i < c; i += nt) dst[i] = col[i];
    }
}

// diagonal block of panel k: unblocked Cholesky in LDS
template <typename T>
__global__ __launch_bounds__(256) void k_potrf(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int k,
    T *__restrict__ L, int64_t Lsize, int32_t *__restrict__ info) {
    __shared__ T tile[kTile * kTile];
    const int s = list[blockIdx.x];
    const int b = blockIdx.y;
    const SnDesc d = sn[s];
    if (k >= d.w) return;
    const int kb = min(kTile, d.w - k);
    const int c = d.c;
    T *Lb = L + int64_t(b) * Lsize + d.loff;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < kb * kb; e += nt) {
        const int j = e / kb, i = e - j * kb;
        tile[j * kTile + i] = Lb[int64_t(k + j) * c + k + i];
    }
    __syncthreads();
    lds_partial_chol(tile, kTile, kb, kb, d.first + k, info + b);
    for (int e = tid; e < kb * kb; e += nt) {
        const int j = e / kb, i = e - j * kb;
        Lb[int64_t(k + j) * c + k + i] = i >= j ? tile[j * kTile + i] : T(0);
    }
}

// panel rows below the diagonal block: X <- X L_kk^{-T}, one row per lane.
// L_kk is read as a broadcast; the row tile is stored transposed ([t][lane])
// so that every lane hits its own LDS bank.
template <typename T>
__global__ __launch_bounds__(64) void k_trsm(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int k,
    T *__restrict__ L, int64_t Lsize) {
    __shared__ T Lkk[kTile * kTile];
    __shared__ T X[kTile * kTile];
    const int s = list[blockIdx.y];
    const int b = blockIdx.z;
    const SnDesc d = sn[s];
    if (k >= d.w) return;
    const int kb = min(kTile, d.w - k);
    const int c = d.c;
    const int r0 = k + kb + blockIdx.x * kTile;
    if (r0 >= c) return;
    T *Lb = L + int64_t(b) * Lsize + d.loff;
    const int lane = threadIdx.x;
    for (int e = lane; e < kb * kb; e += 64) {
        const int t = e / kb, j = e - t * kb;
        Lkk[j * kTile + t] = Lb[int64_t(k + t) * c + k + j];
    }
    const int r = r0 + lane;
    if (r < c)
        for (int t = 0; t < kb; t++) X[t * kTile + lane] = Lb[int64_t(k + t) * c + r];
    __syncthreads();
    if (r < c) {
        for (int j = 0; j < kb; j++) {
            T a = X[j * kTile + lane];
            const T *lj = Lkk + j * kTile;
            for (int t = 0; t < j; t++) a -= X[t * kTile + lane] * lj[t];
            X[j * kTile + lane] = a / lj[j];
        }
        for (int t = 0; t < kb; t++) Lb[int64_t(k + t) * c + r] = X[t * kTile + lane];
    }
}

// trailing update F[i, j] -= sum_t P[i, t] P[j, t] over the lower tiles of
// the trailing block, P = panel k after the TRSM.  One 64 x 64 tile per
// workgroup, four waves of 32 x 32, MFMA 16x16x4.  The MFMA's row index runs
// over matrix columns so that each lane group writes 16 consecutive rows of
// one column (column-major storage).
template <typename T>
__global__ __launch_bounds__(256) void k_syrk(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list, int k,
    T *__restrict__ L, int64_t Lsize, T *__restrict__ U, int64_t Usize) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sI = reinterpret_cast<T *>(smem_raw);  // [t][i] panel rows of tile I
    T *sJ = sI + kTile * kTile;               // [t][j] panel rows of tile J
    const int s = list[blockIdx.y];
    const int b = blockIdx.z;
    const SnDesc d = sn[s];
    if (k >= d.w) return;
    const int c = d.c, w = d.w, m = d.m;
    const int kb = min(kTile, w - k);
    const int t0 = k + kb;
    const int nrem = c - t0;
    if (nrem <= 0) return;
    const int ntl = (nrem + kTile - 1) / kTile;
    const int64_t p = blockIdx.x;
    if (p >= int64_t(ntl) * (ntl + 1) / 2) return;
    int I = int((sqrt(8.0 * double(p) + 1.0) - 1.0) * 0.5);
    while (int64_t(I) * (I + 1) / 2 > p) I--;
    while (int64_t(I + 1) * (I + 2) / 2 <= p) I++;
    const int J = int(p - int64_t(I) * (I + 1) / 2);
    const int row0 = t0 + I * kTile, col0 = t0 + J * kTile;
    T *Lb = L + int64_t(b) * Lsize + d.loff;
    T *Ub = U + int64_t(b) * Usize + d.uoff;
    const int tid = threadIdx.x;
    const int kbr = (kb + 3) & ~3;
    for (int e = tid; e < kbr * kTile; e += 256) {
        const int t = e / kTile, i = e - t * kTile;
        const bool tk = t < kb;
        const T *pc = Lb + int64_t(k + t) * c;
        sI[e] = (tk && row0 + i < c) ? pc[row0 + i] : T(0);
        sJ[e] = (tk && col0 + i < c) ? pc[col0 + i] : T(0);
    }
    __syncthreads();
    const int wv = tid >> 6, lane = tid & 63;
    const int jw = (wv & 1) * 32, iw = (wv >> 1) * 32;
    const int lk = lane >> 4, lm = lane & 15;
    typedef typename Mma<T>::acc_t acc_t;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int q = 0; q < 2; q++) acc[a][q] = Mma<T>::zero();
    for (int kk = 0; kk < kbr; kk += 4) {
        const T *rJ = sJ + (kk + lk) * kTile;
        const T *rI = sI + (kk + lk) * kTile;
        T av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; a++) av[a] = rJ[jw + 16 * a + lm];
#pragma unroll
        for (int q = 0; q < 2; q++) bv[q] = rI[iw + 16 * q + lm];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int q = 0; q < 2; q++) acc[a][q] = Mma<T>::mma(av[a], bv[q], acc[a][q]);
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int q = 0; q < 2; q++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int j = col0 + jw + 16 * a + Mma<T>::row(lk, r);
                const int i = row0 + iw + 16 * q + lm;
                if (i < c && j < c && i >= j) {
                    T *pcol = front_col(Lb, Ub, c, w, m, j);
                    pcol[i] -= acc[a][q][r];
                }
            }
}

template <typename T>
void set_lds_limits(int big) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_front_small<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_assemble<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_syrk<T>),
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
    for (int32_t l = 0; l < P->nlevels; l++) {
        const int32_t s0 = P->lvl_small_ptr[l], s1 = P->lvl_small_ptr[l + 1];
        if (s1 > s0) {
            FLaunch f{FLaunch::Small, l, 0, s0, s1 - s0, s1 - s0,
                      P->lvl_small_maxc[l] * P->lvl_small_maxc[l], 0.0, 0.0, 0.0};
            for (int32_t e = s0; e < s1; e++) {
                const SnDesc &d = P->sn[P->lvl_small[e]];
                f.flops += front_flops(d.c, d.w);
                f.words += children_words(d) + double(d.c) * d.w + double(d.m) * (d.m + 1) / 2;
                f.ibytes += a_entries(d) * 20.0;
            }
            D->fsched.push_back(f);
        }
        const int32_t b0 = P->lvl_big_ptr[l], b1 = P->lvl_big_ptr[l + 1];
        if (b1 == b0) continue;
        FLaunch fa{FLaunch::Assemble, l, 0, b0, b1 - b0, P->lvl_bigcols[l],
                   P->lvl_big_maxc[l], 0.0, 0.0, 0.0};
        for (int32_t e = b0; e < b1; e++) {
            const SnDesc &d = P->sn[P->lvl_big[e]];
            const double cw = children_words(d);
            fa.flops += cw;
            fa.words += cw + double(d.c) * d.w + double(d.m) * (d.m + 1) / 2;
            fa.ibytes += a_entries(d) * 20.0;
        }
        D->fsched.push_back(fa);
        for (int32_t k = 0; k < P->lvl_big_maxw[l]; k += kTile) {
            int64_t trsm_tiles = 0, pairs = 0;
            FLaunch fp{FLaunch::Potrf, l, k, b0, b1 - b0, b1 - b0, 0, 0.0, 0.0, 0.0};
            FLaunch ft{FLaunch::Trsm, l, k, b0, b1 - b0, 0, 0, 0.0, 0.0, 0.0};
            FLaunch fs{FLaunch::Syrk, l, k, b0, b1 - b0, 0, 2 * kTile * kTile, 0.0, 0.0, 0.0};
            for (int32_t e = b0; e < b1; e++) {
                const SnDesc &d = P->sn[P->lvl_big[e]];
                if (k >= d.w) continue;
                const int kb = std::min(kTile, d.w - k);
                const int64_t nrem = d.c - k - kb;
                const int64_t nt = (nrem + kTile - 1) / kTile;
                trsm_tiles = std::max(trsm_tiles, nt);
                pairs = std::max(pairs, nt * (nt + 1) / 2);
                const double r = double(nrem);
                fp.flops += front_flops(kb, kb);
                fp.words += double(kb) * (kb + 1);
                ft.flops += r * kb * kb;
                ft.words += 2.0 * r * kb + double(kb) * (kb + 1) / 2;
                fs.flops += double(kb) * r * (r + 1);
                fs.words += r * (r + 1) + r * kb;
            }
            ft.gridx = trsm_tiles;
            fs.gridx = pairs;
            D->fsched.push_back(fp);
            if (trsm_tiles > 0) {
                D->fsched.push_back(ft);
                D->fsched.push_back(fs);
            }
        }
    }
}

template <typename T>
hipError_t factor_impl(const sc_plan *P, sc_numeric *N, const double *vals,
                       int64_t ldv, hipStream_t st) {
    DevPlan *D = P->dev;
    T *L = static_cast<T *>(N->L);
    T *U = static_cast<T *>(N->U);
    const int B = N->batch;
    {
        const int64_t nb = (B + 255) / 256;
        hipLaunchKernelGGL(k_fill_i32, dim3(unsigned(nb)), dim3(256), 0, st,
                           N->info, int64_t(B), int32_t(INT_MAX));
    }
    for (const FLaunch &f : D->fsched)
        if (size_t(f.lds) * sizeof(T) > size_t(g_max_lds)) return hipErrorInvalidValue;
    Profiler &prof = N->prof;
    const double wsz = double(sizeof(T));
    for (const FLaunch &f : D->fsched) {
        static const int kinds[] = {KK_SmallFront, KK_Assemble, KK_Potrf, KK_Trsm, KK_Syrk};
        prof.begin(kinds[f.kind], f.flops * B, (f.words * wsz + f.ibytes) * B, st);
        switch (f.kind) {
        case FLaunch::Small:
            hipLaunchKernelGGL(k_front_small<T>, dim3(unsigned(f.gridx), B), dim3(256),
                               size_t(f.lds) * sizeof(T), st, D->sn, D->lvl_small + f.list0,
                               D->relmap, D->chlist, D->acolptr, D->aoff, D->avidx,
                               vals, ldv, L, P->Lsize, U, P->Usize, N->info);
            break;
        case FLaunch::Assemble:
            hipLaunchKernelGGL(k_assemble<T>, dim3(unsigned(f.gridx), B), dim3(256),
                               size_t(f.lds) * sizeof(T), st, D->sn, D->lvl_big + f.list0,
                               D->big_colstart + f.list0, f.nlist, D->relmap, D->chlist,
                               D->acolptr, D->aoff, D->avidx, vals, ldv, L, P->Lsize, U,
                               P->Usize);
            break;
        case FLaunch::Potrf:
            hipLaunchKernelGGL(k_potrf<T>, dim3(unsigned(f.gridx), B), dim3(256), 0, st,
                               D->sn, D->lvl_big + f.list0, f.k, L, P->Lsize, N->info);
            break;
        case FLaunch::Trsm:
            hipLaunchKernelGGL(k_trsm<T>, dim3(unsigned(f.gridx), f.nlist, B), dim3(64), 0,
                               st, D->sn, D->lvl_big + f.list0, f.k, L, P->Lsize);
            break;
        case FLaunch::Syrk:
            hipLaunchKernelGGL(k_syrk<T>, dim3(unsigned(f.gridx), f.nlist, B), dim3(256),
                               size_t(f.lds) * sizeof(T), st, D->sn, D->lvl_big + f.list0,
                               f.k, L, P->Lsize, U, P->Usize);
            break;
        }
        prof.end(st);
    }
    return hipGetLastError();
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
    if (N->dtype == SC_F64) return factor_impl<double>(P, N, vals, ldv, st);
    return factor_impl<float>(P, N, vals, ldv, st);
}
