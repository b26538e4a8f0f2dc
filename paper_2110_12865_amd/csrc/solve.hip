// Forward and backward triangular solves with the supernodal factor
// (gfx950).  y = L^{-1} P b by levels ascending, z = L^{-T} y by levels
// descending, x = P^T z.  The factor may be stored in FP64 or FP32; the
// solves always compute in FP64.
//
// Forward solve, multifrontal style: supernode s solves its diagonal block
// and produces an update vector u_s (its m update rows), which the parent
// pulls and folds into its own right-hand side and update vector.  Every
// value is written by exactly one workgroup, children are read in a fixed
// order, and no floating-point atomics are used.
// Backward solve: supernode s gathers the already final solution on its
// update rows (owned by its ancestors) and solves with L_ss^T.
#include <algorithm>

#include "device.hpp"

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_fwd(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ relmap,
    const int32_t *__restrict__ chlist, const T *__restrict__ L, int64_t Lsize,
    const double *__restrict__ B, int64_t ldb, double *__restrict__ Y,
    double *__restrict__ UV, int64_t n, int64_t relsize, int nrhs,
    const int32_t *__restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *v = reinterpret_cast<double *>(smem_raw);
    const int s = list[blockIdx.x];
    const int br = blockIdx.y;
    const int b = br / nrhs;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w, m = d.m;
    const int tid = threadIdx.x, nt = blockDim.x;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    const double *bb = B + int64_t(br) * ldb;
    double *y = Y + int64_t(br) * n;
    double *uv = UV + int64_t(br) * relsize;

    for (int i = tid; i < c; i += nt) v[i] = i < w ? bb[perm[d.first + i]] : 0.0;
    for (int q = d.chbeg; q < d.chend; q++) {
        const SnDesc cd = sn[chlist[q]];
        const int32_t *rm = relmap + cd.relptr;
        const double *uc = uv + cd.relptr;
        __syncthreads();
        for (int i = tid; i < cd.m; i += nt) {
            const int p = rm[i];
            if (p < w) v[p] -= uc[i]; else v[p] += uc[i];
        }
    }
    __syncthreads();
    for (int j = 0; j < w; j++) {
        const T *lj = Lb + int64_t(j) * c;
        const double yj = v[j] / double(lj[j]);
        __syncthreads();
        for (int i = j + 1 + tid; i < c; i += nt) {
            const double l = double(lj[i]);
            if (i < w) v[i] -= l * yj; else v[i] += l * yj;
        }
        if (tid == 0) v[j] = yj;
        __syncthreads();
    }
    for (int i = tid; i < w; i += nt) y[d.first + i] = v[i];
    for (int i = tid; i < m; i += nt) uv[d.relptr + i] = v[w + i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_bwd(
    const SnDesc *__restrict__ sn, const int32_t *__restrict__ list,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ rows,
    const T *__restrict__ L, int64_t Lsize, double *__restrict__ X,
    int64_t ldb, double *__restrict__ Y, int64_t n, int nrhs,
    const int32_t *__restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *v = reinterpret_cast<double *>(smem_raw);
    __shared__ double red[4];
    const int s = list[blockIdx.x];
    const int br = blockIdx.y;
    const int b = br / nrhs;
    if (active && !active[b]) return;
    const SnDesc d = sn[s];
    const int c = d.c, w = d.w;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6;
    const T *Lb = L + int64_t(b) * Lsize + d.loff;
    double *y = Y + int64_t(br) * n;
    double *x = X + int64_t(br) * ldb;
    const int32_t *R = rows + d.rowptr;
    for (int i = tid; i < c; i += nt) v[i] = y[i < w ? d.first + i : R[i]];
    __syncthreads();
    for (int j = w - 1; j >= 0; j--) {
        const T *lj = Lb + int64_t(j) * c;
        double t = 0.0;
        for (int i = j + 1 + tid; i < c; i += nt) t += double(lj[i]) * v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
        if (lane == 0) red[wv] = t;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int q = 0; q < (nt >> 6); q++) tot += red[q];
            v[j] = (v[j] - tot) / double(lj[j]);
        }
        __syncthreads();
    }
    for (int i = tid; i < w; i += nt) {
        y[d.first + i] = v[i];
        x[perm[d.first + i]] = v[i];
    }
}

template <typename T>
hipError_t solve_impl(const sc_plan *P, sc_numeric *N, double *b, int32_t nrhs,
                      int64_t ldb, hipStream_t st, const int32_t *active) {
    DevPlan *D = P->dev;
    for (const SLaunch &l : D->ssched)
        if (size_t(l.maxc) * sizeof(double) > size_t(g_max_lds)) return hipErrorInvalidValue;
    const T *L = static_cast<const T *>(N->L);
    const unsigned gy = unsigned(N->batch) * unsigned(nrhs);
    Profiler &prof = N->prof;
    const double sz = double(sizeof(T)), nr = double(gy);
    for (const SLaunch &l : D->ssched) {
        prof.begin(KK_Fwd, l.flops * nr, (l.words * sz + l.vbytes) * nr, st);
        hipLaunchKernelGGL(k_fwd<T>, dim3(unsigned(l.nlist), gy), dim3(256),
                           size_t(l.maxc) * sizeof(double), st, D->sn, D->lvl_sn + l.list0,
                           D->perm, D->relmap, D->chlist, L, P->Lsize, b, ldb, N->ws_y,
                           N->ws_u, P->n, P->relsize, nrhs, active);
        prof.end(st);
    }
    for (auto it = D->ssched.rbegin(); it != D->ssched.rend(); ++it) {
        const SLaunch &l = *it;
        prof.begin(KK_Bwd, l.flops * nr, (l.words * sz + l.vbytes) * nr, st);
        hipLaunchKernelGGL(k_bwd<T>, dim3(unsigned(l.nlist), gy), dim3(256),
                           size_t(l.maxc) * sizeof(double), st, D->sn, D->lvl_sn + l.list0,
                           D->perm, D->rows, L, P->Lsize, b, ldb, N->ws_y, P->n, nrhs,
                           active);
        prof.end(st);
    }
    return hipGetLastError();
}

template <typename T>
void set_solve_lds(int big) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bwd<T>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

}  // namespace

void spchol_build_solve_schedule(const sc_plan *P, DevPlan *D) {
    D->ssched.clear();
    for (int32_t l = 0; l < P->nlevels; l++) {
        SLaunch s{l, P->lvl_ptr[l], P->lvl_ptr[l + 1] - P->lvl_ptr[l], P->lvl_maxc[l],
                  0.0, 0.0, 0.0};
        for (int32_t e = s.list0; e < s.list0 + s.nlist; e++) {
            const SnDesc &d = P->sn[P->lvl_sn[e]];
            const double lw = double(d.c) * d.w - double(d.w) * (d.w - 1) / 2;
            s.flops += 2.0 * lw;
            s.words += lw;
            s.vbytes += 8.0 * (2.0 * d.c + d.m) + 4.0 * d.c;
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

hipError_t spchol_solve_run(const sc_plan *P, sc_numeric *N, double *b, int32_t nrhs,
                            int64_t ldb, hipStream_t st, const int32_t *active) {
    if (N->dtype == SC_F64) return solve_impl<double>(P, N, b, nrhs, ldb, st, active);
    return solve_impl<float>(P, N, b, nrhs, ldb, st, active);
}
