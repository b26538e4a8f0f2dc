// C ABI of libspchol: argument checks, plan upload and object lifetimes.
// The numeric work itself lives in factor.hip and solve.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "device.hpp"
#include "spchol.h"

const char *const kKernelNames[KK_Count] = {
    "front_small", "assemble", "potrf", "trsm", "syrk_mfma", "diag_inverse",
    "solve_fwd", "solve_fwd_panel", "solve_bwd", "solve_bwd_panel", "spmv_residual",
    "refine_vector", "solve_permute", "solve_gather", "solve_fwd_rows", "solve_bwd_rows",
    "solve_copy_interleaved"};

void spchol_build_factor_schedule(const sc_plan *P, DevPlan *D);
void spchol_build_solve_schedule(const sc_plan *P, DevPlan *D);
hipError_t spchol_build_subtrees(const sc_plan *P, DevPlan *D);
hipError_t spchol_solve_init();
bool spchol_nd_order(int64_t n, const int64_t *colptr, const int32_t *rowind, int32_t *perm_out);

// Static scratch of the no-allocation solve (sc_solve_noalloc): its solve
// vectors live in this file-scope device array instead of the numeric
// object's workspaces.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code `scratch` only names the host-side
// shadow of the symbol; host code reaches the array exclusively through the
// address hipGetSymbolAddress returns for the current device, kept per
// device in g_scratch_dev at the device's set-up (ensure_device).
static __device__ __align__(256) unsigned char scratch[SC_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_upload_mutex;
bool g_kernels_ready[64] = {};
void *g_scratch_dev[64] = {};  // device address of `scratch` on each device

template <typename V>
hipError_t upload(V **dst, const std::vector<V> &src) {
    size_t bytes = std::max<size_t>(src.size() * sizeof(V), 8);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice);
    return e;
}

void free_devplan(DevPlan *D) {
    if (!D) return;
    void *ptrs[] = {D->sn, D->rows, D->relmap, D->chlist, D->acolptr, D->aoff,
                    D->avidx, D->perm, D->pinv, D->lvl_small, D->lvl_big, D->lvl_sn,
                    D->asm_col, D->csr_ptr, D->sell_ptr, D->sell_col, D->sell_vidx,
                    D->slv_small, D->slv_pan, D->asm_pc, D->colblk, D->blk_col0, D->gptr,
                    D->gidx, D->dinv_list, D->soa_it_s, D->soa_it_r0, D->soa_chunks, D->grow_q, D->grow_y,
                    D->val_row, D->val_col, D->xoff, D->x_list, D->xg_q, D->xg_y,
                    D->xs_list, D->soa_chunks_x};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int32_t *p : D->fz_ptr)
        if (p) (void)hipFree(p);
    for (int32_t *p : D->fz_sn)
        if (p) (void)hipFree(p);
    delete D;
}

// Upload the plan to the current device on first use.
sc_status ensure_device(const sc_plan *P) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    std::lock_guard<std::mutex> lock(g_upload_mutex);
    if (dev >= 0 && dev < 64 && !g_kernels_ready[dev]) {
        if (spchol_kernels_init() != hipSuccess) return SC_EDEVICE;
        if (spchol_solve_init() != hipSuccess) return SC_EDEVICE;
        void *sp = nullptr;
        if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) return SC_EDEVICE;
        g_scratch_dev[dev] = sp;
        g_kernels_ready[dev] = true;
    }
    if (P->dev) return P->dev_id == dev ? SC_OK : SC_EINVAL;
    DevPlan *D = new (std::nothrow) DevPlan();
    if (!D) return SC_ENOMEM;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload(&D->sn, P->sn);
    if (e == hipSuccess) e = upload(&D->rows, P->rows);
    if (e == hipSuccess) e = upload(&D->relmap, P->relmap);
    if (e == hipSuccess) e = upload(&D->chlist, P->chlist);
    if (e == hipSuccess) e = upload(&D->acolptr, P->acolptr);
    if (e == hipSuccess) e = upload(&D->aoff, P->aoff);
    if (e == hipSuccess) e = upload(&D->avidx, P->avidx);
    if (e == hipSuccess) e = upload(&D->perm, P->perm);
    if (e == hipSuccess) e = upload(&D->pinv, P->pinv);
    if (e == hipSuccess) e = upload(&D->lvl_small, P->lvl_small);
    if (e == hipSuccess) e = upload(&D->lvl_big, P->lvl_big);
    if (e == hipSuccess) e = upload(&D->lvl_sn, P->lvl_sn);
    if (e == hipSuccess) e = upload(&D->asm_col, P->asm_col);
    if (e == hipSuccess) e = upload(&D->asm_pc, P->asm_pc);
    if (e == hipSuccess) e = upload(&D->slv_small, P->slv_small);
    if (e == hipSuccess) e = upload(&D->slv_pan, P->slv_pan);
    if (e == hipSuccess) e = upload(&D->dinv_list, P->dinv_list);
    if (e == hipSuccess) e = upload(&D->xoff, P->xoff);
    if (e == hipSuccess) e = upload(&D->x_list, P->x_list);
    if (e == hipSuccess) e = upload(&D->xg_q, P->xg_q);
    if (e == hipSuccess) e = upload(&D->xg_y, P->xg_y);
    if (e == hipSuccess) e = upload(&D->xs_list, P->xs_list);
    if (e == hipSuccess) e = upload(&D->csr_ptr, P->csr_ptr);
    if (e == hipSuccess) e = upload(&D->sell_ptr, P->sell_ptr);
    if (e == hipSuccess) e = upload(&D->sell_col, P->sell_col);
    if (e == hipSuccess) e = upload(&D->sell_vidx, P->sell_vidx);
    if (e == hipSuccess) e = upload(&D->colblk, P->colblk);
    if (e == hipSuccess) e = upload(&D->gptr, P->gptr);
    if (e == hipSuccess) e = upload(&D->gidx, P->gidx);
    if (e == hipSuccess) e = upload(&D->soa_it_s, P->soa_it_s);
    if (e == hipSuccess) e = upload(&D->soa_it_r0, P->soa_it_r0);
    if (e == hipSuccess) e = upload(&D->soa_chunks, P->soa_chunks);
    if (e == hipSuccess) e = upload(&D->soa_chunks_x, P->soa_chunks_x);
    if (e == hipSuccess) e = upload(&D->grow_q, P->grow_q);
    if (e == hipSuccess) e = upload(&D->grow_y, P->grow_y);
    if (e == hipSuccess) e = upload(&D->val_row, P->val_row);
    if (e == hipSuccess) e = upload(&D->val_col, P->val_col);
    if (e == hipSuccess) e = upload(&D->blk_col0, P->blk_col0);
    if (e != hipSuccess) {
        free_devplan(D);
        return e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EDEVICE;
    }
    spchol_build_factor_schedule(P, D);
    spchol_build_solve_schedule(P, D);
    if (spchol_build_subtrees(P, D) != hipSuccess) {
        free_devplan(D);
        return SC_ENOMEM;
    }
    P->dev = D;
    P->dev_id = dev;
    return SC_OK;
}

// Built-in nested dissection of a pattern (order.cpp), after the checks
// the ordering needs (the full validation follows in the plan builder).
sc_status built_in_order(int64_t n, const int64_t *colptr, const int32_t *rowind,
                         std::vector<int32_t> &perm) {
    if (n < 1 || n >= INT32_MAX || !colptr || !rowind) return SC_EINVAL;
    if (colptr[0] != 0) return SC_EPATTERN;
    for (int64_t j = 0; j < n; j++)
        if (colptr[j + 1] < colptr[j]) return SC_EPATTERN;
    for (int64_t q = 0; q < colptr[n]; q++)
        if (rowind[q] < 0 || rowind[q] >= n) return SC_EPATTERN;
    try {
        perm.resize(n);
    } catch (const std::bad_alloc &) {
        return SC_ENOMEM;
    }
    return spchol_nd_order(n, colptr, rowind, perm.data()) ? SC_OK : SC_ENOMEM;
}

sc_status map_err(hipError_t e) {
    if (e == hipSuccess) return SC_OK;
    if (e == hipErrorOutOfMemory) return SC_ENOMEM;
    return SC_EDEVICE;
}

// Sizes (in doubles) of the solve workspaces for nrhs right-hand sides per
// matrix (matrices rounded up to whole groups of 64 in the batch-interleaved
// form): y, u, part, ps, in that order.
void solve_ws_words(const sc_plan *P, const sc_numeric *N, int32_t nrhs, size_t out[4]) {
    const size_t nb = N->soa ? size_t((N->batch + 63) / 64) * 64 : size_t(N->batch);
    const size_t cnt = nb * size_t(nrhs);
    out[0] = cnt * size_t(P->n);
    out[1] = cnt * P->rows.size();
    out[2] = cnt * size_t(P->part_size);
    out[3] = N->soa ? cnt * size_t(P->soa_psize) : 0;
}

void free_solve_ws(SolveWs &W) {
    void *old[] = {W.y, W.u, W.part, W.ps};
    for (void *q : old)
        if (q) (void)hipFree(q);
    W = SolveWs{};
}

// Solve workspaces for nrhs right-hand sides per matrix.  Growing them
// moves their addresses, which a captured graph on this numeric object
// still holds, so growth is refused (SC_EINVAL) while such a graph exists.
sc_status ensure_solve_ws(const sc_plan *P, sc_numeric *N, int32_t nrhs) {
    if (nrhs <= N->ws.nrhs) return SC_OK;
    if (N->graphs > 0) return SC_EINVAL;
    free_solve_ws(N->ws);
    size_t words[4];
    solve_ws_words(P, N, nrhs, words);
    double **dst[4] = {&N->ws.y, &N->ws.u, &N->ws.part, &N->ws.ps};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 4 && e == hipSuccess; k++)
        if (words[k] > 0 || k < 3)
            e = hipMalloc(reinterpret_cast<void **>(dst[k]),
                          std::max<size_t>(words[k] * sizeof(double), 8));
    if (e != hipSuccess) {
        free_solve_ws(N->ws);
        return map_err(e);
    }
    N->ws.nrhs = nrhs;
    return SC_OK;
}

void free_refine_ws(RefineWs &W) {
    void *ptrs[] = {W.r, W.sc, W.part, W.part2, W.anorm, W.vc, W.stat, W.conv, W.active, W.count};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    W = RefineWs{};
}

// Refinement workspaces: vectors per (matrix, right-hand side), scalars
// per system (matrix, right-hand side, block).  Refused (SC_EINVAL) when
// they would have to grow while a captured graph holds their addresses.
sc_status ensure_refine_ws(sc_numeric *N, int32_t nrhs, int64_t ldb) {
    RefineWs &W = N->rws;
    const int32_t nsys = N->batch * nrhs;
    const size_t nseg = size_t(nsys) * N->plan->nblk;
    if (W.r && W.nsys >= nsys && W.ldb >= ldb) return SC_OK;
    if (N->graphs > 0) return SC_EINVAL;
    free_refine_ws(W);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&W.r), 5 * sizeof(double) * nsys * ldb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&W.sc), 4 * sizeof(double) * nseg);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&W.part), 32 * 3 * sizeof(double) * nseg);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&W.part2),
                      sizeof(double) * size_t(3 * nsys + N->batch) *
                          size_t((N->plan->n + 255) / 256));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&W.anorm),
                      sizeof(double) * N->batch * N->plan->nblk);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&W.vc),
                      sizeof(double) * N->batch * std::max<int64_t>(N->plan->sell_ptr.back(), 1));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&W.stat), sizeof(double) * 6 * nseg);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&W.conv), sizeof(int32_t) * nseg);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&W.active), sizeof(int32_t) * N->batch);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&W.count), sizeof(int32_t));
    if (e != hipSuccess) {
        free_refine_ws(W);
        return map_err(e);
    }
    W.nsys = nsys;
    W.ldb = ldb;
    return SC_OK;
}

}  // namespace

extern "C" {

const char *sc_status_string(sc_status s) {
    switch (s) {
    case SC_OK: return "ok";
    case SC_EINVAL: return "invalid argument";
    case SC_EPATTERN: return "malformed pattern or permutation";
    case SC_ENOMEM: return "out of memory";
    case SC_EDEVICE: return "HIP runtime error";
    case SC_ENOTSPD: return "matrix not positive definite";
    case SC_ENOCONV: return "refinement did not converge";
    case SC_ESCRATCH: return "workspace exceeds the no-allocation scratch (SC_NOALLOC_SCRATCH_BYTES)";
    }
    return "unknown status";
}

sc_status sc_options_default(sc_options *opt) {
    if (!opt) return SC_EINVAL;
    opt->relax = 1;
    opt->relax_cols = 4;
    opt->relax_zeros = 0.05;
    opt->small_front = 64;
    opt->soa_min_batch = kSoaMinBatch;
    opt->soa_seg_max = kSoaSegMax;
    opt->soa_subtree_min = kSoaSubtreeMin;
    opt->ordering = SC_ORDER_GIVEN;
    opt->panel_inverse = 0;
    return SC_OK;
}

sc_status sc_analyze(int64_t n, const int64_t *colptr_host, const int32_t *rowind_host,
                     const int32_t *perm_host, const sc_options *opt, sc_plan_t **plan_out) {
    if (!plan_out) return SC_EINVAL;
    *plan_out = nullptr;
    sc_options o;
    sc_options_default(&o);
    if (opt) o = *opt;
    if (o.relax_cols < 0 || o.small_front < 0 || !(o.relax_zeros >= 0.0)) return SC_EINVAL;
    if (o.ordering < SC_ORDER_NATURAL || o.ordering > SC_ORDER_ND) return SC_EINVAL;
    if (perm_host && o.ordering != SC_ORDER_GIVEN) return SC_EINVAL;
    if (o.ordering != SC_ORDER_ND)
        return spchol_build_plan(n, colptr_host, rowind_host, perm_host, o, 1, nullptr, nullptr,
                                 plan_out);
    std::vector<int32_t> perm;
    sc_status st = built_in_order(n, colptr_host, rowind_host, perm);
    if (st != SC_OK) return st;
    return spchol_build_plan(n, colptr_host, rowind_host, perm.data(), o, 1, nullptr, nullptr,
                             plan_out);
}

sc_status sc_analyze_group(int32_t npat, const int64_t *n_host, const int64_t *const *colptr_host,
                           const int32_t *const *rowind_host, const int32_t *const *perm_host,
                           const sc_options *opt, sc_plan_t **plan_out) {
    if (!plan_out) return SC_EINVAL;
    *plan_out = nullptr;
    if (npat < 1 || !n_host || !colptr_host || !rowind_host) return SC_EINVAL;
    sc_options o;
    sc_options_default(&o);
    if (opt) o = *opt;
    if (o.relax_cols < 0 || o.small_front < 0 || !(o.relax_zeros >= 0.0)) return SC_EINVAL;
    if (o.ordering < SC_ORDER_NATURAL || o.ordering > SC_ORDER_ND) return SC_EINVAL;
    if (o.ordering != SC_ORDER_GIVEN && perm_host)
        for (int32_t k = 0; k < npat; k++)
            if (perm_host[k]) return SC_EINVAL;
    std::vector<int64_t> col0(npat + 1, 0), val0(npat + 1, 0);
    for (int32_t k = 0; k < npat; k++) {
        const int64_t nk = n_host[k];
        if (nk < 1 || !colptr_host[k] || !rowind_host[k]) return SC_EINVAL;
        if (nk > INT32_MAX - 1 - col0[k]) return SC_EINVAL;
        const int64_t *cp = colptr_host[k];
        if (cp[0] != 0) return SC_EPATTERN;
        for (int64_t j = 0; j < nk; j++)
            if (cp[j + 1] < cp[j]) return SC_EPATTERN;
        // rows of pattern k must stay inside it once shifted into the group
        for (int64_t q = 0; q < cp[nk]; q++)
            if (rowind_host[k][q] < 0 || rowind_host[k][q] >= nk) return SC_EPATTERN;
        if (perm_host && perm_host[k])
            for (int64_t j = 0; j < nk; j++)
                if (perm_host[k][j] < 0 || perm_host[k][j] >= nk) return SC_EPATTERN;
        col0[k + 1] = col0[k] + nk;
        val0[k + 1] = val0[k] + cp[nk];
    }
    const int64_t n = col0[npat];
    std::vector<int64_t> colptr;
    std::vector<int32_t> rowind, perm;
    try {
        colptr.resize(n + 1);
        rowind.resize(val0[npat]);
        perm.resize(n);
    } catch (const std::bad_alloc &) {
        return SC_ENOMEM;
    }
    for (int32_t k = 0; k < npat; k++) {
        const int64_t nk = n_host[k], c0 = col0[k], v0 = val0[k];
        for (int64_t j = 0; j < nk; j++) colptr[c0 + j] = v0 + colptr_host[k][j];
        for (int64_t q = 0; q < val0[k + 1] - v0; q++)
            rowind[v0 + q] = int32_t(c0 + rowind_host[k][q]);
        std::vector<int32_t> own;
        if (o.ordering == SC_ORDER_ND) {
            const sc_status st = built_in_order(nk, colptr_host[k], rowind_host[k], own);
            if (st != SC_OK) return st;
        }
        for (int64_t j = 0; j < nk; j++) {
            int64_t pj = j;
            if (o.ordering == SC_ORDER_ND) pj = own[j];
            else if (o.ordering == SC_ORDER_GIVEN && perm_host && perm_host[k]) pj = perm_host[k][j];
            perm[c0 + j] = int32_t(c0 + pj);
        }
    }
    colptr[n] = val0[npat];
    return spchol_build_plan(n, colptr.data(), rowind.data(), perm.data(), o, npat, col0.data(),
                             val0.data(), plan_out);
}

sc_status sc_plan_export_blocks(const sc_plan_t *P, int64_t *col0_host, int64_t *val0_host) {
    if (!P) return SC_EINVAL;
    if (col0_host) std::memcpy(col0_host, P->blk_col0.data(), sizeof(int64_t) * (P->nblk + 1));
    if (val0_host) std::memcpy(val0_host, P->blk_val0.data(), sizeof(int64_t) * (P->nblk + 1));
    return SC_OK;
}

sc_status sc_plan_info(const sc_plan_t *P, sc_plan_stats *out) {
    if (!P || !out) return SC_EINVAL;
    out->n = P->n;
    out->nnzA = P->nnzA;
    out->nnzL = P->nnzL;
    out->nfund = int64_t(P->ffirst.size()) - 1;
    out->nsuper = P->ns;
    out->nlevels = P->nlevels;
    out->L_store = P->Lsize;
    out->U_store = P->Usize;
    out->max_front = P->max_front;
    out->max_width = P->max_width;
    out->flops = P->flops;
    out->etree_height = P->etree_height;
    out->nblocks = P->nblk;
    return SC_OK;
}

sc_status sc_plan_export_symbolic(const sc_plan_t *P, int32_t *perm_host, int32_t *parent_host,
                                  int64_t *Lcolptr_host, int32_t *Lrowind_host) {
    if (!P) return SC_EINVAL;
    const int64_t n = P->n;
    if (perm_host) std::memcpy(perm_host, P->perm.data(), sizeof(int32_t) * n);
    if (parent_host) std::memcpy(parent_host, P->parent.data(), sizeof(int32_t) * n);
    if (Lcolptr_host) {
        Lcolptr_host[0] = 0;
        for (int64_t j = 0; j < n; j++) Lcolptr_host[j + 1] = Lcolptr_host[j] + P->colcount[j];
    }
    if (Lrowind_host) {
        int64_t o = 0;
        const int64_t nf = int64_t(P->ffirst.size()) - 1;
        for (int64_t t = 0; t < nf; t++)
            for (int32_t j = P->ffirst[t]; j < P->ffirst[t + 1]; j++) {
                const int64_t a = P->frowptr[t] + (j - P->ffirst[t]);
                const int64_t b = P->frowptr[t + 1];
                std::memcpy(Lrowind_host + o, P->frows.data() + a, sizeof(int32_t) * (b - a));
                o += b - a;
            }
    }
    return SC_OK;
}

sc_status sc_plan_export_supernodes(const sc_plan_t *P, int32_t *first_host,
                                    int32_t *parent_host, int32_t *level_host,
                                    int64_t *rowptr_host, int32_t *rows_host) {
    if (!P) return SC_EINVAL;
    for (int32_t s = 0; s < P->ns; s++) {
        const SnDesc &d = P->sn[s];
        if (first_host) first_host[s] = d.first;
        if (parent_host) parent_host[s] = d.parent;
        if (level_host) level_host[s] = d.level;
        if (rowptr_host) rowptr_host[s] = d.rowptr;
    }
    if (first_host) first_host[P->ns] = int32_t(P->n);
    if (rowptr_host) rowptr_host[P->ns] = int64_t(P->rows.size());
    if (rows_host && !P->rows.empty())
        std::memcpy(rows_host, P->rows.data(), sizeof(int32_t) * P->rows.size());
    return SC_OK;
}

void sc_plan_destroy(sc_plan_t *P) {
    if (!P) return;
    free_devplan(P->dev);
    delete P;
}

sc_status sc_numeric_create(const sc_plan_t *P, int32_t batch, sc_dtype dtype,
                            sc_numeric_t **num_out) {
    if (!P || !num_out || batch < 1 || (dtype != SC_F64 && dtype != SC_F32)) return SC_EINVAL;
    *num_out = nullptr;
    sc_status st = ensure_device(P);
    if (st != SC_OK) return st;
    sc_numeric *N = new (std::nothrow) sc_numeric();
    if (!N) return SC_ENOMEM;
    N->plan = P;
    N->batch = batch;
    N->dtype = dtype;
    N->device = P->dev_id;
    const int32_t soa_min = P->opt.soa_min_batch == 0 ? kSoaMinBatch : P->opt.soa_min_batch;
    N->soa = soa_min > 0 && batch >= soa_min;
    const size_t sz = dtype == SC_F64 ? 8 : 4;
    hipError_t e = hipMalloc(&N->L, std::max<size_t>(size_t(batch) * P->Lsize * sz, 8));
    if (e == hipSuccess) e = hipMalloc(&N->U, std::max<size_t>(size_t(batch) * P->Usize * sz, 8));
    const size_t ninfo = size_t(batch) * P->nblk;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&N->info), sizeof(int32_t) * ninfo);
    if (e == hipSuccess)
        e = hipMalloc(&N->pinv,
                      std::max<size_t>(size_t(batch) * P->max_lvl_big * kTile * kTile * sz, 8));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&N->dinv),
                      std::max<size_t>(size_t(batch) * P->dinv_size * sizeof(double), 8));
    if (e == hipSuccess && N->soa)
        e = hipMalloc(&N->Ls, std::max<size_t>(size_t((batch + 63) / 64) * 64 * P->Lsize * sz, 8));
    const bool xinv = P->xsize > 0 && batch >= kXMinBatch &&
                      (P->opt.panel_inverse > 0 || (P->opt.panel_inverse == 0 && dtype == SC_F32));
    if (e == hipSuccess && xinv) e = hipMalloc(&N->xinv, size_t(batch) * P->xsize * sz);
    if (e == hipSuccess) e = hipMemset(N->info, 0, sizeof(int32_t) * ninfo);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&N->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&N->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&N->ev_join, hipEventDisableTiming);
    if (e == hipSuccess && N->soa) e = hipStreamCreateWithFlags(&N->side2, hipStreamNonBlocking);
    if (e == hipSuccess && N->soa) e = hipEventCreateWithFlags(&N->ev_fork2, hipEventDisableTiming);
    if (e == hipSuccess && N->soa) e = hipEventCreateWithFlags(&N->ev_join2, hipEventDisableTiming);
    if (e != hipSuccess) {
        sc_numeric_destroy(N);
        return map_err(e);
    }
    *num_out = N;
    return SC_OK;
}

void sc_numeric_destroy(sc_numeric_t *N) {
    if (!N) return;
    if (N->side) (void)hipStreamDestroy(N->side);  // waits for its work
    if (N->side2) (void)hipStreamDestroy(N->side2);
    if (N->L) (void)hipFree(N->L);
    if (N->U) (void)hipFree(N->U);
    if (N->info) (void)hipFree(N->info);
    void *ws[] = {N->pinv, N->dinv, N->Ls, N->xinv};
    for (void *q : ws)
        if (q) (void)hipFree(q);
    free_solve_ws(N->ws);
    free_refine_ws(N->rws);
    if (N->ev_fork) (void)hipEventDestroy(N->ev_fork);
    if (N->ev_join) (void)hipEventDestroy(N->ev_join);
    if (N->ev_fork2) (void)hipEventDestroy(N->ev_fork2);
    if (N->ev_join2) (void)hipEventDestroy(N->ev_join2);
    delete N;
}

sc_status sc_factor(const sc_plan_t *P, sc_numeric_t *N, const double *values_dev, int64_t ldv,
                    void *stream) {
    if (!P || !N || N->plan != P || !values_dev || ldv < P->nnzA) return SC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (dev != N->device) return SC_EINVAL;
    return map_err(spchol_factor_run(P, N, values_dev, ldv, static_cast<hipStream_t>(stream)));
}

sc_status sc_factor_info(const sc_numeric_t *N, int32_t *info_host, void *stream) {
    if (!N || !info_host) return SC_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t ninfo = int64_t(N->batch) * N->plan->nblk;
    hipError_t e = hipMemcpyAsync(info_host, N->info, sizeof(int32_t) * ninfo,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return map_err(e);
    bool bad = false;
    for (int64_t q = 0; q < ninfo; q++) {
        if (info_host[q] == INT_MAX) info_host[q] = 0;
        if (info_host[q] != 0) bad = true;
    }
    return bad ? SC_ENOTSPD : SC_OK;
}

sc_status sc_solve(const sc_plan_t *P, sc_numeric_t *N, double *b_dev, int32_t nrhs, int64_t ldb,
                   void *stream) {
    if (!P || !N || N->plan != P || !b_dev || nrhs < 1 || ldb < P->n) return SC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (dev != N->device) return SC_EINVAL;
    const sc_status ws = ensure_solve_ws(P, N, nrhs);
    if (ws != SC_OK) return ws;
    return map_err(
        spchol_solve_run(P, N, b_dev, nrhs, ldb, static_cast<hipStream_t>(stream), nullptr));
}

sc_status sc_solve_noalloc(const sc_plan_t *P, sc_numeric_t *N, double *b_dev, int32_t nrhs,
                           int64_t ldb, void *stream) {
    if (!P || !N || N->plan != P || !b_dev || nrhs < 1 || ldb < P->n) return SC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (dev != N->device || dev < 0 || dev >= 64) return SC_EINVAL;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_upload_mutex);
        base = g_scratch_dev[dev];
    }
    if (!base) return SC_EDEVICE;  // the device was never set up by sc_numeric_create
    // the four solve vectors of sc_solve, each at a 256-byte boundary
    size_t words[4];
    solve_ws_words(P, N, nrhs, words);
    SolveWs W;
    double **dst[4] = {&W.y, &W.u, &W.part, &W.ps};
    size_t off = 0;
    for (int k = 0; k < 4; k++) {
        if (words[k] > (SIZE_MAX >> 4)) return SC_ESCRATCH;
        *dst[k] = reinterpret_cast<double *>(static_cast<unsigned char *>(base) + off);
        off += (std::max<size_t>(words[k] * sizeof(double), 8) + 255) & ~size_t(255);
        if (off > size_t(SC_NOALLOC_SCRATCH_BYTES)) return SC_ESCRATCH;
    }
    W.nrhs = nrhs;
    N->wsc = &W;
    const hipError_t e =
        spchol_solve_run(P, N, b_dev, nrhs, ldb, static_cast<hipStream_t>(stream), nullptr);
    N->wsc = &N->ws;
    return map_err(e);
}

sc_status sc_refine_solve(const sc_plan_t *P, sc_numeric_t *N, const double *values_dev,
                          int64_t ldv, const double *b_dev, double *x_dev, int32_t nrhs,
                          int64_t ldb, double tol, int32_t maxit, int32_t method,
                          sc_refine_stats *stats_host, void *stream) {
    if (!P || !N || N->plan != P || !values_dev || !b_dev || !x_dev || nrhs < 1 ||
        ldb < P->n || ldv < P->nnzA || maxit < 0 || !(tol >= 0.0) ||
        (method != SC_REFINE_CLASSICAL && method != SC_REFINE_PCG))
        return SC_EINVAL;
    if (b_dev == x_dev) return SC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (dev != N->device) return SC_EINVAL;
    sc_status ws = ensure_solve_ws(P, N, nrhs);
    if (ws == SC_OK) ws = ensure_refine_ws(N, nrhs, ldb);
    if (ws != SC_OK) return ws;
    const int32_t nsys = N->batch * nrhs * P->nblk;
    std::vector<double> stat(size_t(6) * nsys);
    int32_t nact = 0;
    hipError_t e = spchol_refine_run(P, N, values_dev, ldv, b_dev, x_dev, nrhs, ldb, tol, maxit, method,
                          stat.data(), &nact, true, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return map_err(e);
    bool fail = false;
    for (int32_t k = 0; k < nsys; k++) {
        const double *q = &stat[size_t(6) * k];
        if (q[1] == 0.0) fail = true;
        if (stats_host) {
            stats_host[k].iters = int32_t(q[0]);
            stats_host[k].clause = int32_t(q[1]);
            stats_host[k].relres = q[2];
            stats_host[k].rnorm = q[3];
            stats_host[k].bnorm = q[4];
            stats_host[k].xnorm = q[5];
        }
    }
    return fail ? SC_ENOCONV : SC_OK;
}

sc_status sc_numeric_get_columns(const sc_plan_t *P, const sc_numeric_t *N, int32_t b,
                                 int64_t ncols, const int32_t *cols_host, double *out_host) {
    if (!P || !N || N->plan != P || b < 0 || b >= N->batch || ncols < 0) return SC_EINVAL;
    if (ncols > 0 && (!cols_host || !out_host)) return SC_EINVAL;
    for (int64_t q = 0; q < ncols; q++)
        if (cols_host[q] < 0 || cols_host[q] >= P->n) return SC_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return SC_EDEVICE;
    const size_t sz = N->dtype == SC_F64 ? 8 : 4;
    std::vector<unsigned char> blk;
    int32_t cached = -1;
    int64_t o = 0;
    for (int64_t q = 0; q < ncols; q++) {
        const int32_t j = cols_host[q];
        const int32_t s = P->col2sn[j];
        const SnDesc &d = P->sn[s];
        if (s != cached) {
            blk.resize(size_t(d.c) * d.w * sz);
            const unsigned char *src = static_cast<const unsigned char *>(N->L) +
                                       (size_t(b) * P->Lsize + d.loff) * sz;
            if (hipMemcpy(blk.data(), src, blk.size(), hipMemcpyDeviceToHost) != hipSuccess)
                return SC_EDEVICE;
            cached = s;
        }
        const int64_t t = int64_t(std::upper_bound(P->ffirst.begin(), P->ffirst.end(), j) -
                                  P->ffirst.begin()) - 1;
        const int64_t a = P->frowptr[t] + (j - P->ffirst[t]);
        const int32_t *R = P->rows.data() + d.rowptr;
        const int64_t cbase = int64_t(j - d.first) * d.c;
        int32_t pos = j - d.first;
        for (int64_t e = a; e < P->frowptr[t + 1]; e++) {
            const int32_t r = P->frows[e];
            while (pos < d.c && R[pos] < r) pos++;
            if (pos >= d.c) return SC_EINVAL;  // cannot happen for a valid plan
            const size_t idx = size_t(cbase + pos);
            out_host[o++] = sz == 8 ? reinterpret_cast<const double *>(blk.data())[idx]
                                    : double(reinterpret_cast<const float *>(blk.data())[idx]);
        }
    }
    return SC_OK;
}

sc_status sc_numeric_get_block(const sc_plan_t *P, const sc_numeric_t *N, int32_t b, int32_t s,
                               double *out_host) {
    if (!P || !N || N->plan != P || b < 0 || b >= N->batch || s < 0 || s >= P->ns || !out_host)
        return SC_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return SC_EDEVICE;
    const SnDesc &d = P->sn[s];
    const size_t sz = N->dtype == SC_F64 ? 8 : 4;
    const size_t cnt = size_t(d.c) * d.w;
    std::vector<unsigned char> blk(cnt * sz);
    const unsigned char *src =
        static_cast<const unsigned char *>(N->L) + (size_t(b) * P->Lsize + d.loff) * sz;
    if (hipMemcpy(blk.data(), src, blk.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return SC_EDEVICE;
    for (size_t q = 0; q < cnt; q++)
        out_host[q] = sz == 8 ? reinterpret_cast<const double *>(blk.data())[q]
                              : double(reinterpret_cast<const float *>(blk.data())[q]);
    return SC_OK;
}

sc_status sc_numeric_profile(sc_numeric_t *N, int32_t enable) {
    if (!N) return SC_EINVAL;
    N->prof.on = enable != 0;
    return SC_OK;
}

sc_status sc_numeric_profile_read(sc_numeric_t *N, int32_t cap, sc_kernel_stat *out_host,
                                  int32_t *count_out) {
    if (!N || cap < 0 || (cap > 0 && !out_host) || !count_out) return SC_EINVAL;
    Profiler &pr = N->prof;
    std::vector<sc_kernel_stat> acc(KK_Count);
    for (int k = 0; k < KK_Count; k++) {
        std::memset(&acc[k], 0, sizeof(sc_kernel_stat));
        std::strncpy(acc[k].name, kKernelNames[k], sizeof(acc[k].name) - 1);
    }
    sc_status st = SC_OK;
    for (const Profiler::Rec &r : pr.recs) {
        float ms = 0.f;
        if (!r.a || !r.b || hipEventSynchronize(r.b) != hipSuccess ||
            hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            st = SC_EDEVICE;
            continue;
        }
        sc_kernel_stat &a = acc[r.kind];
        a.launches++;
        a.ms += ms;
        a.flops += r.flops;
        a.bytes += r.bytes;
        a.alg_bytes += r.abytes;
    }
    pr.recs.clear();
    pr.used = 0;
    int32_t n = 0;
    for (int k = 0; k < KK_Count && n < cap; k++)
        if (acc[k].launches > 0) out_host[n++] = acc[k];
    *count_out = n;
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One captured step: factorization of the batch plus the refined solve with
// a fixed number of refinement steps (converged systems are skipped on the
// device), recorded once into a HIP graph on a private stream and replayed.

struct sc_graph {
    const sc_plan *plan = nullptr;
    sc_numeric *num = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t nsys = 0;
    bool counted = false;  // counted in num->graphs
};

namespace {

sc_status stats_to_host(const sc_numeric *N, int32_t nsys, sc_refine_stats *out, hipStream_t st) {
    std::vector<double> stat(size_t(6) * nsys);
    hipError_t e = hipMemcpyAsync(stat.data(), N->rws.stat, sizeof(double) * stat.size(),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return map_err(e);
    bool fail = false;
    for (int32_t k = 0; k < nsys; k++) {
        const double *q = &stat[size_t(6) * k];
        if (q[1] == 0.0) fail = true;
        if (out) {
            out[k].iters = int32_t(q[0]);
            out[k].clause = int32_t(q[1]);
            out[k].relres = q[2];
            out[k].rnorm = q[3];
            out[k].bnorm = q[4];
            out[k].xnorm = q[5];
        }
    }
    return fail ? SC_ENOCONV : SC_OK;
}

}  // namespace

sc_status sc_step_graph_create(const sc_plan_t *P, sc_numeric_t *N, const double *values_dev,
                               int64_t ldv, const double *b_dev, double *x_dev, int32_t nrhs,
                               int64_t ldb, double tol, int32_t iters, int32_t method,
                               sc_graph_t **out) {
    if (!out) return SC_EINVAL;
    *out = nullptr;
    if (!P || !N || N->plan != P || !values_dev || !b_dev || !x_dev || nrhs < 1 ||
        ldb < P->n || ldv < P->nnzA || iters < 0 || !(tol >= 0.0) || b_dev == x_dev ||
        (method != SC_REFINE_CLASSICAL && method != SC_REFINE_PCG))
        return SC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (dev != N->device) return SC_EINVAL;
    // every workspace exists before the capture (no allocation inside it)
    sc_status ws = ensure_solve_ws(P, N, nrhs);
    if (ws == SC_OK) ws = ensure_refine_ws(N, nrhs, ldb);
    if (ws != SC_OK) return ws;
    hipError_t e = hipSuccess;
    sc_graph *G = new (std::nothrow) sc_graph();
    if (!G) return SC_ENOMEM;
    G->plan = P;
    G->num = N;
    G->nsys = N->batch * nrhs * P->nblk;
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete G;
        return map_err(e);
    }
    const bool prof = N->prof.on;
    N->prof.on = false;  // no event records inside the graph
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = spchol_factor_run(P, N, values_dev, ldv, cs);
        int32_t nact = 0;
        if (e1 == hipSuccess)
            e1 = spchol_refine_run(P, N, values_dev, ldv, b_dev, x_dev, nrhs, ldb, tol, iters,
                                   method, nullptr, &nact, false, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e1;
        G->graph = g;
    }
    N->prof.on = prof;
    if (e == hipSuccess) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        sc_step_graph_destroy(G);
        return map_err(e);
    }
    N->graphs++;
    G->counted = true;
    *out = G;
    return SC_OK;
}

sc_status sc_step_graph_launch(sc_graph_t *G, void *stream) {
    if (!G || !G->exec) return SC_EINVAL;
    return map_err(hipGraphLaunch(G->exec, static_cast<hipStream_t>(stream)));
}

sc_status sc_step_graph_stats(sc_graph_t *G, sc_refine_stats *stats_host, void *stream) {
    if (!G) return SC_EINVAL;
    return stats_to_host(G->num, G->nsys, stats_host, static_cast<hipStream_t>(stream));
}

void sc_step_graph_destroy(sc_graph_t *G) {
    if (!G) return;
    if (G->counted && G->num) G->num->graphs--;
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate option sets on the caller's pattern, values and
// right-hand sides (factor of the whole batch, then one solve) with HIP
// events and keeps the fastest by factor_ms + solves_per_factor * solve_ms.

namespace {

// One factor + one solve of candidate `o` (plan made by `make_plan`), timed
// with events on `st` (best of `reps` after one warm-up pass).
template <typename MakePlan>
sc_status time_candidate(const MakePlan &make_plan, const sc_options &o,
                         const double *values_dev, int64_t ldv, int32_t batch, sc_dtype dtype,
                         const double *b_dev, double *bw, int32_t nrhs, int64_t ldb, int reps,
                         hipStream_t st, double *fms, double *sms) {
    sc_plan_t *P = nullptr;
    sc_status r = make_plan(o, &P);
    if (r != SC_OK) return r;
    sc_numeric_t *N = nullptr;
    r = sc_numeric_create(P, batch, dtype, &N);
    hipEvent_t ev[4] = {};
    for (auto &x : ev)
        if (r == SC_OK && hipEventCreate(&x) != hipSuccess) r = SC_EDEVICE;
    const size_t bbytes = sizeof(double) * size_t(batch) * nrhs * ldb;
    *fms = *sms = 1e300;
    for (int rep = 0; rep <= reps && r == SC_OK; rep++) {
        (void)hipEventRecord(ev[0], st);
        r = sc_factor(P, N, values_dev, ldv, st);
        (void)hipEventRecord(ev[1], st);
        if (r == SC_OK &&
            hipMemcpyAsync(bw, b_dev, bbytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
            r = SC_EDEVICE;
        (void)hipEventRecord(ev[2], st);
        if (r == SC_OK) r = sc_solve(P, N, bw, nrhs, ldb, st);
        (void)hipEventRecord(ev[3], st);
        if (r == SC_OK && hipEventSynchronize(ev[3]) != hipSuccess) r = SC_EDEVICE;
        float f = 0.f, sv = 0.f;
        if (r == SC_OK && rep > 0 && hipEventElapsedTime(&f, ev[0], ev[1]) == hipSuccess &&
            hipEventElapsedTime(&sv, ev[2], ev[3]) == hipSuccess) {
            *fms = std::min(*fms, double(f));
            *sms = std::min(*sms, double(sv));
        }
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (N) sc_numeric_destroy(N);
    sc_plan_destroy(P);
    return r;
}


// Candidates: front-kernel threshold x amalgamation width x solve layout
// (x the built-in ordering against the natural one when no permutation is
// given).
std::vector<sc_options> tune_candidates(int32_t batch, bool try_orderings) {
    std::vector<sc_options> cand;
    const int32_t small_fronts[] = {32, 64, 128, 192};
    const int32_t relax_cols[] = {4, 16};
    for (int ord = 0; ord < (try_orderings ? 2 : 1); ord++)
        for (int32_t sf : small_fronts)
            for (int32_t rc : relax_cols)
                for (int soa = 0; soa < (batch >= 16 ? 2 : 1); soa++) {
                    sc_options o;
                    sc_options_default(&o);
                    o.small_front = sf;
                    o.relax_cols = rc;
                    o.soa_min_batch = soa ? 1 : -1;
                    if (try_orderings) o.ordering = ord ? SC_ORDER_ND : SC_ORDER_NATURAL;
                    cand.push_back(o);
                }
    return cand;
}

// Time every candidate (plans from make_plan) and keep the best score.
template <typename MakePlan>
sc_status tune_run(const MakePlan &make_plan, const std::vector<sc_options> &cand,
                   const double *values_dev, int64_t ldv, int32_t batch, sc_dtype dtype,
                   const double *b_dev, int32_t nrhs, int64_t ldb, double solves_per_factor,
                   sc_options *best_out, sc_tune_entry *table_host, int32_t table_cap,
                   int32_t *ntable_out, hipStream_t st) {
    double *bw = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&bw),
                             sizeof(double) * size_t(batch) * nrhs * ldb);
    if (e != hipSuccess) return map_err(e);
    double best = 1e300;
    int32_t nt = 0;
    sc_status result = SC_OK;
    for (const sc_options &o : cand) {
        double fms = 0.0, sms = 0.0;
        result = time_candidate(make_plan, o, values_dev, ldv, batch, dtype, b_dev, bw, nrhs,
                                ldb, 2, st, &fms, &sms);
        if (result != SC_OK) break;
        const double score = fms + solves_per_factor * sms;
        if (nt < table_cap) table_host[nt] = sc_tune_entry{o, fms, sms, score};
        nt++;
        if (score < best) {
            best = score;
            *best_out = o;
        }
    }
    (void)hipFree(bw);
    if (ntable_out) *ntable_out = std::min(nt, table_cap);
    return result;
}

}  // namespace

sc_status sc_autotune_group(int32_t npat, const int64_t *n_host,
                            const int64_t *const *colptr_host, const int32_t *const *rowind_host,
                            const int32_t *const *perm_host, const double *values_dev,
                            int64_t ldv, int32_t batch, sc_dtype dtype, const double *b_dev,
                            int32_t nrhs, int64_t ldb, double solves_per_factor,
                            sc_options *best_out, sc_tune_entry *table_host, int32_t table_cap,
                            int32_t *ntable_out, void *stream) {
    if (!best_out || !values_dev || !b_dev || npat < 1 || !n_host || batch < 1 || nrhs < 1 ||
        !(solves_per_factor >= 0.0) || (dtype != SC_F64 && dtype != SC_F32) ||
        table_cap < 0 || (table_cap > 0 && !table_host))
        return SC_EINVAL;
    int64_t ntot = 0;
    for (int32_t k = 0; k < npat; k++) ntot += n_host[k];
    if (ldb < ntot) return SC_EINVAL;
    auto make = [&](const sc_options &o, sc_plan_t **P) {
        return sc_analyze_group(npat, n_host, colptr_host, rowind_host, perm_host, &o, P);
    };
    return tune_run(make, tune_candidates(batch, false), values_dev, ldv, batch, dtype, b_dev,
                    nrhs, ldb, solves_per_factor, best_out, table_host, table_cap, ntable_out,
                    static_cast<hipStream_t>(stream));
}

sc_status sc_autotune(int64_t n, const int64_t *colptr_host, const int32_t *rowind_host,
                      const int32_t *perm_host, const double *values_dev, int64_t ldv,
                      int32_t batch, sc_dtype dtype, const double *b_dev, int32_t nrhs,
                      int64_t ldb, double solves_per_factor, sc_options *best_out,
                      sc_tune_entry *table_host, int32_t table_cap, int32_t *ntable_out,
                      void *stream) {
    if (!best_out || !values_dev || !b_dev || batch < 1 || nrhs < 1 || ldb < n ||
        !(solves_per_factor >= 0.0) || (dtype != SC_F64 && dtype != SC_F32) ||
        table_cap < 0 || (table_cap > 0 && !table_host))
        return SC_EINVAL;
    auto make = [&](const sc_options &o, sc_plan_t **P) {
        return sc_analyze(n, colptr_host, rowind_host, perm_host, &o, P);
    };
    return tune_run(make, tune_candidates(batch, perm_host == nullptr), values_dev, ldv, batch,
                    dtype, b_dev, nrhs, ldb, solves_per_factor, best_out, table_host, table_cap,
                    ntable_out, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// Adjoint of the solve: lambda = A^{-1} g_x with the stored factor, then the
// value gradients on the pattern.

sc_status sc_adjoint(const sc_plan_t *P, sc_numeric_t *N, const double *x_dev,
                     const double *gx_dev, double *gvalues_dev, int64_t ldv, double *gb_dev,
                     int32_t nrhs, int64_t ldb, void *stream) {
    if (!P || !N || N->plan != P || !x_dev || !gx_dev || !gvalues_dev || !gb_dev || nrhs < 1 ||
        ldb < P->n || ldv < P->nnzA || gb_dev == x_dev)
        return SC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (dev != N->device) return SC_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const sc_status ws = ensure_solve_ws(P, N, nrhs);
    if (ws != SC_OK) return ws;
    hipError_t e = spchol_solve_run(P, N, gb_dev, nrhs, ldb, st, nullptr, gx_dev);  // lambda
    if (e == hipSuccess)
        e = spchol_adjoint_values(P, N->batch, x_dev, gb_dev, nrhs, ldb, gvalues_dev, ldv, st);
    return map_err(e);
}
