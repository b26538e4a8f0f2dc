// Device-side state of a plan and of a batch of numeric factors, and the
// launchers of the factor and solve kernels.  Internal to libspchol.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "plan.hpp"

// Tile of the blocked dense kernels (rows/columns of a trailing-update tile
// and panel width of the blocked partial factorization).
constexpr int kTile = 64;
// Width of the outer blocks of the blocked partial factorization: panels of
// kTile columns update only the columns of their block; the trailing matrix
// beyond the block is updated once per block with a rank-kBlock product.
constexpr int kBlock = 256;

// One kernel launch of the factor schedule.  The schedule depends only on
// the pattern, so it is built once per plan and replayed by every call.
struct FLaunch {
    // Fork: the side stream waits for the main stream's work so far; Join:
    // the main stream waits for the side stream's work so far
    enum Kind : int { Small, Assemble, Potrf, Trsm, Syrk, Fork, Join } kind;
    int32_t level;
    int32_t k;        // panel start column (Potrf/Trsm/Syrk inner)
    int32_t K0;       // block start column (Syrk)
    int32_t outer;    // Syrk: 0 = inside the block, 1 = beyond it, 2 = the next
                      // kBlock columns beyond it, 3 = the columns after those
    int32_t list0;    // first entry in the level's list
    int32_t nlist;    // entries
    int64_t gridx;    // workgroups along x
    int32_t lds;      // dynamic LDS size in scalars (times sizeof(T) at launch)
    double flops;     // algorithmic flops per matrix of the batch
    double words;     // algorithmic scalars of L/U moved per matrix
    double ibytes;    // algorithmic index/value bytes per matrix
    int32_t side = 0; // 1: launched on the side stream
    double a_entries = 0.0;  // entries of A read per matrix
    double l_exact = 0.0;    // exact entries of L written per matrix
};

struct SPanel {  // one 64-column panel step of a level's panel-solved supernodes
    int64_t fwd_tiles = 0;   // 64-row tiles below the panel (max over supernodes)
    int64_t bwd_chunks = 0;  // kSolveChunk-row chunks below the panel (max)
    double flops = 0.0;      // per right-hand side
    double words = 0.0;      // factor scalars read per right-hand side
    double vwords = 0.0;     // vector entries per right-hand side
    double dwords = 0.0;     // inverse-block entries per matrix
    double lx = 0.0;         // exact entries of L in the panel's columns
};

struct SClass {  // supernodes of one row class in one level
    int32_t list0 = 0, n = 0;  // entries of slv_small
    double flops = 0.0;        // per right-hand side
    double words = 0.0;        // factor scalars read
    double vwords = 0.0;       // vector entries per right-hand side
    double ibytes = 0.0;       // index bytes per right-hand side
    double lx = 0.0;           // exact entries of L of these supernodes
};

struct SLaunch {  // one level of a triangular solve
    int32_t level = 0;
    SClass cls[kSolveClasses];
    // batch-interleaved form: all supernodes of the level not solved by
    // panels, and their row-block items
    int32_t all0 = 0, nall = 0;
    int32_t it0 = 0, nit = 0;
    int32_t grow0 = 0, ngrow = 0;     // gather rows of those supernodes
    // flops, factor scalars, vector entries and index bytes (per right-hand
    // side) of the gather, the diagonal blocks and the rows below them
    double vw_gather = 0.0, ib_gather = 0.0;
    double f_diag = 0.0, w_diag = 0.0, vw_diag = 0.0, ib_diag = 0.0;
    double f_rows = 0.0, w_rows = 0.0, vw_rows = 0.0, ib_rows = 0.0;
    double lx_diag = 0.0, lx_rows = 0.0;  // exact entries of L in those parts
    int32_t pan0 = 0, npan = 0;      // supernodes solved by panels
    int32_t maxc_pan = 0;
    int32_t maxw_pan = 0;
    bool xpan = false;  // the panel-solved supernodes have whole-block inverses
    double x_words = 0.0, x_lx = 0.0;  // X and L21 scalars read per sweep; exact L entries
    int32_t xg0 = 0, nxg = 0;          // their front rows in xg_q / xg_y
    double vw_xg = 0.0, ib_xg = 0.0;
    // the supernodes outside the panel kernels have whole-block inverses
    bool xsmall = false;
    int32_t maxw_small = 0, maxc_small = 0;
    double xs_words = 0.0, xs_lx = 0.0;
    double vw_pan = 0.0, ib_pan = 0.0;
    std::vector<SPanel> panels;
};

struct DevPlan {
    SnDesc *sn = nullptr;
    int32_t *rows = nullptr;
    int32_t *relmap = nullptr;
    int32_t *chlist = nullptr;
    int64_t *acolptr = nullptr;
    int32_t *aoff = nullptr;
    int64_t *avidx = nullptr;
    int32_t *perm = nullptr;
    int32_t *pinv = nullptr;
    int32_t *lvl_small = nullptr;
    int32_t *lvl_big = nullptr;
    int32_t *lvl_sn = nullptr;
    AsmCol *asm_col = nullptr;        // assembly of the large fronts
    AsmPiece *asm_pc = nullptr;
    int32_t *slv_small = nullptr;     // solve schedule lists
    int32_t *slv_pan = nullptr;
    int32_t *dinv_list = nullptr;     // panel-solved small fronts
    int64_t *xoff = nullptr;          // whole-block inverses: offset per supernode
    int32_t *x_list = nullptr;        // supernodes that have one
    int32_t *xg_q = nullptr;          // their front rows (forward gather)
    int32_t *xg_y = nullptr;
    int32_t *xs_list = nullptr;       // small supernodes with whole-block inverses
    int64_t *csr_ptr = nullptr;       // A (both triangles) by rows, for A x
    int64_t *sell_ptr = nullptr;      // the same rows sliced by kSellRows
    int32_t *sell_col = nullptr;
    int64_t *sell_vidx = nullptr;
    int32_t *soa_it_s = nullptr;      // batch-interleaved solve items
    int32_t *soa_it_r0 = nullptr;
    int64_t *soa_chunks = nullptr;    // chunk starts of the interleaved L copy
    int64_t *soa_chunks_x = nullptr;  // the same without the levels with inverses
    int32_t *grow_q = nullptr;        // forward gather rows
    int32_t *grow_y = nullptr;
    int32_t *val_row = nullptr;       // (row, column) of every stored entry
    int32_t *val_col = nullptr;
    int32_t *gptr = nullptr;          // forward-solve gather map
    int32_t *gidx = nullptr;
    int32_t *colblk = nullptr;        // block of every column
    int64_t *blk_col0 = nullptr;      // nblk + 1 block column offsets
    std::vector<FLaunch> fsched;
    std::vector<SLaunch> ssched;
    // bottom subtrees of the batch-interleaved solve, for each level K that
    // may close them (every level up to K without panel-solved supernodes):
    // fz_ptr[K][t] .. fz_ptr[K][t + 1] index fz_sn[K], the postorder of the
    // subtree of root t (a supernode of level <= K whose parent lies above
    // K); fz_roots[K] roots (device arrays, one pair per K)
    std::vector<int32_t *> fz_ptr, fz_sn;
    std::vector<int32_t> fz_roots;
};

// Kernel kinds for per-launch timing.
enum KernelKind : int {
    KK_SmallFront = 0, KK_Assemble, KK_Potrf, KK_Trsm, KK_Syrk, KK_Dinv,
    KK_Fwd, KK_FwdPanel, KK_Bwd, KK_BwdPanel, KK_Spmv, KK_Vec, KK_Perm, KK_Gather,
    KK_FwdRows, KK_BwdRows, KK_ToSoa, KK_Count
};
extern const char *const kKernelNames[KK_Count];

// Optional event timing of every launch (off by default).  Each launch is
// bracketed by two events on the stream it runs on; its algorithmic flops
// and two byte counts are attached so rates can be formed: `bytes`, the
// library's model of what the launch moves (front and update blocks,
// vectors, indices), and `abytes`, the algorithmic bytes of the method
// itself (the factor: entries of A read, with their row index, plus the
// exact entries of L written; a triangular solve: the exact entries of L
// read once for all right-hand sides; the residual product: entries of A
// read; other launches: none).
struct Profiler {
    bool on = false;
    struct Rec { int kind; hipEvent_t a, b; double flops, bytes, abytes; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin(int kind, double flops, double bytes, hipStream_t st, double abytes = 0.0) {
        if (!on) return;
        Rec r{kind, get(), get(), flops, bytes, abytes};
        if (r.a) (void)hipEventRecord(r.a, st);
        recs.push_back(r);
    }
    void end(hipStream_t st) {
        if (!on || recs.empty()) return;
        if (recs.back().b) (void)hipEventRecord(recs.back().b, st);
    }
    ~Profiler() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

// Workspace of iterative refinement (allocated on first use).
struct RefineWs {
    int32_t nsys = 0;
    int64_t ldb = 0;
    double *r = nullptr;        // 5 vectors of nsys * ldb (residual, correction, CG)
    // per system (matrix, right-hand side, block): nseg = nsys * nblk
    double *sc = nullptr;       // scalars, 4 * nseg
    double *part = nullptr;     // reduction partials, nseg * 32 * 3
    // partials of the fused residual product, nsys * ceil(n/256) * 3, then
    // the row-sum maxima of |A| per (matrix, 256-row block), batch * ceil(n/256)
    double *part2 = nullptr;
    double *anorm = nullptr;    // batch * nblk
    double *vc = nullptr;       // values of A in row order, batch * nnz(both triangles)
    double *stat = nullptr;     // nseg * 6
    int32_t *conv = nullptr;    // nseg
    int32_t *active = nullptr;  // batch
    int32_t *count = nullptr;   // 1
};

// Vectors of the triangular solves, right-hand sides interleaved
// (index * nrhs + r), in the factor's precision (sized in doubles).
struct SolveWs {
    double *y = nullptr;     // nb * n * nrhs: P b, then y, then z
    double *u = nullptr;     // nb * sum(c_s) * nrhs: front vectors
    double *part = nullptr;  // nb * nrhs * part_size
    double *ps = nullptr;    // nb * soa_psize * nrhs partial sums (interleaved form)
    int32_t nrhs = 0;        // right-hand sides the buffers hold
};

struct sc_numeric {
    const sc_plan *plan = nullptr;
    int32_t batch = 0;
    sc_dtype dtype = SC_F64;
    int device = -1;
    void *L = nullptr;       // batch * Lsize scalars
    void *U = nullptr;       // batch * Usize scalars
    int32_t *info = nullptr; // batch
    void *pinv = nullptr;    // batch * max_lvl_big * 64 * 64: panel inverses (factor)
    double *dinv = nullptr;  // batch * dinv_size: inverted diagonal blocks
    // batch * xsize scalars: whole-block inverses of the diagonal blocks of
    // the plan's X supernodes (null: the solves substitute panel by panel)
    void *xinv = nullptr;
    // solve workspaces owned by the numeric object (allocated on first use,
    // grown for more right-hand sides), and the set the solve kernels use:
    // `wsc` points at `ws` except inside sc_solve_noalloc, which points it at
    // the library's static scratch array for the duration of the call
    SolveWs ws;
    const SolveWs *wsc = &ws;
    // batch-interleaved solves (batch >= soa_min): L copied to groups of 64
    // matrices with the matrix index fastest, refreshed after each factor;
    // the solve vectors then use the same interleaving
    bool soa = false;
    void *Ls = nullptr;         // ceil(batch / 64) * Lsize * 64 scalars
    bool ls_ok = false;
    Profiler prof;
    RefineWs rws;
    // captured step graphs alive on this object: their kernels hold the
    // workspace addresses, so workspaces may not be reallocated meanwhile
    int32_t graphs = 0;
    // second stream of the factorization (lookahead in the panel chain of
    // large fronts) and the events that order it against the caller's stream
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // third stream: the interleaved copy of L, beside the factorization of
    // the levels above the copied supernodes (forked and joined inside the
    // factorization)
    hipStream_t side2 = nullptr;
    hipEvent_t ev_fork2 = nullptr, ev_join2 = nullptr;
};

// Launchers (factor.hip / solve.hip).  Return hipSuccess or the first error.
hipError_t spchol_factor_run(const sc_plan *P, sc_numeric *N,
                             const double *vals, int64_t ldv, hipStream_t st);
// active (nullable, device): matrices b with active[b] == 0 are left untouched
// (used by refinement to stop correcting converged matrices).  bin
// (nullable): the right-hand sides are read from bin instead of b (same
// layout) and the solutions written to b.
hipError_t spchol_solve_run(const sc_plan *P, sc_numeric *N, double *b,
                            int32_t nrhs, int64_t ldb, hipStream_t st,
                            const int32_t *active, const double *bin = nullptr);
// parts: 1 = whole-block inverses of the small levels (xs_list), 2 = the
// inverted diagonal blocks of dinv_list, 3 = both
hipError_t spchol_dinv_run(const sc_plan *P, sc_numeric *N, hipStream_t st, int parts = 3);
// The interleaved copy of L (batch-interleaved numeric objects), on stream st.
hipError_t spchol_to_soa_run(const sc_plan *P, sc_numeric *N, hipStream_t st);
hipError_t spchol_refine_run(const sc_plan *P, sc_numeric *N, const double *vals,
                             int64_t ldv, const double *b, double *x, int32_t nrhs,
                             int64_t ldb, double tol, int32_t maxit, int32_t method,
                             double *stat_host, int32_t *nactive_out, bool sync,
                             hipStream_t st);
hipError_t spchol_kernels_init();
// Value gradients of the adjoint: g[b][k] = -sum_r (lam_i x_j + lam_j x_i)
// for stored entry k = (i, j), i != j, and -sum_r lam_i x_i on the diagonal.
hipError_t spchol_adjoint_values(const sc_plan *P, int batch, const double *x, const double *lam,
                                 int32_t nrhs, int64_t ldb, double *g, int64_t ldv,
                                 hipStream_t st);

// Largest dynamic LDS allocation per workgroup on the current device.
extern int g_max_lds;
