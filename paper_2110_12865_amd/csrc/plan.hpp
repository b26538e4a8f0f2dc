// Internal plan layout shared by the host symbolic pass and the HIP
// launchers.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <vector>

#include "spchol.h"

// One supernode as the GPU kernels see it.  A workgroup reads a single
// record, so an array of structs is the natural layout here.
struct SnDesc {
    int64_t loff;    // offset of the c x w column-major L block (scalars)
    int64_t uoff;    // offset of the m x m column-major update block
    int64_t rowptr;  // offset of the row list R_s in Plan::rows
    int64_t relptr;  // offset of the m relative positions in the parent
    int32_t first;   // first column (permuted numbering)
    int32_t w;       // width (columns)
    int32_t c;       // rows of the front, |R_s|
    int32_t m;       // c - w: update rows
    int32_t chbeg;   // children: chlist[chbeg .. chend)
    int32_t chend;
    int32_t parent;  // supernodal parent, -1 for a root
    int32_t level;   // longest path from the leaves
    int64_t dinv;    // offset of the inverted 64x64 diagonal blocks (solve
                     // by panels), -1 when the supernode is solved in LDS
    int64_t part;    // offset of the backward-solve partial sums
    int32_t blk;     // diagonal block (pattern of a group plan) it belongs to
    int32_t bcol0;   // first column of that block
};
static_assert(sizeof(SnDesc) == 88, "SnDesc layout");

// Assembly of one column of a large front: destination of rows tj..c-1
// (front entry (i, tj) at dst + i in L or, for update columns, in U), the
// column's entries of A (for L columns) and the pieces of the children's
// update columns that land in it.
struct AsmCol {
    int64_t dst;   // L: loff + tj*c; U: uoff + (tj-w)*m - w
    int64_t a0;    // first entry of A's column first+tj (permuted), na entries
    int32_t na;
    int32_t c;     // rows of the front
    int32_t tj;    // column inside the front
    int32_t base;  // tj*c: aoff of row i is base + i
    int32_t ch0;   // pieces [ch0, ch0 + nch)
    int32_t nch;
    int32_t isU;   // 1: update column (destination in U)
    int32_t pad;
};
static_assert(sizeof(AsmCol) == 48, "AsmCol layout");
// Up to 64 consecutive rows of one child's update column: U[src + k] is
// added to front row relmap[rmp + k], k < cnt.  A column's pieces follow the
// children's order, rows ascending inside a child.
constexpr int kAsmPiece = 64;
struct AsmPiece {
    int64_t src;
    int64_t rmp;
    int32_t cnt;
    int32_t pad;
};
static_assert(sizeof(AsmPiece) == 24, "AsmPiece layout");

// A supernode is solved by 64-column panels across many workgroups when it
// is wide or tall; otherwise one workgroup solves it out of LDS.
constexpr int kSolvePanel = 64;
constexpr int kSolveChunk = 256;  // rows per workgroup in the backward panel step
// Supernodes that are not solved by panels fall into row classes; a class
// fixes the number of lanes that cooperate on one (supernode, matrix) and
// the rows each lane keeps: c <= 16 and c <= 32 use 16 and 32 lanes (several
// supernodes per wave), the others one wave with 1, 2, 4 or 8 rows per lane.
constexpr int kSolveClasses = 6;
constexpr int kSolveClassMaxC[kSolveClasses] = {16, 32, 64, 128, 256, 512};
inline int solve_class(int c) {
    int k = 0;
    while (k + 1 < kSolveClasses && c > kSolveClassMaxC[k]) k++;
    return k;
}
inline bool solve_by_panels(const SnDesc &d) { return d.w > kSolvePanel || d.c > 512; }
// Batch-interleaved solves (groups of 64 matrices, one matrix per lane):
// rows below a supernode's diagonal block are cut into blocks of kSoaRows
// rows, one work item each; L is copied to the interleaved layout in
// chunks of kSoaChunk scalars.
constexpr int kSoaRows = 16;
constexpr int kSoaChunk = 128;
constexpr int kSoaMinBatch = 64;  // default of sc_options::soa_min_batch: whole lane groups
constexpr int kSoaSegMax = 96;    // default of sc_options::soa_seg_max
constexpr int kSoaSubtreeMin = 2048;  // default of sc_options::soa_subtree_min

constexpr int kSellRows = 64;  // rows per slice of the sliced row structure of A

// Whole-block inverses X = L11^{-1} of the diagonal blocks of panel-solved
// supernodes (sc_options::panel_inverse): levels whose panel-solved
// supernodes are all at most kXMaxW columns wide, for numeric objects of at
// least kXMinBatch matrices (the batched solves that use them).
// Levels with at most kXSmallMax supernodes outside the panel kernels (the
// top levels, where one wave per supernode and matrix leaves the chip idle)
// get whole-block inverses of those supernodes' diagonal blocks as well.
constexpr int kXMaxW = 1024;
constexpr int kXMinBatch = 16;
constexpr int kXSmallMax = 96;

// Fronts of 64 < c rows factored by one workgroup keep their packed lower
// triangle and the 64-row tiles of L21 ([k][64], k padded to 4) in LDS;
// scalars needed for a front of c rows and width w.  A front goes there only
// if that fits the 160 KiB of LDS of a gfx950 workgroup in FP64 (with 1 KiB
// of the kernel's own), so a plan serves both precisions.
constexpr int kFrontWgMaxC = 256;
constexpr int kLdsBytes = 160 * 1024;
inline int front_wg_lds(int c, int w) {
    const int m = c - w;
    return c * (c + 1) / 2 + ((m + 63) / 64) * 64 * ((w + 3) & ~3);
}
inline bool front_wg_fits(int c, int w) {
    return c <= kFrontWgMaxC && int64_t(front_wg_lds(c, w)) * 8 + 1024 <= kLdsBytes;
}

struct DevPlan;  // device copies, defined by the HIP side

struct sc_plan {
    int64_t n = 0, nnzA = 0;
    sc_options opt{};

    // independent diagonal blocks (the patterns of a group plan; one block
    // otherwise): block k owns columns [blk_col0[k], blk_col0[k+1]) in both
    // numberings and values [blk_val0[k], blk_val0[k+1])
    int32_t nblk = 1;
    std::vector<int64_t> blk_col0, blk_val0;  // nblk + 1
    std::vector<int32_t> colblk;              // n: block of each column

    // permutation (perm[new] = old) and its inverse
    std::vector<int32_t> perm, pinv;
    // column elimination tree and exact column counts (diagonal included)
    std::vector<int32_t> parent;
    std::vector<int64_t> colcount;
    int64_t nnzL = 0;
    double flops = 0.0;
    int64_t etree_height = 0;

    // fundamental supernodes: columns [ffirst[t], ffirst[t+1]) and the exact
    // structure of their first column
    std::vector<int32_t> ffirst;
    std::vector<int64_t> frowptr;
    std::vector<int32_t> frows;

    // supernodes after amalgamation
    int32_t ns = 0;
    std::vector<SnDesc> sn;
    std::vector<int32_t> col2sn;  // n
    std::vector<int32_t> rows;    // concatenated R_s (sorted ascending)
    std::vector<int32_t> relmap;  // concatenated relative maps
    std::vector<int32_t> chlist;  // children, ascending per parent
    int64_t Lsize = 0, Usize = 0, relsize = 0;
    int32_t nlevels = 0;
    int64_t max_front = 0, max_width = 0;

    // permuted lower triangle of A by columns: offset of the entry inside
    // the c x w column-major L block of the column's supernode, and index
    // into the caller's values
    std::vector<int64_t> acolptr;  // n+1
    std::vector<int32_t> aoff;
    std::vector<int64_t> avidx;

    // A in the caller's numbering with both triangles, by rows, for the
    // residual A x: column index and index into the caller's values
    std::vector<int64_t> csr_ptr;  // n+1
    std::vector<int32_t> csr_col;
    std::vector<int64_t> csr_vidx;
    // the same entries sliced by kSellRows rows (row-interleaved per slice)
    std::vector<int64_t> sell_ptr;  // slices + 1
    std::vector<int32_t> sell_col;
    std::vector<int64_t> sell_vidx;
    // row and column of every stored entry of the caller's lower triangle
    std::vector<int32_t> val_row, val_col;

    // level schedule: supernodes of each level split into fronts done by
    // one workgroup ("small") and fronts done by the tiled kernels ("big")
    std::vector<int32_t> lvl_small_ptr, lvl_small;
    std::vector<int32_t> lvl_big_ptr, lvl_big;
    std::vector<int32_t> lvl_small_maxc, lvl_big_maxc, lvl_big_maxw;
    std::vector<int32_t> lvl_ptr, lvl_sn;  // all supernodes of each level
    std::vector<int32_t> lvl_maxc;
    // solve schedule: per level, supernodes solved in LDS and by panels
    // slv_small holds the level's other supernodes by row class: class k of
    // level l is slv_small[slv_cls_ptr[l * kSolveClasses + k] ..
    // slv_cls_ptr[l * kSolveClasses + k + 1]), supernodes ascending
    std::vector<int32_t> slv_cls_ptr, slv_small, slv_pan_ptr, slv_pan;
    std::vector<int32_t> slv_pan_maxw, slv_pan_maxc;
    // forward-solve gather map: the update-vector entries of the children
    // that land in row i of supernode s are FV[gidx[g]] for g in
    // [gptr[rowptr_s + i], gptr[rowptr_s + i + 1]), children in order
    std::vector<int32_t> gptr, gidx;
    // batch-interleaved solves: per level, the row blocks (supernode, first
    // row) of the supernodes not solved by panels; the partial sums of a
    // supernode's row blocks start at its SnDesc::part (w per block);
    // chunk starts of the L copy
    std::vector<int32_t> soa_it_ptr, soa_it_s, soa_it_r0;
    // forward gather rows of those supernodes, per level: front-vector
    // position rowptr_s + i and the right-hand-side row first_s + i (or -1
    // below the diagonal block); level l owns [grow_ptr[l], grow_ptr[l+1])
    std::vector<int32_t> grow_ptr, grow_q, grow_y;
    int64_t soa_psize = 0;
    std::vector<int64_t> soa_chunks, soa_chunks_x;
    int32_t soa_copy_lev = -1, soa_copy_lev_x = -1;  // highest level each copy covers
    int32_t xs_lev = -1;  // highest level of the supernodes in xs_list
    int64_t dinv_size = 0;   // scalars of inverted diagonal blocks
    // panel-solved supernodes factored as small fronts (their inverted
    // diagonal blocks are formed after the factorization; the tiled factor
    // writes the others as it factors each block)
    std::vector<int32_t> dinv_list;
    int64_t part_size = 0;   // partial sums per right-hand side
    // whole-block inverses: per supernode the offset of its w x w
    // column-major X (-1: none), scalars per matrix, the supernodes that have
    // one
    // (x_list widest first), and per level whether its panel-solved
    // supernodes use them, with their front rows for the forward gather
    // (as grow_*: position rowptr_s + i, right-hand-side row or -1)
    std::vector<int64_t> xoff;
    int64_t xsize = 0;
    std::vector<int32_t> x_list;
    std::vector<uint8_t> slv_pan_x;
    std::vector<int32_t> xg_ptr, xg_q, xg_y;
    // the other supernodes (at most 64 wide) of the levels with at most
    // kXSmallMax of them: their inverses, and per level whether it has them
    std::vector<int32_t> xs_list;
    std::vector<uint8_t> slv_small_x;
    int32_t x_nbmax = 0;  // most 64-column blocks of one X
    int32_t npan = 0;        // supernodes solved by panels
    std::vector<int64_t> lvl_bigcols;     // sum of c over big fronts
    int32_t max_lvl_big = 0;              // most large fronts in one level
    // assembly of the large fronts: one descriptor per target column (level
    // l owns [lvl_colent_off[l], + lvl_bigcols[l])) and its pieces
    std::vector<AsmCol> asm_col;
    std::vector<AsmPiece> asm_pc;
    std::vector<int64_t> lvl_colent_off;  // nlevels

    mutable DevPlan *dev = nullptr;
    mutable int dev_id = -1;
};

// Host symbolic pass (analyze.cpp).  Returns SC_OK or an error; on success
// *out owns a fully built plan.
// nblk > 1 declares the pattern block diagonal with the given column and
// value offsets (nblk + 1 entries each); the permutation must keep every
// block's columns inside the block.
sc_status spchol_build_plan(int64_t n, const int64_t *colptr,
                            const int32_t *rowind, const int32_t *perm,
                            const sc_options &opt, int32_t nblk, const int64_t *blk_col0,
                            const int64_t *blk_val0, sc_plan **out);
