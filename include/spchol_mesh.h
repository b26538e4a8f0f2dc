/*
 * spchol_mesh.h -- on-device assembly of mesh systems for libspchol.
 *
 * The values of A = K + c diag(m) for a triangle mesh, K the cotangent
 * stiffness matrix, computed on the GPU straight into the value array that
 * sc_factor reads (the operator the paper assembles in its cotan
 * construction, Sec. 5.3; its expressions grouped by dependency level with
 * harvested index tables, Sec. 4.2-4.4):
 *
 *   level 1, one thread per edge (p, q) with opposite corners o (one or two
 *   triangles), every value set s:
 *       cot_o = (u . v) / |u_0 v_1 - u_1 v_0|,  u = x_p - x_o,  v = x_q - x_o
 *       w     = clip(1/2 sum_o cot_o, clip_lo, clip_hi)
 *       w^s   = clip(w * scale_s[e], clip_lo, clip_hi)   (no scale: w^s = w)
 *       A_pq  = -w^s
 *   level 2, one thread per vertex p, every value set:
 *       A_pp  = sum_q w^s_pq + c m_p
 *     summed over the neighbours q > p in ascending order, then q < p in
 *     ascending order; the edge weights are read back from the level-1
 *     entries (they are the stored intermediates: each is used by one
 *     off-diagonal and two diagonal entries).
 *
 * Every product, sum and quotient is rounded once (no fused multiply-add),
 * so the values are reproducible to the bit and equal those of the same
 * formulas evaluated in IEEE double arithmetic in this order.
 * Conventions as in spchol.h (pattern in lower CSC form, *_host / *_dev
 * pointers, stream passed as void*, sc_status returns).
 */
#ifndef SPCHOL_MESH_H
#define SPCHOL_MESH_H

#include "spchol.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sc_cotan sc_cotan_t; /* assembly tables of one mesh pattern */

/*
 * Assembly tables for a mesh with nv vertices and ntri triangles
 * (tris_host int32[ntri][3], vertex indices) on the lower CSC pattern
 * (colptr_host int64[nv+1], rowind_host int32[nnz]) of its stiffness
 * matrix.  The stored off-diagonal entries must be exactly the mesh edges,
 * each an edge of one or two triangles; edge e is the e-th stored
 * off-diagonal entry in pattern order (the order of edge_scale_dev below).
 * Host work only, except the upload of the tables to the current device.
 * Errors: SC_EINVAL (NULL, sizes), SC_EPATTERN (pattern malformed, an entry
 * that is not a mesh edge, a mesh edge that is not stored, an edge of more
 * than two triangles, a vertex index out of range, a degenerate triangle),
 * SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_cotan_create(int64_t nv, const int64_t *colptr_host, const int32_t *rowind_host,
                          int64_t ntri, const int32_t *tris_host, sc_cotan_t **out);

/* Number of edges (stored off-diagonal entries) of the pattern. */
sc_status sc_cotan_nedges(const sc_cotan_t *asm_tables, int64_t *nedge_out);

/*
 * Assemble `batch` value sets into values_dev [batch][ldv] (ldv >= nnz;
 * every stored entry of each set is written).  pos_dev: float64 vertex
 * positions [nv][2]; with pos_stride > 0 set s reads its own positions at
 * pos_dev + s * pos_stride (pos_stride >= 2 nv), with pos_stride == 0 all
 * sets share one.  edge_scale_dev: float64 [batch][nedge] per-set weight
 * scales, or NULL.  mass_dev: float64 [nv].  Asynchronous on `stream`; no
 * allocation.  Errors: SC_EINVAL, SC_EDEVICE.
 */
sc_status sc_cotan_assemble(const sc_cotan_t *asm_tables, int32_t batch, const double *pos_dev,
                            int64_t pos_stride, const double *edge_scale_dev,
                            const double *mass_dev, double mass_coeff, double clip_lo,
                            double clip_hi, double *values_dev, int64_t ldv, void *stream);

void sc_cotan_destroy(sc_cotan_t *asm_tables);

#ifdef __cplusplus
}
#endif

#endif /* SPCHOL_MESH_H */
