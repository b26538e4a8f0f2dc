/*
 * spchol_products.h -- sparse matrix products on fixed patterns (libspchol).
 *
 * C = A B or C = A B^T, plus an optional D on C's pattern, for CSR matrices
 * whose patterns are fixed while their values change: the structured sparse
 * products the paper evaluates with its generated kernels (powers A^2, A^3,
 * A^4 of a mesh Laplacian and L M L^T + K, Sec. 5.2 and Table tab:Lpow).
 * As in the paper, a one-time host pass unrolls every output entry into its
 * sum of products and harvests the leaves (Sec. 4.4): for entry (i, j) the
 * value positions of the pairs (A_ik, B_kj) in ascending k, and of D_ij.
 * Each launch evaluates every entry of C (Sec. 4.3's grouping at the
 * granularity of one wave: 64 consecutive entries share one loop over the
 * longest term list among them), with the position tables interleaved so
 * lane l of a wave reads word l (the coalesced layout of Sec. 4.8).  Chains
 * are products of products: A^3 = (A^2) A, L M L^T + K = (L diag(M)) L^T +
 * K, the intermediate results stored once and read by every term that uses
 * them (the global decomposition of Sec. 4.2.1).
 *
 * Every entry is   C_ij = fl( sum_k A_ik B_kj ) (+ D_ij),   summed in
 * ascending k with one fused multiply-add per term, then D added.
 * Conventions as in spchol.h (*_host / *_dev, stream as void*, sc_status).
 */
#ifndef SPCHOL_PRODUCTS_H
#define SPCHOL_PRODUCTS_H

#include "spchol.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sc_spprod sc_spprod_t;

/*
 * Symbolic product: A is m x p (rowptr int64[m+1], colind int32), B is p x n
 * (transB = 0; rows p) or n x p (transB = 1, C = A B^T; rows n), D (both
 * pointers NULL for none) is m x n.  Column indices strictly ascending in
 * every row.  C's pattern is the structural pattern of the product union
 * D's (entries whose terms cancel numerically are kept).  Host work only;
 * the first sc_spprod_run uploads the tables to its device (later runs
 * must use that device).
 * Errors: SC_EINVAL (NULL, sizes), SC_EPATTERN (unsorted or duplicate or
 * out-of-range column indices, rowptr not monotone), SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_spprod_create(int64_t m, int64_t p, int64_t n, const int64_t *A_rowptr_host,
                           const int32_t *A_colind_host, const int64_t *B_rowptr_host,
                           const int32_t *B_colind_host, int32_t transB,
                           const int64_t *D_rowptr_host, const int32_t *D_colind_host,
                           sc_spprod_t **out);

/* Sizes: stored entries of C and terms (products) of all entries. */
sc_status sc_spprod_info(const sc_spprod_t *prod, int64_t *nnzC_out, int64_t *nterms_out);

/* C's pattern (host): rowptr int64[m+1], colind int32[nnzC]; either may be NULL. */
sc_status sc_spprod_export(const sc_spprod_t *prod, int64_t *C_rowptr_host,
                           int32_t *C_colind_host);

/*
 * Numeric product of `batch` value sets: A_dev [batch][lda], B_dev
 * [batch][ldb], D_dev [batch][ldd] (NULL when the plan has no D), C_dev
 * [batch][ldc], all float64 (dtype SC_F64) or all float32 (SC_F32), values
 * in the order of their patterns.  Asynchronous on `stream`; the first call
 * allocates and uploads the position tables, later calls allocate nothing.
 * Errors: SC_EINVAL (sizes, dtype, D missing or unexpected, another device
 * than the first call's), SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_spprod_run(const sc_spprod_t *prod, sc_dtype dtype, int32_t batch,
                        const void *A_dev, int64_t lda, const void *B_dev, int64_t ldb,
                        const void *D_dev, int64_t ldd, void *C_dev, int64_t ldc, void *stream);

void sc_spprod_destroy(sc_spprod_t *prod);

#ifdef __cplusplus
}
#endif

#endif /* SPCHOL_PRODUCTS_H */
