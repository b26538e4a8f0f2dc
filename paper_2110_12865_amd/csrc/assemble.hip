// On-device assembly of the cotangent stiffness + mass matrix of a triangle
// mesh into the value array of its fixed pattern (spchol_mesh.h).
//
// The expression DAG of the assembly has two levels (the paper's grouping
// by dependency level, Sec. 4.3): the edge weights (each read by one
// off-diagonal and two diagonal entries, so they are stored: the global
// intermediates of Sec. 4.2.1) and the diagonal sums.  The host harvests
// the leaves of every expression into index tables once (Sec. 4.4): per
// edge its endpoints, its one or two opposite corners and the position of
// its value; per vertex the position of its diagonal and its incident
// edges in summation order.  Floating-point contraction is switched off for
// this file (the pragma below), so every product, sum and quotient is
// rounded on its own and the bits do not depend on the compiler's choice of
// fused multiply-adds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "spchol.h"
#include "spchol_mesh.h"

// Applies to every expression of the file below; HIP's __dmul_rn and
// __dadd_rn are plain operators defined in a header outside its reach, so
// the kernels use the operators directly.
#pragma clang fp contract(off)

namespace {

struct EdgeDesc {      // one stored off-diagonal entry = one mesh edge
    int32_t p, q;      // endpoints, p < q
    int32_t o1, o2;    // opposite corners (o2 = -1 on the boundary)
};

__device__ __forceinline__ double cot_at(const double *x, int32_t o, int32_t p, int32_t q) {
    const double ox = x[2 * o], oy = x[2 * o + 1];
    const double ux = x[2 * p] - ox, uy = x[2 * p + 1] - oy;
    const double vx = x[2 * q] - ox, vy = x[2 * q + 1] - oy;
    const double dot = ux * vx + uy * vy;
    const double cr = fabs(ux * vy - uy * vx);
    return dot / cr;
}

__device__ __forceinline__ double clip(double w, double lo, double hi) {
    return fmin(fmax(w, lo), hi);
}

// Level 1: one thread per edge, every value set.  With shared positions the
// clipped weight is formed once and only the per-set scale is applied per
// set.
__global__ void __launch_bounds__(256)
k_cotan_edges(const EdgeDesc *__restrict__ E, const int32_t *__restrict__ eval, int64_t nedge,
              int32_t batch, const double *__restrict__ pos, int64_t pos_stride,
              const double *__restrict__ scale, double lo, double hi,
              double *__restrict__ vals, int64_t ldv) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nedge) return;
    const EdgeDesc d = E[e];
    const int64_t k = eval[e];
    double w = 0.0;
    for (int32_t s = 0; s < batch; s++) {
        if (s == 0 || pos_stride != 0) {
            const double *x = pos + int64_t(s) * pos_stride;
            double h = 0.5 * cot_at(x, d.o1, d.p, d.q);
            if (d.o2 >= 0) h = h + 0.5 * cot_at(x, d.o2, d.p, d.q);
            w = clip(h, lo, hi);
        }
        const double ws = scale ? clip(w * scale[int64_t(s) * nedge + e], lo, hi) : w;
        vals[int64_t(s) * ldv + k] = -ws;
    }
}

// Level 2: one thread per vertex, every value set: the diagonal from the
// stored edge entries of level 1, in the tables' order, plus c m_p.
__global__ void __launch_bounds__(256)
k_cotan_diag(const int32_t *__restrict__ vdiag, const int32_t *__restrict__ iptr,
             const int32_t *__restrict__ ival, int64_t nv, int32_t batch,
             const double *__restrict__ mass, double coeff, double *__restrict__ vals,
             int64_t ldv) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int32_t a = iptr[v], b = iptr[v + 1];
    const double cm = coeff * mass[v];
    for (int32_t s = 0; s < batch; s++) {
        const double *row = vals + int64_t(s) * ldv;
        double deg = 0.0;
        for (int32_t t = a; t < b; t++) deg = deg - row[ival[t]];
        vals[int64_t(s) * ldv + vdiag[v]] = deg + cm;
    }
}

template <typename V>
hipError_t upload(V **dst, const std::vector<V> &src) {
    const size_t bytes = std::max<size_t>(src.size() * sizeof(V), 8);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), bytes);
    if (e == hipSuccess && !src.empty())
        e = hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice);
    return e;
}

}  // namespace

struct sc_cotan {
    int64_t nv = 0, nedge = 0, nnz = 0;
    int device = -1;
    EdgeDesc *edges = nullptr;  // [nedge]
    int32_t *eval = nullptr;    // [nedge] value index of each edge
    int32_t *vdiag = nullptr;   // [nv] value index of each diagonal
    int32_t *iptr = nullptr;    // [nv + 1]
    int32_t *ival = nullptr;    // [2 nedge] value indices of incident edges, summation order
};

extern "C" {

sc_status sc_cotan_create(int64_t nv, const int64_t *colptr, const int32_t *rowind, int64_t ntri,
                          const int32_t *tris, sc_cotan_t **out) {
    if (!out) return SC_EINVAL;
    *out = nullptr;
    if (nv < 1 || nv >= INT32_MAX || ntri < 0 || !colptr || !rowind || (ntri > 0 && !tris))
        return SC_EINVAL;
    const int64_t nnz = colptr[nv];
    if (colptr[0] != 0 || nnz < nv || nnz >= INT32_MAX) return SC_EPATTERN;
    try {
        // validate the lower CSC pattern and list its off-diagonal entries
        std::vector<int32_t> ep, eq, eval;
        std::vector<int32_t> vdiag(nv);
        for (int64_t c = 0; c < nv; c++) {
            const int64_t a = colptr[c], b = colptr[c + 1];
            if (b <= a || b > nnz || rowind[a] != c) return SC_EPATTERN;
            vdiag[c] = int32_t(a);
            for (int64_t t = a + 1; t < b; t++) {
                if (rowind[t] <= rowind[t - 1] || rowind[t] >= nv) return SC_EPATTERN;
                ep.push_back(int32_t(c));
                eq.push_back(rowind[t]);
                eval.push_back(int32_t(t));
            }
        }
        const int64_t nedge = int64_t(ep.size());
        // the edge of (lo, hi): binary search inside column lo
        auto find_edge = [&](int32_t lo, int32_t hi) -> int64_t {
            const int32_t *first = rowind + colptr[lo] + 1, *last = rowind + colptr[lo + 1];
            const int32_t *it = std::lower_bound(first, last, hi);
            if (it == last || *it != hi) return -1;
            // edges are numbered in storage order skipping the diagonals:
            // value index t in column lo is edge t - (lo + 1)
            return int64_t(it - rowind) - (lo + 1);
        };
        std::vector<EdgeDesc> E(nedge);
        for (int64_t e = 0; e < nedge; e++) E[e] = EdgeDesc{ep[e], eq[e], -1, -1};
        for (int64_t t = 0; t < ntri; t++) {
            const int32_t *v = tris + 3 * t;
            for (int c = 0; c < 3; c++)
                if (v[c] < 0 || v[c] >= nv) return SC_EPATTERN;
            if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) return SC_EPATTERN;
            for (int c = 0; c < 3; c++) {
                const int32_t o = v[c], a = v[(c + 1) % 3], b = v[(c + 2) % 3];
                const int64_t e = find_edge(std::min(a, b), std::max(a, b));
                if (e < 0) return SC_EPATTERN;
                if (E[e].o1 < 0) E[e].o1 = o;
                else if (E[e].o2 < 0) E[e].o2 = o;
                else return SC_EPATTERN;  // more than two triangles
            }
        }
        for (int64_t e = 0; e < nedge; e++)
            if (E[e].o1 < 0) return SC_EPATTERN;  // a stored entry that is no edge
        // incident edges of every vertex: neighbours above (column p, rows
        // ascending), then below (columns q < p ascending)
        std::vector<int32_t> iptr(nv + 1, 0), ival(2 * nedge);
        for (int64_t e = 0; e < nedge; e++) {
            iptr[ep[e] + 1]++;
            iptr[eq[e] + 1]++;
        }
        for (int64_t v = 0; v < nv; v++) iptr[v + 1] += iptr[v];
        std::vector<int32_t> fill(iptr.begin(), iptr.end() - 1);
        for (int64_t e = 0; e < nedge; e++) ival[fill[ep[e]]++] = eval[e];  // column order
        for (int64_t e = 0; e < nedge; e++) ival[fill[eq[e]]++] = eval[e];  // lo ascending
        sc_cotan *A = new sc_cotan();
        A->nv = nv;
        A->nedge = nedge;
        A->nnz = nnz;
        if (hipGetDevice(&A->device) != hipSuccess) {
            delete A;
            return SC_EDEVICE;
        }
        hipError_t err = upload(&A->edges, E);
        if (err == hipSuccess) err = upload(&A->eval, eval);
        if (err == hipSuccess) err = upload(&A->vdiag, vdiag);
        if (err == hipSuccess) err = upload(&A->iptr, iptr);
        if (err == hipSuccess) err = upload(&A->ival, ival);
        if (err != hipSuccess) {
            sc_cotan_destroy(A);
            return err == hipErrorOutOfMemory ? SC_ENOMEM : SC_EDEVICE;
        }
        *out = A;
    } catch (const std::bad_alloc &) {
        return SC_ENOMEM;
    }
    return SC_OK;
}

sc_status sc_cotan_nedges(const sc_cotan_t *A, int64_t *nedge_out) {
    if (!A || !nedge_out) return SC_EINVAL;
    *nedge_out = A->nedge;
    return SC_OK;
}

sc_status sc_cotan_assemble(const sc_cotan_t *A, int32_t batch, const double *pos,
                            int64_t pos_stride, const double *scale, const double *mass,
                            double coeff, double lo, double hi, double *vals, int64_t ldv,
                            void *stream) {
    if (!A || batch < 1 || !pos || !mass || !vals || ldv < A->nnz || pos_stride < 0 ||
        (pos_stride > 0 && pos_stride < 2 * A->nv) || !(lo <= hi))
        return SC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (dev != A->device) return SC_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (A->nedge > 0)
        hipLaunchKernelGGL(k_cotan_edges, dim3(unsigned((A->nedge + 255) / 256)), dim3(256), 0,
                           st, A->edges, A->eval, A->nedge, batch, pos, pos_stride, scale, lo,
                           hi, vals, ldv);
    hipLaunchKernelGGL(k_cotan_diag, dim3(unsigned((A->nv + 255) / 256)), dim3(256), 0, st,
                       A->vdiag, A->iptr, A->ival, A->nv, batch, mass, coeff, vals, ldv);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

void sc_cotan_destroy(sc_cotan_t *A) {
    if (!A) return;
    void *p[] = {A->edges, A->eval, A->vdiag, A->iptr, A->ival};
    for (void *q : p)
        if (q) (void)hipFree(q);
    delete A;
}

}  // extern "C"
