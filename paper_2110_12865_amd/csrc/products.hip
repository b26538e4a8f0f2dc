// Sparse matrix products on fixed patterns (spchol_products.h): the host
// unrolls every entry of C into its term list once; one launch evaluates
// all entries from position tables interleaved per wave of 64 entries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>
#include <new>
#include <vector>

#include "spchol.h"
#include "spchol_products.h"

namespace {

constexpr int kWave = 64;

// One thread per entry of C.  Wave w's terms sit at toff[w] + t*64 + lane
// for t < nterm[w] (the wave's longest list; shorter lists are padded with
// position 0 and masked by the entry's own count), so every index load of a
// wave is 64 consecutive words.  Values of A and B are gathered (they are
// small next to the tables and mostly served from cache).
template <typename T>
__global__ void __launch_bounds__(256)
k_spprod(int64_t nnzC, const int64_t *__restrict__ toff, const int32_t *__restrict__ cnt,
         const int32_t *__restrict__ ia, const int32_t *__restrict__ ib,
         const int32_t *__restrict__ di, int32_t batch, const T *__restrict__ A, int64_t lda,
         const T *__restrict__ B, int64_t ldb, const T *__restrict__ D, int64_t ldd,
         T *__restrict__ C, int64_t ldc) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnzC) return;
    const int64_t w = e / kWave;
    const int lane = int(e % kWave);
    const int64_t base = toff[w];
    const int32_t nt = int32_t((toff[w + 1] - base) / kWave);
    const int32_t c = cnt[e];
    const int32_t d = D ? di[e] : -1;
    for (int32_t s = 0; s < batch; s++) {
        const T *a = A + int64_t(s) * lda;
        const T *b = B + int64_t(s) * ldb;
        T acc = T(0);
        for (int32_t t = 0; t < nt; t++) {
            const int64_t q = base + int64_t(t) * kWave + lane;
            const T x = a[ia[q]], y = b[ib[q]];  // padded slots read position 0
            acc = t < c ? fma(x, y, acc) : acc;
        }
        if (d >= 0) acc += D[int64_t(s) * ldd + d];
        C[int64_t(s) * ldc + e] = acc;
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

bool valid_csr(int64_t rows, int64_t cols, const int64_t *rp, const int32_t *ci) {
    if (rp[0] != 0) return false;
    for (int64_t i = 0; i < rows; i++) {
        if (rp[i + 1] < rp[i]) return false;
        for (int64_t q = rp[i]; q < rp[i + 1]; q++) {
            if (ci[q] < 0 || ci[q] >= cols) return false;
            if (q > rp[i] && ci[q] <= ci[q - 1]) return false;
        }
    }
    return true;
}

}  // namespace

struct sc_spprod {
    int64_t m = 0, n = 0, nnzA = 0, nnzB = 0, nnzD = 0, nnzC = 0, nterms = 0;
    bool has_d = false;
    int device = -1;
    std::vector<int64_t> rowptr;   // C's pattern (host)
    std::vector<int32_t> colind;
    int64_t *toff = nullptr;       // [nwaves + 1]
    int32_t *cnt = nullptr;        // [nnzC]
    int32_t *ia = nullptr, *ib = nullptr;  // [toff[nwaves]]
    int32_t *di = nullptr;         // [nnzC] position in D or -1
    // host copies until the first sc_spprod_run uploads them
    std::vector<int64_t> h_toff;
    std::vector<int32_t> h_cnt, h_ia, h_ib, h_di;
    std::mutex mu;
};

namespace {

// Upload the tables to the current device on first use.
sc_status ensure_uploaded(sc_spprod *P) {
    std::lock_guard<std::mutex> lock(P->mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (P->toff) return dev == P->device ? SC_OK : SC_EINVAL;
    hipError_t err = upload(&P->toff, P->h_toff);
    if (err == hipSuccess) err = upload(&P->cnt, P->h_cnt);
    if (err == hipSuccess) err = upload(&P->ia, P->h_ia);
    if (err == hipSuccess) err = upload(&P->ib, P->h_ib);
    if (err == hipSuccess) err = upload(&P->di, P->h_di);
    if (err != hipSuccess) {
        void *q[] = {P->toff, P->cnt, P->ia, P->ib, P->di};
        for (void *x : q)
            if (x) (void)hipFree(x);
        P->toff = nullptr;
        P->cnt = P->ia = P->ib = P->di = nullptr;
        return err == hipErrorOutOfMemory ? SC_ENOMEM : SC_EDEVICE;
    }
    P->device = dev;
    P->h_toff = {};
    P->h_cnt = P->h_ia = P->h_ib = P->h_di = {};
    return SC_OK;
}

}  // namespace

extern "C" {

sc_status sc_spprod_create(int64_t m, int64_t p, int64_t n, const int64_t *Ar, const int32_t *Ac,
                           const int64_t *Br, const int32_t *Bc, int32_t transB,
                           const int64_t *Dr, const int32_t *Dc, sc_spprod_t **out) {
    if (!out) return SC_EINVAL;
    *out = nullptr;
    if (m < 1 || p < 1 || n < 1 || m >= INT32_MAX || p >= INT32_MAX || n >= INT32_MAX || !Ar ||
        !Ac || !Br || !Bc || (transB != 0 && transB != 1) || (!Dr) != (!Dc))
        return SC_EINVAL;
    const int64_t brows = transB ? n : p, bcols = transB ? p : n;
    if (!valid_csr(m, p, Ar, Ac) || !valid_csr(brows, bcols, Br, Bc)) return SC_EPATTERN;
    if (Dr && !valid_csr(m, n, Dr, Dc)) return SC_EPATTERN;
    if (Ar[m] >= INT32_MAX || Br[brows] >= INT32_MAX || (Dr && Dr[m] >= INT32_MAX))
        return SC_EINVAL;
    try {
        // the rows of the right factor by the inner index k: (j, value
        // position of B_kj), j ascending
        std::vector<int64_t> kp(p + 1, 0);
        std::vector<int32_t> kj, kq;
        if (!transB) {
            kp.assign(Br, Br + p + 1);
            kj.assign(Bc, Bc + Br[p]);
            kq.resize(Br[p]);
            for (int64_t q = 0; q < Br[p]; q++) kq[q] = int32_t(q);
        } else {  // B^T: column k of B, rows j ascending
            for (int64_t q = 0; q < Br[n]; q++) kp[Bc[q] + 1]++;
            for (int64_t k = 0; k < p; k++) kp[k + 1] += kp[k];
            kj.resize(Br[n]);
            kq.resize(Br[n]);
            std::vector<int64_t> fill(kp.begin(), kp.end() - 1);
            for (int64_t j = 0; j < n; j++)
                for (int64_t q = Br[j]; q < Br[j + 1]; q++) {
                    const int64_t f = fill[Bc[q]]++;
                    kj[f] = int32_t(j);
                    kq[f] = int32_t(q);
                }
        }
        sc_spprod *P = new sc_spprod();
        P->m = m;
        P->n = n;
        P->nnzA = Ar[m];
        P->nnzB = Br[brows];
        P->nnzD = Dr ? Dr[m] : 0;
        P->has_d = Dr != nullptr;
        P->rowptr.assign(1, 0);
        // per entry of C: its term list (positions in A and B, ascending k)
        std::vector<int32_t> ecnt, eD, tA, tB;
        std::vector<int64_t> estart;
        std::vector<int32_t> slot(n, -1), cols, rcnt;
        for (int64_t i = 0; i < m; i++) {
            cols.clear();
            for (int64_t qa = Ar[i]; qa < Ar[i + 1]; qa++) {
                const int32_t k = Ac[qa];
                for (int64_t t = kp[k]; t < kp[k + 1]; t++)
                    if (slot[kj[t]] < 0) {
                        slot[kj[t]] = 0;
                        cols.push_back(kj[t]);
                    }
            }
            if (Dr)
                for (int64_t q = Dr[i]; q < Dr[i + 1]; q++)
                    if (slot[Dc[q]] < 0) {
                        slot[Dc[q]] = 0;
                        cols.push_back(Dc[q]);
                    }
            std::sort(cols.begin(), cols.end());
            const int64_t e0 = int64_t(P->colind.size());
            for (size_t u = 0; u < cols.size(); u++) {
                slot[cols[u]] = int32_t(u);
                P->colind.push_back(cols[u]);
            }
            // count, then fill the term lists in ascending k
            rcnt.assign(cols.size(), 0);
            for (int64_t qa = Ar[i]; qa < Ar[i + 1]; qa++) {
                const int32_t k = Ac[qa];
                for (int64_t t = kp[k]; t < kp[k + 1]; t++) rcnt[slot[kj[t]]]++;
            }
            const int64_t t0 = int64_t(tA.size());
            for (size_t u = 0; u < cols.size(); u++) {
                estart.push_back(u == 0 ? t0 : estart.back() + rcnt[u - 1]);
                ecnt.push_back(rcnt[u]);
                eD.push_back(-1);
            }
            int64_t rterms = 0;
            for (int32_t c : rcnt) rterms += c;
            tA.resize(t0 + rterms);
            tB.resize(tA.size());
            std::vector<int64_t> fillp(cols.size());
            for (size_t u = 0; u < cols.size(); u++) fillp[u] = estart[e0 + u];
            for (int64_t qa = Ar[i]; qa < Ar[i + 1]; qa++) {
                const int32_t k = Ac[qa];
                for (int64_t t = kp[k]; t < kp[k + 1]; t++) {
                    const int32_t u = slot[kj[t]];
                    tA[fillp[u]] = int32_t(qa);
                    tB[fillp[u]] = kq[t];
                    fillp[u]++;
                }
            }
            if (Dr)
                for (int64_t q = Dr[i]; q < Dr[i + 1]; q++) eD[e0 + slot[Dc[q]]] = int32_t(q);
            for (int32_t c : cols) slot[c] = -1;
            P->rowptr.push_back(int64_t(P->colind.size()));
        }
        P->nnzC = int64_t(P->colind.size());
        P->nterms = int64_t(tA.size());
        if (P->nnzC >= INT32_MAX) {
            delete P;
            return SC_EINVAL;
        }
        // interleave the term lists per wave of 64 entries
        const int64_t nw = (P->nnzC + kWave - 1) / kWave;
        std::vector<int64_t> toff(nw + 1, 0);
        for (int64_t w = 0; w < nw; w++) {
            int32_t mx = 0;
            for (int64_t e = w * kWave; e < std::min<int64_t>(P->nnzC, (w + 1) * kWave); e++)
                mx = std::max(mx, ecnt[e]);
            toff[w + 1] = toff[w] + int64_t(mx) * kWave;
        }
        std::vector<int32_t> ia(toff[nw], 0), ib(toff[nw], 0);
        for (int64_t e = 0; e < P->nnzC; e++) {
            const int64_t w = e / kWave, lane = e % kWave;
            for (int32_t t = 0; t < ecnt[e]; t++) {
                ia[toff[w] + int64_t(t) * kWave + lane] = tA[estart[e] + t];
                ib[toff[w] + int64_t(t) * kWave + lane] = tB[estart[e] + t];
            }
        }
        P->h_toff = std::move(toff);
        P->h_cnt = std::move(ecnt);
        P->h_ia = std::move(ia);
        P->h_ib = std::move(ib);
        P->h_di = std::move(eD);
        *out = P;
    } catch (const std::bad_alloc &) {
        return SC_ENOMEM;
    }
    return SC_OK;
}

sc_status sc_spprod_info(const sc_spprod_t *P, int64_t *nnzC, int64_t *nterms) {
    if (!P) return SC_EINVAL;
    if (nnzC) *nnzC = P->nnzC;
    if (nterms) *nterms = P->nterms;
    return SC_OK;
}

sc_status sc_spprod_export(const sc_spprod_t *P, int64_t *rowptr, int32_t *colind) {
    if (!P) return SC_EINVAL;
    if (rowptr) std::copy(P->rowptr.begin(), P->rowptr.end(), rowptr);
    if (colind) std::copy(P->colind.begin(), P->colind.end(), colind);
    return SC_OK;
}

sc_status sc_spprod_run(const sc_spprod_t *P, sc_dtype dtype, int32_t batch, const void *A,
                        int64_t lda, const void *B, int64_t ldb, const void *D, int64_t ldd,
                        void *C, int64_t ldc, void *stream) {
    if (!P || batch < 1 || !A || !B || !C || lda < P->nnzA || ldb < P->nnzB || ldc < P->nnzC ||
        (dtype != SC_F64 && dtype != SC_F32) || (P->has_d != (D != nullptr)) ||
        (D && ldd < P->nnzD))
        return SC_EINVAL;
    const sc_status up = ensure_uploaded(const_cast<sc_spprod *>(P));
    if (up != SC_OK) return up;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const dim3 grid(unsigned((P->nnzC + 255) / 256));
    if (dtype == SC_F64)
        hipLaunchKernelGGL(k_spprod<double>, grid, dim3(256), 0, st, P->nnzC, P->toff, P->cnt,
                           P->ia, P->ib, P->di, batch, static_cast<const double *>(A), lda,
                           static_cast<const double *>(B), ldb, static_cast<const double *>(D),
                           ldd, static_cast<double *>(C), ldc);
    else
        hipLaunchKernelGGL(k_spprod<float>, grid, dim3(256), 0, st, P->nnzC, P->toff, P->cnt,
                           P->ia, P->ib, P->di, batch, static_cast<const float *>(A), lda,
                           static_cast<const float *>(B), ldb, static_cast<const float *>(D),
                           ldd, static_cast<float *>(C), ldc);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

void sc_spprod_destroy(sc_spprod_t *P) {
    if (!P) return;
    void *q[] = {P->toff, P->cnt, P->ia, P->ib, P->di};
    for (void *x : q)
        if (x) (void)hipFree(x);
    delete P;
}

}  // extern "C"
