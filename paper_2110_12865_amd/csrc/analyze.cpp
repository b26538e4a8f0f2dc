// Host symbolic pass: everything that depends only on the sparsity pattern.
//
// This is the counterpart of the paper's one-time analysis (Sec. 3.2, 4.2 -
// 4.4): instead of tracing a program into an expression DAG, the DAG of
// numeric Cholesky is derived from the pattern directly.
//   * Global intermediates (Sec. 4.2.1) are the entries of L; the
//     supernodal update blocks are second-level intermediates.
//   * Tagged dense blocks (Sec. 4.2.4) are the supernodes, found
//     automatically (fundamental supernodes, then amalgamation).
//   * Grouping by level (Sec. 4.3) is the level of a supernode in the
//     supernodal elimination tree, counted as the longest path from the
//     leaves so that no member of a level depends on another.
//   * Leaf harvesting (Sec. 4.4) becomes the index tables the kernels read:
//     row lists, relative maps child -> parent and the value scatter map.
//
// Textbook algorithms used: Liu's elimination tree with path compression,
// column counts by row-subtree traversal, supernode detection from column
// counts, and relaxed amalgamation with a zero-fraction threshold.
#include <algorithm>
#include <climits>
#include <cstring>
#include <new>

#include "plan.hpp"

namespace {

struct Groups {
    int32_t f0, f1;   // fundamental supernodes [f0, f1]
    int64_t W, c, Z;  // width, rows, stored zeros
};

bool accept_merge(const sc_options &o, int64_t W, int64_t Z, int64_t E) {
    if (W <= o.relax_cols) return true;
    double frac = E > 0 ? double(Z) / double(E) : 0.0;
    if (W <= 16) return frac < 0.8;
    if (W <= 48) return frac < 0.1;
    return frac < o.relax_zeros;
}

}  // namespace

sc_status spchol_build_plan(int64_t n, const int64_t *colptr,
                            const int32_t *rowind, const int32_t *perm_in,
                            const sc_options &opt, int32_t nblk, const int64_t *blk_col0,
                            const int64_t *blk_val0, sc_plan **out) {
    if (!colptr || !rowind || !out || n < 1 || nblk < 1) return SC_EINVAL;
    if (nblk > 1 && (!blk_col0 || !blk_val0)) return SC_EINVAL;
    if (n > INT32_MAX - 1) return SC_EINVAL;
    // ---- validation of the lower-CSC pattern -----------------------------
    if (colptr[0] != 0) return SC_EPATTERN;
    for (int64_t c = 0; c < n; c++) {
        int64_t a = colptr[c], b = colptr[c + 1];
        if (b <= a) return SC_EPATTERN;  // the diagonal is required
        if (rowind[a] != c) return SC_EPATTERN;
        for (int64_t p = a + 1; p < b; p++) {
            if (rowind[p] <= rowind[p - 1] || rowind[p] >= n) return SC_EPATTERN;
        }
    }
    const int64_t nnzA = colptr[n];

    sc_plan *P = new (std::nothrow) sc_plan();
    if (!P) return SC_ENOMEM;
    try {
        P->n = n;
        P->nnzA = nnzA;
        P->opt = opt;
        P->nblk = nblk;
        if (nblk == 1) {
            P->blk_col0 = {0, n};
            P->blk_val0 = {0, nnzA};
        } else {
            P->blk_col0.assign(blk_col0, blk_col0 + nblk + 1);
            P->blk_val0.assign(blk_val0, blk_val0 + nblk + 1);
        }
        if (P->blk_col0[0] != 0 || P->blk_col0[nblk] != n || P->blk_val0[0] != 0 ||
            P->blk_val0[nblk] != nnzA) {
            delete P;
            return SC_EINVAL;
        }
        P->colblk.assign(n, 0);
        for (int32_t k = 0; k < nblk; k++) {
            if (P->blk_col0[k + 1] <= P->blk_col0[k] ||
                colptr[P->blk_col0[k]] != P->blk_val0[k]) {
                delete P;
                return SC_EINVAL;
            }
            for (int64_t j = P->blk_col0[k]; j < P->blk_col0[k + 1]; j++) P->colblk[j] = k;
        }
        for (int64_t c = 0; c < n; c++)
            for (int64_t p = colptr[c]; p < colptr[c + 1]; p++)
                if (P->colblk[rowind[p]] != P->colblk[c]) {
                    delete P;
                    return SC_EPATTERN;
                }
        P->perm.resize(n);
        P->pinv.assign(n, -1);
        for (int64_t k = 0; k < n; k++) {
            int32_t o = perm_in ? perm_in[k] : int32_t(k);
            if (o < 0 || o >= n || P->pinv[o] != -1 || P->colblk[o] != P->colblk[k]) {
                delete P;
                return SC_EPATTERN;
            }
            P->perm[k] = o;
            P->pinv[o] = int32_t(k);
        }
        const std::vector<int32_t> &pinv = P->pinv;

        // ---- permuted lower triangle, by columns and by rows -------------
        std::vector<int64_t> &acp = P->acolptr;
        acp.assign(n + 1, 0);
        std::vector<int64_t> rcp(n + 1, 0);  // strict lower by rows
        for (int64_t c = 0; c < n; c++)
            for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
                int32_t i = pinv[rowind[p]], j = pinv[c];
                int32_t lo = std::min(i, j), hi = std::max(i, j);
                acp[lo + 1]++;
                if (hi != lo) rcp[hi + 1]++;
            }
        for (int64_t j = 0; j < n; j++) { acp[j + 1] += acp[j]; rcp[j + 1] += rcp[j]; }
        std::vector<int32_t> arow(nnzA);
        P->avidx.resize(nnzA);
        std::vector<int32_t> rcol(rcp[n]);
        {
            std::vector<int64_t> fa(acp.begin(), acp.end() - 1), fr(rcp.begin(), rcp.end() - 1);
            for (int64_t c = 0; c < n; c++)
                for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
                    int32_t i = pinv[rowind[p]], j = pinv[c];
                    int32_t lo = std::min(i, j), hi = std::max(i, j);
                    int64_t q = fa[lo]++;
                    arow[q] = hi;
                    P->avidx[q] = p;
                    if (hi != lo) rcol[fr[hi]++] = lo;
                }
        }
        // sort each permuted column by row (keeping the value index along)
        {
            std::vector<std::pair<int32_t, int64_t>> tmp;
            for (int64_t j = 0; j < n; j++) {
                int64_t a = acp[j], b = acp[j + 1];
                bool sorted = true;
                for (int64_t q = a + 1; q < b && sorted; q++) sorted = arow[q] > arow[q - 1];
                if (sorted) continue;
                tmp.clear();
                for (int64_t q = a; q < b; q++) tmp.emplace_back(arow[q], P->avidx[q]);
                std::sort(tmp.begin(), tmp.end());
                for (int64_t q = a; q < b; q++) { arow[q] = tmp[q - a].first; P->avidx[q] = tmp[q - a].second; }
            }
        }

        // ---- elimination tree (Liu, path compression) --------------------
        std::vector<int32_t> &parent = P->parent;
        parent.assign(n, -1);
        {
            std::vector<int32_t> anc(n, -1);
            for (int64_t i = 0; i < n; i++) {
                for (int64_t q = rcp[i]; q < rcp[i + 1]; q++) {
                    int32_t k = rcol[q];
                    while (k != -1 && k < i) {
                        int32_t nx = anc[k];
                        anc[k] = int32_t(i);
                        if (nx == -1) parent[k] = int32_t(i);
                        k = nx;
                    }
                }
            }
        }
        // ---- column counts: every row subtree visits its columns once ----
        std::vector<int64_t> &cc = P->colcount;
        cc.assign(n, 1);
        {
            std::vector<int32_t> mark(n, -1);
            for (int64_t i = 0; i < n; i++) {
                mark[i] = int32_t(i);
                for (int64_t q = rcp[i]; q < rcp[i + 1]; q++) {
                    int32_t k = rcol[q];
                    while (mark[k] != i) {
                        mark[k] = int32_t(i);
                        cc[k]++;
                        k = parent[k];
                    }
                }
            }
        }
        P->nnzL = 0;
        P->flops = 0.0;
        for (int64_t j = 0; j < n; j++) {
            P->nnzL += cc[j];
            P->flops += double(cc[j]) * double(cc[j]);
        }
        {
            std::vector<int32_t> depth(n, 0);
            int64_t h = 0;
            for (int64_t j = n - 1; j >= 0; j--) {
                depth[j] = parent[j] < 0 ? 1 : depth[parent[j]] + 1;
                h = std::max<int64_t>(h, depth[j]);
            }
            P->etree_height = h;
        }

        // ---- fundamental supernodes (nested column structures) -----------
        std::vector<int32_t> &ff = P->ffirst;
        ff.clear();
        for (int64_t j = 0; j < n; j++) {
            bool cont = j > 0 && parent[j - 1] == j && cc[j - 1] == cc[j] + 1;
            if (!cont) ff.push_back(int32_t(j));
        }
        const int32_t nf = int32_t(ff.size());
        ff.push_back(int32_t(n));
        std::vector<int32_t> col2f(n);
        for (int32_t t = 0; t < nf; t++)
            for (int32_t j = ff[t]; j < ff[t + 1]; j++) col2f[j] = t;
        std::vector<int32_t> fpar(nf, -1);
        for (int32_t t = 0; t < nf; t++) {
            int32_t pc = parent[ff[t + 1] - 1];
            fpar[t] = pc < 0 ? -1 : col2f[pc];
        }
        // children of fundamental supernodes (CSR)
        std::vector<int32_t> fchp(nf + 1, 0), fch;
        for (int32_t t = 0; t < nf; t++) if (fpar[t] >= 0) fchp[fpar[t] + 1]++;
        for (int32_t t = 0; t < nf; t++) fchp[t + 1] += fchp[t];
        fch.resize(fchp[nf]);
        {
            std::vector<int32_t> fl(fchp.begin(), fchp.end() - 1);
            for (int32_t t = 0; t < nf; t++) if (fpar[t] >= 0) fch[fl[fpar[t]]++] = t;
        }
        // exact structure of each fundamental supernode's first column:
        // its own columns, rows of A below it, and the children's update rows
        std::vector<int64_t> &frp = P->frowptr;
        std::vector<int32_t> &fr = P->frows;
        frp.assign(nf + 1, 0);
        for (int32_t t = 0; t < nf; t++) frp[t + 1] = frp[t] + cc[ff[t]];
        fr.resize(frp[nf]);
        {
            std::vector<int32_t> mark(n, -1);
            for (int32_t t = 0; t < nf; t++) {
                int32_t f = ff[t], l = ff[t + 1] - 1, w = l - f + 1;
                int64_t base = frp[t], len = 0;
                for (int32_t j = f; j <= l; j++) { fr[base + len++] = j; mark[j] = t; }
                int64_t cap = frp[t + 1] - base;
                auto add = [&](int32_t r) {
                    if (mark[r] != t) {
                        mark[r] = t;
                        if (len >= cap) throw std::bad_alloc();  // structure mismatch
                        fr[base + len++] = r;
                    }
                };
                for (int32_t j = f; j <= l; j++)
                    for (int64_t q = acp[j]; q < acp[j + 1]; q++)
                        if (arow[q] > l) add(arow[q]);
                for (int32_t q = fchp[t]; q < fchp[t + 1]; q++) {
                    int32_t u = fch[q];
                    int32_t wu = ff[u + 1] - ff[u];
                    for (int64_t r = frp[u] + wu; r < frp[u + 1]; r++)
                        if (fr[r] > l) add(fr[r]);
                }
                if (len != cap) throw std::bad_alloc();
                std::sort(fr.begin() + base + w, fr.begin() + base + len);
            }
        }

        // ---- relaxed amalgamation of contiguous parent/child chains ------
        std::vector<Groups> grp;
        grp.reserve(nf);
        for (int32_t p = 0; p < nf; p++) {
            int64_t wp = ff[p + 1] - ff[p], cp = cc[ff[p]];
            Groups G{p, p, wp, cp, 0};
            if (opt.relax && !grp.empty()) {
                const Groups &g = grp.back();
                if (fpar[g.f1] == p) {
                    int64_t W2 = g.W + wp, c2 = g.W + cp;
                    int64_t Z2 = g.Z + g.W * (c2 - g.c);
                    int64_t E2 = W2 * c2 - W2 * (W2 - 1) / 2;
                    if (accept_merge(opt, W2, Z2, E2)) {
                        G = Groups{g.f0, p, W2, c2, Z2};
                        grp.pop_back();
                    }
                }
            }
            grp.push_back(G);
        }
        const int32_t ns = int32_t(grp.size());
        P->ns = ns;
        P->sn.assign(ns, SnDesc{});
        P->col2sn.assign(n, -1);
        std::vector<int64_t> rowptr(ns + 1, 0);
        for (int32_t s = 0; s < ns; s++) {
            SnDesc &d = P->sn[s];
            d.first = ff[grp[s].f0];
            d.w = int32_t(grp[s].W);
            d.c = int32_t(grp[s].c);
            d.m = d.c - d.w;
            for (int32_t j = d.first; j < d.first + d.w; j++) P->col2sn[j] = s;
            rowptr[s + 1] = rowptr[s] + d.c;
        }
        P->rows.resize(rowptr[ns]);
        for (int32_t s = 0; s < ns; s++) {
            SnDesc &d = P->sn[s];
            d.rowptr = rowptr[s];
            int64_t o = rowptr[s];
            for (int32_t j = 0; j < d.w; j++) P->rows[o + j] = d.first + j;
            int32_t T = grp[s].f1, wT = ff[T + 1] - ff[T];
            int64_t q = o + d.w;
            for (int64_t r = frp[T] + wT; r < frp[T + 1]; r++) P->rows[q++] = fr[r];
            if (q != rowptr[s + 1]) throw std::bad_alloc();
            int32_t pc = parent[d.first + d.w - 1];
            d.parent = pc < 0 ? -1 : P->col2sn[pc];
            // no entry joins two blocks, so a supernode never spans two
            d.blk = P->colblk[d.first];
            d.bcol0 = int32_t(P->blk_col0[d.blk]);
        }
        // children (ascending), levels
        std::vector<int32_t> chp(ns + 1, 0);
        for (int32_t s = 0; s < ns; s++) if (P->sn[s].parent >= 0) chp[P->sn[s].parent + 1]++;
        for (int32_t s = 0; s < ns; s++) chp[s + 1] += chp[s];
        P->chlist.resize(chp[ns]);
        {
            std::vector<int32_t> fl(chp.begin(), chp.end() - 1);
            for (int32_t s = 0; s < ns; s++)
                if (P->sn[s].parent >= 0) P->chlist[fl[P->sn[s].parent]++] = s;
        }
        int32_t nlev = 0;
        for (int32_t s = 0; s < ns; s++) {
            SnDesc &d = P->sn[s];
            d.chbeg = chp[s];
            d.chend = chp[s + 1];
            d.level = 0;
        }
        for (int32_t s = 0; s < ns; s++) {
            int32_t p = P->sn[s].parent;
            if (p >= 0) P->sn[p].level = std::max(P->sn[p].level, P->sn[s].level + 1);
            nlev = std::max(nlev, P->sn[s].level + 1);
        }
        P->nlevels = nlev;
        // relative maps: where each update row of s sits in its parent's rows
        int64_t rel = 0, loff = 0, uoff = 0;
        for (int32_t s = 0; s < ns; s++) {
            SnDesc &d = P->sn[s];
            d.relptr = rel;
            d.loff = loff;
            d.uoff = uoff;
            rel += d.m;
            loff += int64_t(d.c) * d.w;
            uoff += int64_t(d.m) * d.m;
            P->max_front = std::max<int64_t>(P->max_front, d.c);
            P->max_width = std::max<int64_t>(P->max_width, d.w);
        }
        P->relsize = rel;
        P->Lsize = loff;
        P->Usize = uoff;
        P->relmap.resize(rel);
        for (int32_t s = 0; s < ns; s++) {
            const SnDesc &d = P->sn[s];
            if (d.m == 0) continue;
            if (d.parent < 0) throw std::bad_alloc();  // a root has no update rows
            const SnDesc &pd = P->sn[d.parent];
            const int32_t *Rs = &P->rows[d.rowptr];
            const int32_t *Rp = &P->rows[pd.rowptr];
            int32_t q = 0;
            for (int32_t i = 0; i < d.m; i++) {
                int32_t r = Rs[d.w + i];
                while (q < pd.c && Rp[q] < r) q++;
                if (q >= pd.c || Rp[q] != r) throw std::bad_alloc();
                P->relmap[d.relptr + i] = q;
            }
        }
        // value scatter map: offset of each A entry inside its L block
        for (int32_t s = 0; s < ns; s++)
            if (int64_t(P->sn[s].c) * P->sn[s].w >= INT32_MAX) {
                delete P;
                return SC_EINVAL;  // a single front beyond 2^31 scalars
            }
        P->aoff.resize(nnzA);
        for (int64_t j = 0; j < n; j++) {
            const SnDesc &d = P->sn[P->col2sn[j]];
            const int32_t *R = &P->rows[d.rowptr];
            int32_t q = int32_t(j - d.first);
            for (int64_t e = acp[j]; e < acp[j + 1]; e++) {
                int32_t r = arow[e];
                while (q < d.c && R[q] < r) q++;
                if (q >= d.c || R[q] != r) throw std::bad_alloc();
                P->aoff[e] = int32_t((j - d.first) * int64_t(d.c) + q);
            }
        }

        // ---- both triangles by rows (caller's numbering) for A x ---------
        P->csr_ptr.assign(n + 1, 0);
        for (int64_t c = 0; c < n; c++)
            for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
                P->csr_ptr[rowind[p] + 1]++;
                if (rowind[p] != c) P->csr_ptr[c + 1]++;
            }
        for (int64_t i = 0; i < n; i++) P->csr_ptr[i + 1] += P->csr_ptr[i];
        P->csr_col.resize(P->csr_ptr[n]);
        P->csr_vidx.resize(P->csr_ptr[n]);
        {
            std::vector<int64_t> fl(P->csr_ptr.begin(), P->csr_ptr.end() - 1);
            for (int64_t c = 0; c < n; c++)
                for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
                    const int32_t r = rowind[p];
                    int64_t q = fl[r]++;
                    P->csr_col[q] = int32_t(c);
                    P->csr_vidx[q] = p;
                    if (r != c) {
                        q = fl[c]++;
                        P->csr_col[q] = r;
                        P->csr_vidx[q] = p;
                    }
                }
        }

        // sliced by 64 rows for the batched product: entry k of row
        // 64 s + l at sell_ptr[s] + 64 k + l, rows padded to the longest row
        // of their slice (padding: column 0, vidx -1)
        {
            const int64_t nsl = (n + kSellRows - 1) / kSellRows;
            P->sell_ptr.assign(nsl + 1, 0);
            for (int64_t sl = 0; sl < nsl; sl++) {
                int64_t len = 0;
                for (int64_t i = sl * kSellRows; i < std::min<int64_t>(n, (sl + 1) * kSellRows); i++)
                    len = std::max(len, P->csr_ptr[i + 1] - P->csr_ptr[i]);
                P->sell_ptr[sl + 1] = P->sell_ptr[sl] + kSellRows * len;
            }
            P->sell_col.assign(P->sell_ptr[nsl], 0);
            P->sell_vidx.assign(P->sell_ptr[nsl], -1);
            for (int64_t i = 0; i < n; i++) {
                const int64_t base = P->sell_ptr[i / kSellRows] + i % kSellRows;
                for (int64_t q = P->csr_ptr[i]; q < P->csr_ptr[i + 1]; q++) {
                    const int64_t e = base + kSellRows * (q - P->csr_ptr[i]);
                    P->sell_col[e] = P->csr_col[q];
                    P->sell_vidx[e] = P->csr_vidx[q];
                }
            }
        }

        // ---- row and column of every stored entry (caller's numbering),
        // for the value gradients of the adjoint ---------------------------
        P->val_row.assign(rowind, rowind + colptr[n]);
        P->val_col.resize(size_t(colptr[n]));
        for (int64_t c = 0; c < n; c++)
            for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) P->val_col[p] = int32_t(c);

        // ---- level schedule ----------------------------------------------
        int32_t small_front = opt.small_front > 0 ? opt.small_front : 64;
        P->opt.small_front = small_front;
        std::vector<std::vector<int32_t>> bys(nlev), byb(nlev), bya(nlev);
        std::vector<char> small_sn(ns, 0);
        for (int32_t s = 0; s < ns; s++) {
            const SnDesc &d = P->sn[s];
            bya[d.level].push_back(s);
            if (d.c <= small_front && (d.c <= 64 || front_wg_fits(d.c, d.w))) {
                bys[d.level].push_back(s);
                small_sn[s] = 1;
            }
            else byb[d.level].push_back(s);
        }
        P->lvl_small_ptr.assign(nlev + 1, 0);
        P->lvl_big_ptr.assign(nlev + 1, 0);
        P->lvl_ptr.assign(nlev + 1, 0);
        P->lvl_small_maxc.assign(nlev, 0);
        P->lvl_big_maxc.assign(nlev, 0);
        P->lvl_big_maxw.assign(nlev, 0);
        P->lvl_maxc.assign(nlev, 0);
        P->lvl_bigcols.assign(nlev, 0);
        for (int32_t l = 0; l < nlev; l++) {
            for (int32_t s : bys[l]) {
                P->lvl_small.push_back(s);
                P->lvl_small_maxc[l] = std::max(P->lvl_small_maxc[l], P->sn[s].c);
            }
            for (int32_t s : byb[l]) {
                P->lvl_big.push_back(s);
                P->lvl_big_maxc[l] = std::max(P->lvl_big_maxc[l], P->sn[s].c);
                P->lvl_big_maxw[l] = std::max(P->lvl_big_maxw[l], P->sn[s].w);
                P->lvl_bigcols[l] += P->sn[s].c;
            }
            for (int32_t s : bya[l]) {
                P->lvl_sn.push_back(s);
                P->lvl_maxc[l] = std::max(P->lvl_maxc[l], P->sn[s].c);
            }
            P->lvl_small_ptr[l + 1] = int32_t(P->lvl_small.size());
            P->lvl_big_ptr[l + 1] = int32_t(P->lvl_big.size());
            P->max_lvl_big = std::max(P->max_lvl_big, P->lvl_big_ptr[l + 1] - P->lvl_big_ptr[l]);
            P->lvl_ptr[l + 1] = int32_t(P->lvl_sn.size());
        }
        // assembly descriptors of the large fronts
        P->lvl_colent_off.assign(nlev, 0);
        for (int32_t l = 0; l < nlev; l++) {
            P->lvl_colent_off[l] = int64_t(P->asm_col.size());
            for (int32_t e = P->lvl_big_ptr[l]; e < P->lvl_big_ptr[l + 1]; e++) {
                const SnDesc &d = P->sn[P->lvl_big[e]];
                const int32_t nch = d.chend - d.chbeg;
                std::vector<std::vector<AsmPiece>> per(d.c);  // per target column
                for (int32_t q = 0; q < nch; q++) {
                    const SnDesc &cd = P->sn[P->chlist[d.chbeg + q]];
                    for (int32_t jc = 0; jc < cd.m; jc++) {
                        const int32_t tj = P->relmap[cd.relptr + jc];
                        for (int32_t i0 = jc; i0 < cd.m; i0 += kAsmPiece)
                            per[tj].push_back(AsmPiece{cd.uoff + int64_t(jc) * cd.m + i0,
                                                       cd.relptr + i0,
                                                       std::min(kAsmPiece, cd.m - i0), 0});
                    }
                }
                for (int32_t tj = 0; tj < d.c; tj++) {
                    AsmCol a{};
                    a.c = d.c;
                    a.tj = tj;
                    a.base = tj * d.c;
                    a.isU = tj >= d.w;
                    a.dst = tj < d.w ? d.loff + int64_t(tj) * d.c
                                     : d.uoff + int64_t(tj - d.w) * d.m - d.w;
                    if (tj < d.w) {
                        a.a0 = P->acolptr[d.first + tj];
                        a.na = int32_t(P->acolptr[d.first + tj + 1] - a.a0);
                    }
                    a.ch0 = int32_t(P->asm_pc.size());
                    a.nch = int32_t(per[tj].size());
                    P->asm_pc.insert(P->asm_pc.end(), per[tj].begin(), per[tj].end());
                    P->asm_col.push_back(a);
                }
                if (int64_t(P->asm_pc.size()) >= INT32_MAX) throw std::bad_alloc();
            }
        }

        // solve schedule and per-supernode solve workspaces
        P->slv_cls_ptr.assign(size_t(nlev) * kSolveClasses + 1, 0);
        P->slv_pan_ptr.assign(nlev + 1, 0);
        if (int64_t(P->rows.size()) >= INT32_MAX) throw std::bad_alloc();
        P->slv_pan_maxw.assign(nlev, 0);
        P->slv_pan_maxc.assign(nlev, 0);
        for (int32_t s = 0; s < ns; s++) { P->sn[s].dinv = -1; P->sn[s].part = 0; }
        for (int32_t l = 0; l < nlev; l++) {
            for (int32_t s : bya[l]) {
                SnDesc &d = P->sn[s];
                if (!solve_by_panels(d)) continue;
                const int64_t np = (d.w + kSolvePanel - 1) / kSolvePanel;
                d.dinv = P->dinv_size;
                P->dinv_size += np * kSolvePanel * kSolvePanel;
                d.part = P->part_size;
                P->part_size += ((d.c + kSolveChunk - 1) / kSolveChunk) * kSolvePanel;
                P->slv_pan.push_back(s);
                P->slv_pan_maxw[l] = std::max(P->slv_pan_maxw[l], d.w);
                P->slv_pan_maxc[l] = std::max(P->slv_pan_maxc[l], d.c);
                P->npan++;
            }
            for (int k = 0; k < kSolveClasses; k++) {
                for (int32_t s : bya[l]) {
                    const SnDesc &d = P->sn[s];
                    if (!solve_by_panels(d) && solve_class(d.c) == k) P->slv_small.push_back(s);
                }
                P->slv_cls_ptr[size_t(l) * kSolveClasses + k + 1] = int32_t(P->slv_small.size());
            }
            P->slv_pan_ptr[l + 1] = int32_t(P->slv_pan.size());
        }
        // whole-block inverses of the diagonal blocks, for the levels whose
        // panel-solved supernodes are all narrow enough
        P->xoff.assign(ns, -1);
        P->slv_pan_x.assign(nlev, 0);
        P->xg_ptr.assign(nlev + 1, 0);
        for (int32_t l = 0; l < nlev; l++) {
            const int32_t e0 = P->slv_pan_ptr[l], e1 = P->slv_pan_ptr[l + 1];
            if (opt.panel_inverse >= 0 && e0 < e1 && P->slv_pan_maxw[l] <= kXMaxW) {
                P->slv_pan_x[l] = 1;
                for (int32_t e = e0; e < e1; e++) {
                    const int32_t s = P->slv_pan[e];
                    const SnDesc &d = P->sn[s];
                    const int64_t w = d.w;
                    P->xoff[s] = P->xsize;
                    P->xsize += w * w;
                    P->x_list.push_back(s);
                    P->x_nbmax = std::max<int32_t>(P->x_nbmax, int32_t((w + kSolvePanel - 1) / kSolvePanel));
                    for (int32_t i = 0; i < d.c; i++) {
                        P->xg_q.push_back(int32_t(d.rowptr + i));
                        P->xg_y.push_back(i < d.w ? d.first + i : -1);
                    }
                }
            }
            P->xg_ptr[l + 1] = int32_t(P->xg_q.size());
        }
        P->slv_small_x.assign(nlev, 0);
        for (int32_t l = 0; l < nlev && opt.panel_inverse >= 0; l++) {
            const int32_t e0 = P->slv_cls_ptr[size_t(l) * kSolveClasses];
            const int32_t e1 = P->slv_cls_ptr[size_t(l + 1) * kSolveClasses];
            if (e0 == e1 || e1 - e0 > kXSmallMax) continue;
            P->slv_small_x[l] = 1;
            P->xs_lev = l;
            for (int32_t e = e0; e < e1; e++) {
                const int32_t s = P->slv_small[e];
                const int64_t w = P->sn[s].w;
                P->xoff[s] = P->xsize;
                P->xsize += w * w;
                P->xs_list.push_back(s);
            }
        }
        // widest first: the longest chains of the inversion start first
        std::stable_sort(P->x_list.begin(), P->x_list.end(),
                         [&](int32_t a, int32_t b) { return P->sn[a].w > P->sn[b].w; });
        // panel-solved supernodes whose diagonal blocks the tiled factor
        // does not invert (small fronts): inverted after the factorization
        for (int32_t s : P->slv_pan)
            if (small_sn[s]) P->dinv_list.push_back(s);
        // batch-interleaved solve items and the chunks of the L copy
        P->soa_it_ptr.assign(nlev + 1, 0);
        P->grow_ptr.assign(nlev + 1, 0);
        P->soa_psize = 0;
        {
            std::vector<std::pair<int64_t, int64_t>> iv, ivx;
            for (int32_t l = 0; l < nlev; l++) {
                for (int32_t e = P->slv_cls_ptr[size_t(l) * kSolveClasses];
                     e < P->slv_cls_ptr[size_t(l + 1) * kSolveClasses]; e++) {
                    const int32_t s = P->slv_small[e];
                    SnDesc &d = P->sn[s];
                    d.part = P->soa_psize;
                    for (int32_t r0 = d.w; r0 < d.c; r0 += kSoaRows) {
                        P->soa_it_s.push_back(s);
                        P->soa_it_r0.push_back(r0);
                        P->soa_psize += d.w;
                    }
                    iv.emplace_back(d.loff, d.loff + int64_t(d.c) * d.w);
                    P->soa_copy_lev = l;
                    if (!P->slv_small_x[l]) {
                        ivx.emplace_back(d.loff, d.loff + int64_t(d.c) * d.w);
                        P->soa_copy_lev_x = l;
                    }
                }
                P->soa_it_ptr[l + 1] = int32_t(P->soa_it_s.size());
                for (int32_t e = P->slv_cls_ptr[size_t(l) * kSolveClasses];
                     e < P->slv_cls_ptr[size_t(l + 1) * kSolveClasses]; e++) {
                    const SnDesc &d = P->sn[P->slv_small[e]];
                    for (int32_t i = 0; i < d.c; i++) {
                        P->grow_q.push_back(int32_t(d.rowptr + i));
                        P->grow_y.push_back(i < d.w ? d.first + i : -1);
                    }
                }
                P->grow_ptr[l + 1] = int32_t(P->grow_q.size());
            }
            // the copy skips the supernodes of levels solved with whole-block
            // inverses when the numeric object has them (soa_chunks_x)
            auto chunks = [](std::vector<std::pair<int64_t, int64_t>> &v,
                             std::vector<int64_t> &out) {
                std::sort(v.begin(), v.end());
                int64_t covered = 0;  // every scalar below this is already covered
                for (const auto &q : v) {
                    int64_t k = std::max(q.first, covered);
                    for (; k < q.second; k += kSoaChunk) out.push_back(k);
                    covered = std::max(covered, k);
                }
            };
            chunks(iv, P->soa_chunks);
            chunks(ivx, P->soa_chunks_x);
        }
        // forward-solve gather map (children in chlist order)
        P->gptr.assign(P->rows.size() + 1, 0);
        for (int32_t s = 0; s < ns; s++) {
            const SnDesc &d = P->sn[s];
            if (d.m == 0) continue;
            const SnDesc &pd = P->sn[d.parent];
            for (int32_t i = 0; i < d.m; i++) P->gptr[pd.rowptr + P->relmap[d.relptr + i] + 1]++;
        }
        for (size_t q = 0; q + 1 < P->gptr.size(); q++) P->gptr[q + 1] += P->gptr[q];
        P->gidx.assign(P->gptr.back(), 0);
        {
            std::vector<int32_t> fill(P->gptr.begin(), P->gptr.end() - 1);
            for (int32_t s = 0; s < ns; s++)
                for (int32_t q = P->sn[s].chbeg; q < P->sn[s].chend; q++) {
                    const SnDesc &cd = P->sn[P->chlist[q]];
                    for (int32_t i = 0; i < cd.m; i++) {
                        const int64_t slot = P->sn[s].rowptr + P->relmap[cd.relptr + i];
                        P->gidx[fill[slot]++] = int32_t(cd.rowptr + cd.w + i);
                    }
                }
        }
    } catch (const std::bad_alloc &) {
        delete P;
        return SC_ENOMEM;
    }
    *out = P;
    return SC_OK;
}
