// Built-in fill-reducing ordering for sc_analyze (options.ordering = 2):
// nested dissection of the adjacency graph of A with separators taken from
// breadth-first level structures, for callers that have no coordinates and
// no ordering library.
//
// For a connected vertex set C the separator comes from a rooted level
// structure (George and Liu, "Computer Solution of Large Sparse Positive
// Definite Systems", 1981, ch. 4 and 8): the root is a pseudo-peripheral
// vertex (repeat a breadth-first search from a vertex of least degree in the
// deepest level while the depth grows), and every level of that search
// separates the levels above it from those below.  Among the levels whose
// split leaves between 35% and 65% of C on the near side, the smallest is
// taken; of it only the vertices with a neighbour in the next level are
// kept in the separator (the rest join the near side, which they touch
// only).  The near side, the far side and then the separator are numbered
// in that order, recursively, so every separator is eliminated after both
// parts it splits; sets of at most kLeaf vertices are numbered in
// breadth-first order.  Disconnected sets are split into their components
// first.  The result is one valid elimination order; it has no single
// correct answer, so the tests check validity and quality (fill) only.
#include <algorithm>
#include <cstdint>
#include <vector>

namespace {

constexpr int32_t kLeaf = 32;

struct Graph {
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;
};

// Symmetric adjacency without the diagonal from the lower CSC pattern.
Graph build_graph(int64_t n, const int64_t *colptr, const int32_t *rowind) {
    Graph g;
    g.ptr.assign(n + 1, 0);
    for (int64_t c = 0; c < n; c++)
        for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
            const int32_t r = rowind[p];
            if (r == c) continue;
            g.ptr[r + 1]++;
            g.ptr[c + 1]++;
        }
    for (int64_t i = 0; i < n; i++) g.ptr[i + 1] += g.ptr[i];
    g.adj.resize(g.ptr[n]);
    std::vector<int64_t> fill(g.ptr.begin(), g.ptr.end() - 1);
    for (int64_t c = 0; c < n; c++)
        for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
            const int32_t r = rowind[p];
            if (r == c) continue;
            g.adj[fill[r]++] = int32_t(c);
            g.adj[fill[c]++] = r;
        }
    return g;
}

struct Work {
    const Graph &g;
    // in_set[v] == stamp: v belongs to the set being processed
    std::vector<int32_t> in_set;
    std::vector<int32_t> level;  // BFS level of v in the current search, -1 = unseen
    int32_t stamp = 0;
    explicit Work(const Graph &gr, int64_t n) : g(gr), in_set(n, -1), level(n, -1) {}

    int32_t degree_in(int32_t v) const {
        int32_t d = 0;
        for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; p++) d += in_set[g.adj[p]] == stamp;
        return d;
    }

    // Breadth-first search inside the current set from root; fills order
    // (visit order) and lstart (level boundaries into order).
    void bfs(int32_t root, std::vector<int32_t> &order, std::vector<int32_t> &lstart) {
        order.clear();
        lstart.clear();
        order.push_back(root);
        level[root] = 0;
        lstart.push_back(0);
        size_t head = 0;
        int32_t cur = 0;
        while (head < order.size()) {
            const int32_t v = order[head++];
            if (level[v] != cur) {
                cur = level[v];
                lstart.push_back(int32_t(head - 1));
            }
            for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; p++) {
                const int32_t u = g.adj[p];
                if (in_set[u] == stamp && level[u] < 0) {
                    level[u] = level[v] + 1;
                    order.push_back(u);
                }
            }
        }
        lstart.push_back(int32_t(order.size()));
    }
    void clear_levels(const std::vector<int32_t> &order) {
        for (int32_t v : order) level[v] = -1;
    }
};

}  // namespace

// perm_out[k] = vertex eliminated k-th.  Returns false on allocation failure.
bool spchol_nd_order(int64_t n, const int64_t *colptr, const int32_t *rowind,
                     int32_t *perm_out) {
    try {
        const Graph g = build_graph(n, colptr, rowind);
        Work wk(g, n);
        // a task: vertices to number into perm_out[off, off + size)
        struct Task {
            std::vector<int32_t> verts;
            int64_t off;
        };
        std::vector<Task> stack;
        {
            Task t;
            t.verts.resize(n);
            for (int64_t v = 0; v < n; v++) t.verts[v] = int32_t(v);
            t.off = 0;
            stack.push_back(std::move(t));
        }
        std::vector<int32_t> order, lstart, comp;
        while (!stack.empty()) {
            Task t = std::move(stack.back());
            stack.pop_back();
            const int64_t sz = int64_t(t.verts.size());
            if (sz == 0) continue;
            wk.stamp++;
            for (int32_t v : t.verts) wk.in_set[v] = wk.stamp;
            // first component, found from the smallest vertex of the set
            const int32_t start = *std::min_element(t.verts.begin(), t.verts.end());
            wk.bfs(start, order, lstart);
            if (int64_t(order.size()) < sz) {
                // disconnected: this component first, the rest as a new task
                Task rest;
                rest.off = t.off + int64_t(order.size());
                for (int32_t v : t.verts)
                    if (wk.level[v] < 0) rest.verts.push_back(v);
                comp = order;
                wk.clear_levels(order);
                stack.push_back(std::move(rest));
                Task c;
                c.verts = comp;
                c.off = t.off;
                stack.push_back(std::move(c));
                continue;
            }
            if (sz <= kLeaf) {
                for (int64_t k = 0; k < sz; k++) perm_out[t.off + k] = order[k];
                wk.clear_levels(order);
                continue;
            }
            // pseudo-peripheral root: restart from a least-degree vertex of
            // the deepest level while the depth increases
            int32_t depth = int32_t(lstart.size()) - 2;
            for (int it = 0; it < 8; it++) {
                int32_t best = order[lstart[depth]], bd = wk.degree_in(best);
                for (int32_t q = lstart[depth] + 1; q < lstart[depth + 1]; q++) {
                    const int32_t d = wk.degree_in(order[q]);
                    if (d < bd) {
                        bd = d;
                        best = order[q];
                    }
                }
                wk.clear_levels(order);
                wk.bfs(best, order, lstart);
                const int32_t nd = int32_t(lstart.size()) - 2;
                if (nd <= depth) break;
                depth = nd;
            }
            if (depth < 2) {  // too shallow to split: number it as it is
                for (int64_t k = 0; k < sz; k++) perm_out[t.off + k] = order[k];
                wk.clear_levels(order);
                continue;
            }
            // separator level: the smallest among balanced splits
            int32_t sep = -1;
            for (int32_t m = 1; m < depth; m++) {
                const double near = double(lstart[m]) / double(sz);
                if (near < 0.35 || near > 0.65) continue;
                if (sep < 0 || lstart[m + 1] - lstart[m] < lstart[sep + 1] - lstart[sep]) sep = m;
            }
            if (sep < 0) {  // no balanced level: the one holding the median vertex
                sep = 1;
                while (sep < depth - 1 && lstart[sep + 1] <= sz / 2) sep++;
            }
            Task a, b;
            std::vector<int32_t> s;
            for (int32_t q = 0; q < lstart[sep]; q++) a.verts.push_back(order[q]);
            for (int32_t q = lstart[sep]; q < lstart[sep + 1]; q++) {
                const int32_t v = order[q];
                bool touches_far = false;
                for (int64_t p = g.ptr[v]; p < g.ptr[v + 1] && !touches_far; p++) {
                    const int32_t u = g.adj[p];
                    touches_far = wk.in_set[u] == wk.stamp && wk.level[u] == sep + 1;
                }
                (touches_far ? s : a.verts).push_back(v);
            }
            for (int32_t q = lstart[sep + 1]; q < int32_t(order.size()); q++)
                b.verts.push_back(order[q]);
            wk.clear_levels(order);
            a.off = t.off;
            b.off = t.off + int64_t(a.verts.size());
            const int64_t s0 = b.off + int64_t(b.verts.size());
            for (size_t k = 0; k < s.size(); k++) perm_out[s0 + int64_t(k)] = s[k];
            stack.push_back(std::move(b));
            stack.push_back(std::move(a));
        }
    } catch (...) {
        return false;
    }
    return true;
}
