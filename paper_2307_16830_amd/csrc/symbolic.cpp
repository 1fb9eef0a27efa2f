// Symbolic analysis of the condensed matrix: ordering, elimination tree,
// column counts, supernodes and supernodal row structure (host, once per
// pattern).  The paper fixes the pivot sequence by an approximate minimum
// degree ordering before the numeric refactorizations (Section V-A); this
// analysis uses the exact (true-degree) minimum degree rule so that the
// result is a function of the graph alone:
//   * pick the uneliminated vertex of smallest degree in the elimination
//     graph, ties to the smallest index; once the minimum degree reaches
//     dense_frac*(remaining-1) or dense_abs, the rest is ordered by index;
//   * elimination tree, postorder with children in ascending order;
//   * fundamental supernodes, then relaxed amalgamation of a supernode into
//     its parent when its columns directly precede the parent's, the merged
//     width is <= max_width and its explicit zeros are <= zero_abs or
//     <= zero_rel of its stored entries.
// The elimination graph is kept as a quotient graph: eliminated vertices
// become elements holding their boundary; a variable's degree is the size of
// the union of its variable neighbours and its elements' boundaries, counted
// when the variable reaches the top of the priority tree (a variable whose
// neighbourhood changed waits there under a lower bound of its degree).
#include "symbolic.h"

#include <algorithm>
#include <climits>
#include <cstring>

namespace opf {

namespace {

// Segment tree over vertices storing packed (degree, index) keys; the root holds the minimum.
struct MinTree {
    int size = 1;
    std::vector<int64_t> t;
    explicit MinTree(int n) {
        while (size < n) size <<= 1;
        t.assign(2 * size, INT64_MAX);
    }
    void set(int i, int64_t key) {
        int p = i + size;
        t[p] = key;
        for (p >>= 1; p >= 1; p >>= 1) t[p] = std::min(t[2 * p], t[2 * p + 1]);
    }
    int64_t min() const { return t[1]; }
};

}  // namespace

std::vector<int32_t> min_degree_order(int n, const std::vector<int32_t>& colptr, const std::vector<int32_t>& rowind,
                                      double dense_frac, int32_t dense_abs) {
    std::vector<std::vector<int32_t>> vadj(n), velem(n), boundary(n);
    for (int j = 0; j < n; j++)
        for (int p = colptr[j]; p < colptr[j + 1]; p++) {
            int i = rowind[p];
            if (i == j) continue;
            vadj[i].push_back(j);
            vadj[j].push_back(i);
        }
    for (auto& a : vadj) {
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    const int64_t W = (int64_t)n + 1;
    MinTree tree(std::max(n, 1));
    std::vector<int32_t> deg(n);
    for (int v = 0; v < n; v++) {
        deg[v] = (int32_t)vadj[v].size();
        tree.set(v, deg[v] * W + v);
    }
    std::vector<char> eliminated(n, 0), absorbed(n, 0), stale(n, 0);
    std::vector<int32_t> inL(n, -1), seen(n, -1);
    std::vector<int32_t> order;
    order.reserve(n);
    int remaining = n;
    int stamp = 0;
    std::vector<int32_t> Lp;
    // Degrees are brought up to date lazily.  A variable next to a new element keeps a lower bound of its
    // degree in the tree (eliminating a neighbour removes one neighbour and adds the rest of the new element's
    // boundary, so the degree is at least max(old degree - 1, boundary size - 1)) and is marked stale; its
    // exact degree is counted when it reaches the top of the tree.  The variable taken is therefore always the
    // one of smallest (exact degree, index), as with every degree recounted after every elimination.
    while (remaining > 0) {
        int64_t key = tree.min();
        int v = (int)(key % W);
        if (stale[v]) {
            ++stamp;
            int cnt = 0;
            seen[v] = stamp;
            auto visit = [&](int w) {
                cnt += seen[w] != stamp;
                seen[w] = stamp;
            };
            for (int w : vadj[v]) visit(w);
            for (int e : velem[v])
                for (int w : boundary[e]) visit(w);
            deg[v] = cnt;
            stale[v] = 0;
            tree.set(v, cnt * W + v);
            if (stamp > INT32_MAX - 4 * n) {
                std::fill(seen.begin(), seen.end(), -1);
                stamp = 0;
            }
            continue;
        }
        int d = (int)(key / W);
        if ((double)d >= dense_frac * (double)(remaining - 1) || d >= dense_abs) {
            for (int u = 0; u < n; u++)
                if (!eliminated[u]) order.push_back(u);
            break;
        }
        // boundary of the new element v
        Lp.clear();
        for (int u : vadj[v])
            if (inL[u] != v) {
                inL[u] = v;
                Lp.push_back(u);
            }
        for (int e : velem[v]) {
            for (int u : boundary[e])
                if (u != v && inL[u] != v) {
                    inL[u] = v;
                    Lp.push_back(u);
                }
            absorbed[e] = 1;
            std::vector<int32_t>().swap(boundary[e]);
        }
        eliminated[v] = 1;
        tree.set(v, INT64_MAX);
        order.push_back(v);
        remaining--;
        std::vector<int32_t>().swap(vadj[v]);
        std::vector<int32_t>().swap(velem[v]);
        // update the neighbours' adjacency: drop v, absorbed elements, and variables now covered by element v
        for (int u : Lp) {
            auto& a = vadj[u];
            size_t k = 0;
            for (int w : a)
                if (w != v && inL[w] != v) a[k++] = w;
            a.resize(k);
            auto& el = velem[u];
            k = 0;
            for (int e : el)
                if (!absorbed[e]) el[k++] = e;
            el.resize(k);
            el.push_back(v);
        }
        boundary[v] = Lp;
        // lower bounds for the boundary variables (exact counts when they reach the top)
        const int nL = (int)Lp.size();
        for (int u : Lp) {
            deg[u] = std::max(deg[u] - 1, nL - 1);
            stale[u] = 1;
            tree.set(u, deg[u] * W + u);
        }
        if (stamp > INT32_MAX - 4 * n) {
            std::fill(seen.begin(), seen.end(), -1);
            stamp = 0;
        }
    }
    return order;
}

// Strictly-lower row lists of P A P^T: rows[i] = {k < i : A(perm(i), perm(k)) != 0}.
static void permuted_rows(int n, const std::vector<int32_t>& colptr, const std::vector<int32_t>& rowind,
                          const std::vector<int32_t>& inv, std::vector<int32_t>& rptr, std::vector<int32_t>& rcol) {
    rptr.assign(n + 1, 0);
    for (int j = 0; j < n; j++)
        for (int p = colptr[j]; p < colptr[j + 1]; p++) {
            int a = inv[rowind[p]], b = inv[j];
            if (a != b) rptr[std::max(a, b) + 1]++;
        }
    for (int i = 0; i < n; i++) rptr[i + 1] += rptr[i];
    rcol.assign(rptr[n], 0);
    std::vector<int32_t> fill(rptr.begin(), rptr.end() - 1);
    for (int j = 0; j < n; j++)
        for (int p = colptr[j]; p < colptr[j + 1]; p++) {
            int a = inv[rowind[p]], b = inv[j];
            if (a != b) rcol[fill[std::max(a, b)]++] = std::min(a, b);
        }
}

// Liu's elimination-tree algorithm with path compression.
static std::vector<int32_t> etree_liu(int n, const std::vector<int32_t>& rptr, const std::vector<int32_t>& rcol) {
    std::vector<int32_t> parent(n, -1), anc(n, -1);
    for (int i = 0; i < n; i++)
        for (int p = rptr[i]; p < rptr[i + 1]; p++) {
            int k = rcol[p];
            while (k != -1 && k != i) {
                int next = anc[k];
                anc[k] = i;
                if (next == -1) {
                    parent[k] = i;
                    break;
                }
                k = next;
            }
        }
    return parent;
}

Symbolic analyze_pattern(int n, const std::vector<int32_t>& colptr, const std::vector<int32_t>& rowind,
                         const chol_options& o) {
    Symbolic S;
    S.n = n;
    std::vector<int32_t> order = min_degree_order(n, colptr, rowind, o.dense_frac, o.dense_abs);
    std::vector<int32_t> inv(n);
    for (int k = 0; k < n; k++) inv[order[k]] = k;
    std::vector<int32_t> rptr, rcol;
    permuted_rows(n, colptr, rowind, inv, rptr, rcol);
    std::vector<int32_t> par0 = etree_liu(n, rptr, rcol);
    // postorder: children ascending, roots ascending (iterative DFS over first-child/next-sibling lists)
    std::vector<int32_t> head(n, -1), next(n, -1), post;
    post.reserve(n);
    for (int j = n - 1; j >= 0; j--)
        if (par0[j] >= 0) {
            next[j] = head[par0[j]];
            head[par0[j]] = j;
        }
    std::vector<int32_t> stack;
    for (int r = 0; r < n; r++) {
        if (par0[r] != -1) continue;
        stack.push_back(r);
        while (!stack.empty()) {
            int v = stack.back();
            int c = head[v];
            if (c == -1) {
                stack.pop_back();
                post.push_back(v);
            } else {
                head[v] = next[c];
                stack.push_back(c);
            }
        }
    }
    std::vector<int32_t> ipost(n);
    for (int k = 0; k < n; k++) ipost[post[k]] = k;
    S.perm.resize(n);
    S.parent.resize(n);
    for (int k = 0; k < n; k++) {
        S.perm[k] = order[post[k]];
        int p = par0[post[k]];
        S.parent[k] = p < 0 ? -1 : ipost[p];
    }
    S.iperm.resize(n);
    for (int k = 0; k < n; k++) S.iperm[S.perm[k]] = k;
    // column counts by row-subtree traversal in the final order
    permuted_rows(n, colptr, rowind, S.iperm, rptr, rcol);
    S.colcount.assign(n, 1);
    {
        std::vector<int32_t> mark(n, -1);
        for (int i = 0; i < n; i++) {
            mark[i] = i;
            for (int p = rptr[i]; p < rptr[i + 1]; p++)
                for (int j = rcol[p]; mark[j] != i; j = S.parent[j]) {
                    mark[j] = i;
                    S.colcount[j]++;
                }
        }
    }
    // fundamental supernodes
    std::vector<int32_t> nkids(n, 0);
    for (int j = 0; j < n; j++)
        if (S.parent[j] >= 0) nkids[S.parent[j]]++;
    struct SN {
        int first, last;
        int64_t rows, zeros;
        bool alive;
    };
    std::vector<SN> sn;
    for (int j = 0; j < n; j++) {
        bool extend = j > 0 && S.parent[j - 1] == j && S.colcount[j - 1] == S.colcount[j] + 1 && nkids[j] == 1;
        if (extend)
            sn.back().last = j;
        else
            sn.push_back({j, j, S.colcount[j], 0, true});
    }
    std::vector<int32_t> col2sn(n);
    for (size_t t = 0; t < sn.size(); t++)
        for (int j = sn[t].first; j <= sn[t].last; j++) col2sn[j] = (int32_t)t;
    auto trap = [](int64_t w, int64_t m) { return w * m - w * (w - 1) / 2; };
    for (size_t c = 0; c < sn.size(); c++) {
        int pc = S.parent[sn[c].last];
        if (pc < 0) continue;
        SN& P = sn[col2sn[pc]];
        SN& C = sn[c];
        if (C.last + 1 != P.first) continue;
        int64_t wc = C.last - C.first + 1, wp = P.last - P.first + 1, w = wc + wp, mrows = wc + P.rows;
        int64_t z = C.zeros + P.zeros + trap(w, mrows) - trap(wc, C.rows) - trap(wp, P.rows);
        if (w > o.max_width) continue;
        if (!(z <= o.zero_abs || (double)z <= o.zero_rel * (double)trap(w, mrows))) continue;
        P.first = C.first;
        P.rows = mrows;
        P.zeros = z;
        C.alive = false;
        for (int j = C.first; j <= C.last; j++) col2sn[j] = col2sn[pc];
    }
    S.snode_ptr.clear();
    for (const SN& s : sn)
        if (s.alive) S.snode_ptr.push_back(s.first);
    S.snode_ptr.push_back(n);
    const int ns = (int)S.snode_ptr.size() - 1;
    S.nsuper = ns;
    S.col2sn.assign(n, 0);
    for (int s = 0; s < ns; s++)
        for (int j = S.snode_ptr[s]; j < S.snode_ptr[s + 1]; j++) S.col2sn[j] = s;
    S.sparent.assign(ns, -1);
    for (int s = 0; s < ns; s++) {
        int pc = S.parent[S.snode_ptr[s + 1] - 1];
        S.sparent[s] = pc < 0 ? -1 : S.col2sn[pc];
    }
    // supernodal row structure: own columns, entries of A below, children's structures below
    std::vector<std::vector<int32_t>> kids(ns);
    for (int s = 0; s < ns; s++)
        if (S.sparent[s] >= 0) kids[S.sparent[s]].push_back(s);
    std::vector<int32_t> lcptr, lcrow;  // strictly-lower column lists of P A P^T
    {
        lcptr.assign(n + 1, 0);
        for (int i = 0; i < n; i++)
            for (int p = rptr[i]; p < rptr[i + 1]; p++) lcptr[rcol[p] + 1]++;
        for (int j = 0; j < n; j++) lcptr[j + 1] += lcptr[j];
        lcrow.assign(lcptr[n], 0);
        std::vector<int32_t> fill(lcptr.begin(), lcptr.end() - 1);
        for (int i = 0; i < n; i++)
            for (int p = rptr[i]; p < rptr[i + 1]; p++) lcrow[fill[rcol[p]]++] = i;
    }
    S.rows_ptr.assign(ns + 1, 0);
    std::vector<std::vector<int32_t>> rows(ns);
    std::vector<int32_t> mark(n, -1);
    for (int s = 0; s < ns; s++) {
        int f = S.snode_ptr[s], l = S.snode_ptr[s + 1] - 1;
        std::vector<int32_t>& R = rows[s];
        for (int j = f; j <= l; j++) {
            R.push_back(j);
            mark[j] = s;
        }
        for (int j = f; j <= l; j++)
            for (int p = lcptr[j]; p < lcptr[j + 1]; p++) {
                int i = lcrow[p];
                if (i > l && mark[i] != s) {
                    mark[i] = s;
                    R.push_back(i);
                }
            }
        for (int c : kids[s])
            for (int i : rows[c])
                if (i > l && mark[i] != s) {
                    mark[i] = s;
                    R.push_back(i);
                }
        std::sort(R.begin() + (l - f + 1), R.end());
        for (int c : kids[s]) std::vector<int32_t>().swap(rows[c]);  // children no longer needed here
        S.rows_ptr[s + 1] = S.rows_ptr[s] + (int64_t)R.size();
        // keep a copy for the flat array (children lists freed above only after use)
        S.rows_flat.insert(S.rows_flat.end(), R.begin(), R.end());
    }
    return S;
}

}  // namespace opf
