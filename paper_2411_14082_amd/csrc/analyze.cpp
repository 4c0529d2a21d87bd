// Pre-processing (Section III-A): static pivoting, fill-reducing ordering and the
// column elimination tree (Section II-B).
//
// The paper's static pivoting is a maximum weighted matching on the values: with the
// values (cktlu_analyze_values) the rows are matched to columns to maximise the product
// of the matched magnitudes, optionally with the matching's row and column scaling; with
// the pattern alone (cktlu_analyze) a structural maximum transversal takes its place.
// Either gives a zero-free diagonal, which MNA matrices with ideal voltage sources need.
// The orderings (approximate minimum degree after Amestoy, Davis and Duff, SIAM J. Matrix
// Anal. Appl. 17(4), 1996, its minimum-fill variant, nested dissection, and nested
// dissection followed by a constrained minimum degree) act on the pattern of B + B' and
// are written from the published methods; the combined ordering keeps the one with the
// least symbolic fill.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <climits>
#include <set>
#include <limits>
#include <queue>
#include <tuple>

#include "internal.h"

namespace cktlu {

int validate_csc(int n, const int32_t *colptr, const int32_t *rowind) {
    if (n < 0 || !colptr) return CKTLU_E_ARG;
    if (colptr[0] != 0) return CKTLU_E_ARG;
    for (int j = 0; j < n; j++) {
        if (colptr[j + 1] < colptr[j]) return CKTLU_E_ARG;
        for (int p = colptr[j]; p < colptr[j + 1]; p++) {
            int r = rowind[p];
            if (r < 0 || r >= n) return CKTLU_E_ARG;
            if (p > colptr[j] && rowind[p - 1] >= r) return CKTLU_E_ARG;  // sorted, unique
        }
    }
    if (n > 0 && colptr[n] > 0 && !rowind) return CKTLU_E_ARG;
    return CKTLU_OK;
}

// Maximum bipartite matching of columns to rows by depth-first augmenting
// paths with a one-step look-ahead; the diagonal is matched first so that a
// matrix with a zero-free diagonal keeps the identity.
bool max_transversal(int n, const std::vector<int> &Ap, const std::vector<int> &Ai,
                     std::vector<int> &match_of_col) {
    std::vector<int> col_of_row(n, -1);
    match_of_col.assign(n, -1);
    for (int j = 0; j < n; j++)
        for (int p = Ap[j]; p < Ap[j + 1]; p++)
            if (Ai[p] == j) { match_of_col[j] = j; col_of_row[j] = j; break; }
    std::vector<int> look(n), iter(n), stack_col(n), via_row(n), seen(n, -1);
    for (int j = 0; j < n; j++) look[j] = Ap[j];
    for (int j0 = 0; j0 < n; j0++) {
        if (match_of_col[j0] >= 0) continue;
        int top = 0;
        stack_col[0] = j0;
        iter[j0] = Ap[j0];
        bool found = false;
        while (top >= 0 && !found) {
            int j = stack_col[top];
            // look-ahead: a free row in column j ends the path
            for (; look[j] < Ap[j + 1]; look[j]++) {
                int r = Ai[look[j]];
                if (col_of_row[r] < 0) {
                    via_row[top] = r;
                    look[j]++;
                    found = true;
                    break;
                }
            }
            if (found) break;
            // descend through a matched row not seen in this search
            bool pushed = false;
            for (; iter[j] < Ap[j + 1]; iter[j]++) {
                int r = Ai[iter[j]];
                if (seen[r] == j0) continue;
                seen[r] = j0;
                via_row[top] = r;
                int jn = col_of_row[r];
                iter[j]++;
                top++;
                stack_col[top] = jn;
                iter[jn] = Ap[jn];
                pushed = true;
                break;
            }
            if (!pushed) top--;
        }
        if (!found) return false;
        for (int t = top; t >= 0; t--) {
            int j = stack_col[t], r = via_row[t];
            match_of_col[j] = r;
            col_of_row[r] = j;
        }
    }
    return true;
}

// ------------------------------------------------------------------ AMD
namespace {

struct DegreeLists {
    std::vector<int> head, next, prev;
    explicit DegreeLists(int n) : head(n + 2, -1), next(n, -1), prev(n, -1) {}
    void insert(int i, int d) {
        next[i] = head[d];
        prev[i] = -1;
        if (head[d] >= 0) prev[head[d]] = i;
        head[d] = i;
    }
    void remove(int i, int d) {
        if (prev[i] >= 0) next[prev[i]] = next[i]; else head[d] = next[i];
        if (next[i] >= 0) prev[next[i]] = prev[i];
        next[i] = prev[i] = -1;
    }
};

enum : uint8_t { VAR = 0, ELEM = 1, ABSORBED = 2, MERGED = 3, DENSE = 4, DONE = 5 };

}  // namespace

// Minimum-priority ordering of a symmetric pattern given by its adjacency lists
// (no self loops); perm[k] is the k-th eliminated node.  amf == false: approximate
// minimum degree (AMD).  amf == true: approximate minimum fill, the priority of a
// variable being the fill its elimination would add if its neighbours already formed
// the largest clique it touches, d(d-1)/2 - c(c-1)/2 with d its approximate external
// degree and c = max over its adjacent elements of |Le \ i|.
//
// Quotient-graph elimination: eliminating variable p turns it into element p
// whose variable list Lp is the union of p's variable neighbours and the lists
// of its adjacent elements (which are absorbed).  Every i in Lp then gets the
// approximate external degree
//   d_i = min(n_left - |i|, d_i + |Lp \ i|, |A_i| + |Lp \ i| + sum_e |Le \ Lp|),
// elements whose list lies inside Lp are absorbed, and variables with equal
// element and variable lists are merged into supervariables.  Rows denser than
// 10*sqrt(n) are ordered last.
void amd_order(int n, const std::vector<int> &Sp, const std::vector<int> &Si,
               std::vector<int> &perm, bool amf, const std::vector<int> *group) {
    perm.clear();
    perm.reserve(n);
    if (n == 0) return;
    // AMF and the constrained form: (group, priority, node) in an ordered set, so that a node
    // of a later group is never eliminated while one of an earlier group is left; the
    // unconstrained AMD path keeps its degree lists
    const bool useset = amf || group;
    auto grp = [&](int i) { return group ? (int64_t)(*group)[i] : (int64_t)0; };
    std::set<std::tuple<int64_t, int64_t, int>> pq;
    std::vector<int64_t> key(useset ? n : 0, 0);
    std::vector<int64_t> cmax(amf ? n : 0, 0);
    auto fillkey = [](int64_t d, int64_t cl) { return d * (d - 1) / 2 - cl * (cl - 1) / 2; };
    std::vector<std::vector<int>> adjV(n), adjE(n), Le(n), members(n);
    std::vector<int> nv(n, 1), deg(n), mark(n, -1), wtag(n, -1);
    std::vector<int64_t> w(n, 0), esize(n, 0);
    std::vector<uint8_t> st(n, VAR);
    // (no dense rows in the constrained form: they would leave their group)
    const int dense_thr = group ? INT_MAX : std::max(16, (int)(10.0 * std::sqrt((double)n)));
    std::vector<int> dense;
    for (int i = 0; i < n; i++) {
        int d = Sp[i + 1] - Sp[i];
        if (d > dense_thr) { st[i] = DENSE; dense.push_back(i); }
    }
    int64_t nlive = 0;
    for (int i = 0; i < n; i++) {
        if (st[i] != VAR) continue;
        nlive++;
        for (int p = Sp[i]; p < Sp[i + 1]; p++)
            if (st[Si[p]] == VAR) adjV[i].push_back(Si[p]);
        deg[i] = (int)adjV[i].size();
    }
    DegreeLists dl(useset ? 0 : n);
    int mindeg = n;
    for (int i = 0; i < n; i++)
        if (st[i] == VAR) {
            if (useset) {
                key[i] = amf ? fillkey(deg[i], 0) : deg[i];
                pq.insert({grp(i), key[i], i});
            } else {
                dl.insert(i, deg[i]);
                mindeg = std::min(mindeg, deg[i]);
            }
        }
    auto q_remove = [&](int i) {
        if (useset) pq.erase({grp(i), key[i], i}); else dl.remove(i, deg[i]);
    };

    int64_t k = 0;
    int tag = 0;
    std::vector<int> Lp;
    std::vector<uint64_t> hash(n, 0);
    std::vector<int> byhash;
    while (k < nlive) {
        int p;
        if (useset) {
            p = std::get<2>(*pq.begin());
            pq.erase(pq.begin());
        } else {
            while (mindeg <= n && dl.head[mindeg] < 0) mindeg++;
            p = dl.head[mindeg];
            dl.remove(p, mindeg);
        }
        // ---- element p: Lp = A_p united with Le of adjacent elements
        ++tag;
        mark[p] = tag;
        Lp.clear();
        for (int e : adjE[p]) {
            if (st[e] != ELEM) continue;
            for (int i : Le[e])
                if (st[i] == VAR && mark[i] != tag) { mark[i] = tag; Lp.push_back(i); }
            st[e] = ABSORBED;
            std::vector<int>().swap(Le[e]);
        }
        for (int i : adjV[p])
            if (st[i] == VAR && mark[i] != tag) { mark[i] = tag; Lp.push_back(i); }
        st[p] = ELEM;
        std::vector<int>().swap(adjV[p]);
        std::vector<int>().swap(adjE[p]);
        perm.push_back(p);
        for (int m : members[p]) perm.push_back(m);
        std::vector<int>().swap(members[p]);
        k += nv[p];
        int64_t degLp = 0;
        for (int i : Lp) { degLp += nv[i]; q_remove(i); }
        esize[p] = degLp;
        // ---- |Le \ Lp| for every element adjacent to Lp
        for (int i : Lp)
            for (int e : adjE[i]) {
                if (st[e] != ELEM || e == p) continue;
                if (wtag[e] != p) { wtag[e] = p; w[e] = esize[e]; }
                w[e] -= nv[i];
            }
        // ---- degree update, list pruning, aggressive absorption
        int64_t left = nlive - k;
        for (int i : Lp) {
            int64_t dsum = 0, cl = degLp - nv[i];
            std::vector<int> &E = adjE[i];
            size_t o = 0;
            for (int e : E) {
                if (st[e] != ELEM || e == p) continue;
                if (w[e] == 0) {                     // Le inside Lp: absorb into p
                    st[e] = ABSORBED;
                    std::vector<int>().swap(Le[e]);
                    continue;
                }
                E[o++] = e;
                dsum += w[e];
                cl = std::max(cl, esize[e] - nv[i]);
            }
            if (amf) cmax[i] = cl;
            E.resize(o);
            E.push_back(p);
            std::vector<int> &V = adjV[i];
            o = 0;
            for (int j : V) {
                if (st[j] != VAR || mark[j] == tag) continue;
                V[o++] = j;
                dsum += nv[j];
            }
            V.resize(o);
            int64_t ext = degLp - nv[i];
            int64_t d = std::min<int64_t>({(int64_t)deg[i] + ext, dsum + ext, left - nv[i]});
            deg[i] = (int)std::max<int64_t>(0, d);
            uint64_t h = (uint64_t)grp(i) * 0x94D049BB133111EBull;   // supervariables stay inside a group
            for (int e : E) h += (uint64_t)e * 0x9E3779B97F4A7C15ull;
            for (int j : V) h += (uint64_t)(j + 1) * 0xC2B2AE3D27D4EB4Full;
            hash[i] = h ^ ((uint64_t)E.size() << 48) ^ ((uint64_t)V.size() << 32);
        }
        // ---- supervariable detection among Lp
        byhash.assign(Lp.begin(), Lp.end());
        std::sort(byhash.begin(), byhash.end(), [&](int a, int b) {
            return hash[a] != hash[b] ? hash[a] < hash[b] : a < b;
        });
        for (size_t a = 0; a < byhash.size();) {
            size_t b = a + 1;
            while (b < byhash.size() && hash[byhash[b]] == hash[byhash[a]]) b++;
            if (b - a > 1) {
                for (size_t x = a; x < b; x++) {
                    int i = byhash[x];
                    std::sort(adjE[i].begin(), adjE[i].end());
                    std::sort(adjV[i].begin(), adjV[i].end());
                }
                for (size_t x = a; x < b; x++) {
                    int i = byhash[x];
                    if (st[i] != VAR) continue;
                    for (size_t y = x + 1; y < b; y++) {
                        int j = byhash[y];
                        if (st[j] != VAR) continue;
                        if (grp(i) == grp(j) && adjE[i] == adjE[j] && adjV[i] == adjV[j]) {
                            deg[i] = std::max(0, deg[i] - nv[j]);
                            nv[i] += nv[j];
                            nv[j] = 0;
                            st[j] = MERGED;
                            members[i].push_back(j);
                            members[i].insert(members[i].end(), members[j].begin(), members[j].end());
                            std::vector<int>().swap(members[j]);
                            std::vector<int>().swap(adjE[j]);
                            std::vector<int>().swap(adjV[j]);
                        }
                    }
                }
            }
            a = b;
        }
        // ---- element list and reinsertion
        std::vector<int> &L = Le[p];
        for (int i : Lp) {
            if (st[i] != VAR) continue;
            L.push_back(i);
            int d = std::min(deg[i], n);
            deg[i] = d;
            if (useset) {
                key[i] = amf ? fillkey(d, std::min<int64_t>(cmax[i], d)) : d;
                pq.insert({grp(i), key[i], i});
            } else {
                dl.insert(i, d);
                if (d < mindeg) mindeg = d;
            }
        }
    }
    for (int i : dense) perm.push_back(i);
}

// Nested dissection of a symmetric pattern: a node set is split by the smallest
// breadth-first level set near the middle of a level structure rooted at a
// pseudo-peripheral node (two sweeps); both halves are ordered first, then the
// separator.  Disconnected sets split into components; sets of at most `leaf` nodes
// (or with fewer than three levels) are ordered by AMD on their induced subgraph.
void nd_order(int n, const std::vector<int> &Sp, const std::vector<int> &Si, std::vector<int> &perm,
              int leaf, std::vector<int> *groups) {
    perm.clear();
    perm.reserve(n);
    if (groups) groups->assign(n, 0);
    int ngroups = 0;
    if (n == 0) return;
    std::vector<int> inset(n, -1), lev(n, -1), local(n, -1);
    int stamp = 0;
    struct Task { std::vector<int> nodes; bool emit; };
    std::vector<Task> stack;
    std::vector<int> all(n);
    std::iota(all.begin(), all.end(), 0);
    stack.push_back({std::move(all), false});
    std::vector<int> order, lptr;                       // BFS order and level pointers
    auto bfs = [&](int root, int tag) {
        order.clear();
        lptr.assign(1, 0);
        order.push_back(root);
        lev[root] = tag;
        size_t h = 0;
        while (h < order.size()) {
            const size_t e = order.size();
            for (; h < e; h++) {
                const int u = order[h];
                for (int q = Sp[u]; q < Sp[u + 1]; q++) {
                    const int v = Si[q];
                    if (inset[v] == stamp && lev[v] != tag) { lev[v] = tag; order.push_back(v); }
                }
            }
            lptr.push_back((int)e);
        }
        lptr.pop_back();
        lptr.push_back((int)order.size());
    };
    std::vector<int> lSp, lSi, lperm;
    int tag = 0;
    while (!stack.empty()) {
        Task t = std::move(stack.back());
        stack.pop_back();
        if (t.emit) {
            perm.insert(perm.end(), t.nodes.begin(), t.nodes.end());
            if (groups) { for (int v : t.nodes) (*groups)[v] = ngroups; ngroups++; }
            continue;
        }
        std::vector<int> &nodes = t.nodes;
        ++stamp;
        for (int v : nodes) inset[v] = stamp;
        bool split = (int)nodes.size() > leaf;
        if (split) {
            bfs(nodes[0], ++tag);
            if (order.size() < nodes.size()) {            // disconnected: this component, the rest
                std::vector<int> rest;
                for (int v : nodes) if (lev[v] != tag) rest.push_back(v);
                std::vector<int> comp(order.begin(), order.end());
                stack.push_back({std::move(rest), false});
                stack.push_back({std::move(comp), false});
                continue;
            }
            bfs(order.back(), ++tag);                     // from the farthest node
            const int L = (int)lptr.size() - 1;
            if (L < 3) split = false;
            else {
                const int mid = L / 2;
                int m = std::max(1, mid - 3);
                for (int i = m; i <= std::min(L - 2, mid + 3); i++)
                    if (lptr[i + 1] - lptr[i] < lptr[m + 1] - lptr[m]) m = i;
                std::vector<int> A(order.begin(), order.begin() + lptr[m]);
                std::vector<int> sep(order.begin() + lptr[m], order.begin() + lptr[m + 1]);
                std::vector<int> B(order.begin() + lptr[m + 1], order.end());
                stack.push_back({std::move(sep), true});
                stack.push_back({std::move(B), false});
                stack.push_back({std::move(A), false});
                continue;
            }
        }
        if (groups) {                                     // incomplete dissection: the leaf is a group
            perm.insert(perm.end(), nodes.begin(), nodes.end());
            for (int v : nodes) (*groups)[v] = ngroups;
            ngroups++;
            continue;
        }
        // leaf: AMD on the induced subgraph
        const int nl = (int)nodes.size();
        for (int i = 0; i < nl; i++) local[nodes[i]] = i;
        lSp.assign(nl + 1, 0);
        lSi.clear();
        for (int i = 0; i < nl; i++) {
            const int u = nodes[i];
            for (int q = Sp[u]; q < Sp[u + 1]; q++)
                if (inset[Si[q]] == stamp) lSi.push_back(local[Si[q]]);
            lSp[i + 1] = (int)lSi.size();
        }
        amd_order(nl, lSp, lSi, lperm, false);
        for (int i = 0; i < nl; i++) perm.push_back(nodes[lperm[i]]);
    }
}

// Nested dissection followed by a constrained minimum degree (Section III-A): the
// dissection stops at its leaves and numbers its parts (the leaves and separators) in the
// order it would emit them; one AMD over the whole pattern then eliminates the parts in
// that order, each by approximate degree, so that the ordering inside a part sees the fill
// it causes in the separators that border it.
void nd_camd_order(int n, const std::vector<int> &Sp, const std::vector<int> &Si, std::vector<int> &perm,
                   int leaf) {
    std::vector<int> groups, nd;
    nd_order(n, Sp, Si, nd, leaf, &groups);
    amd_order(n, Sp, Si, perm, false, &groups);
}

int64_t symbolic_cholesky_nnz(int n, const std::vector<int> &Sp, const std::vector<int> &Si,
                              const std::vector<int> &perm) {
    std::vector<int> inv(n), parent(n, -1), ancestor(n, -1), mark(n, -1);
    for (int k = 0; k < n; k++) inv[perm[k]] = k;
    // elimination tree, ancestors path-compressed
    for (int k = 0; k < n; k++) {
        const int v = perm[k];
        for (int p = Sp[v]; p < Sp[v + 1]; p++) {
            int i = inv[Si[p]];
            while (i != -1 && i < k) {
                const int nxt = ancestor[i];
                ancestor[i] = k;
                if (nxt == -1) { parent[i] = k; break; }
                i = nxt;
            }
        }
    }
    // row k of L: the union of the tree paths from its neighbours below k up to k
    int64_t nnz = n;
    for (int k = 0; k < n; k++) {
        mark[k] = k;
        const int v = perm[k];
        for (int p = Sp[v]; p < Sp[v + 1]; p++) {
            int i = inv[Si[p]];
            if (i > k) continue;
            while (mark[i] != k) { mark[i] = k; nnz++; i = parent[i]; }
        }
    }
    return nnz;
}

// Column elimination tree of H (the elimination tree of H'H) without forming
// H'H: for every row, the columns that share it are linked through the root
// of the most recent such column, with path compression.
void column_etree(int n, const std::vector<int> &Hp, const std::vector<int> &Hi,
                  std::vector<int> &parent) {
    parent.assign(n, -1);
    std::vector<int> ancestor(n, -1), last(n, -1);
    for (int j = 0; j < n; j++) {
        for (int p = Hp[j]; p < Hp[j + 1]; p++) {
            int k = last[Hi[p]];
            while (k != -1 && k < j) {
                int nxt = ancestor[k];
                ancestor[k] = j;
                if (nxt == -1) { parent[k] = j; break; }
                k = nxt;
            }
            last[Hi[p]] = j;
        }
    }
}

// Static pivoting (Section III-A): the row matched to each column that maximises the
// product of the matched magnitudes, and the scaling that makes every matched entry 1 in
// magnitude and every other entry at most 1.  With column maxima a_j = max_i |A(i,j)| and
// costs c_ij = ln a_j - ln |A(i,j)| >= 0 (entries with A(i,j) = 0 are left out), the
// matching is a minimum-cost perfect matching, found by successive shortest augmenting
// paths: each unmatched column starts a Dijkstra search over reduced costs c_ij + pc_j -
// pr_i >= 0 (column j to row i; a matched row leads on to its column at reduced cost 0),
// stops at the nearest unmatched row, augments, and raises every potential by the
// distance found (capped at the path length), which keeps all reduced costs non-negative
// and the matched ones zero.  Columns whose maximum sits on a free row are matched first.
// At the end u_i = pr_i, v_j = -pc_j satisfy c_ij >= u_i + v_j with equality on the
// matching, so ln of the row scale is u_i and of the column scale v_j - ln a_j.
// Returns false when the nonzero entries admit no perfect matching.
bool max_product_matching(int n, const std::vector<int> &Ap, const std::vector<int> &Ai, const double *Ax,
                          std::vector<int> &match_of_col, std::vector<double> &lnr, std::vector<double> &lnc) {
    const double INF = std::numeric_limits<double>::infinity();
    std::vector<double> cost(Ap[n]), lnmax(n, -INF);
    for (int j = 0; j < n; j++) {
        for (int p = Ap[j]; p < Ap[j + 1]; p++)
            if (Ax[p] != 0.0 && std::isfinite(Ax[p])) lnmax[j] = std::max(lnmax[j], std::log(std::fabs(Ax[p])));
        if (lnmax[j] == -INF) return false;                  // a column without a usable entry
        for (int p = Ap[j]; p < Ap[j + 1]; p++)
            cost[p] = (Ax[p] != 0.0 && std::isfinite(Ax[p])) ? lnmax[j] - std::log(std::fabs(Ax[p])) : INF;
    }
    std::vector<int> col_of_row(n, -1);
    match_of_col.assign(n, -1);
    std::vector<double> pr(n, 0.0), pc(n, 0.0);
    // greedy start: a column's maximum (reduced cost 0) on a free row
    for (int j = 0; j < n; j++)
        for (int p = Ap[j]; p < Ap[j + 1]; p++)
            if (cost[p] == 0.0 && col_of_row[Ai[p]] < 0) {
                col_of_row[Ai[p]] = j;
                match_of_col[j] = Ai[p];
                break;
            }
    std::vector<double> dr(n, INF);                     // distance of each row in the current search
    std::vector<int> via(n, -1), seen(n, -1), touched;
    std::vector<int> done_cols;
    typedef std::pair<double, int> QE;
    for (int j0 = 0; j0 < n; j0++) {
        if (match_of_col[j0] >= 0) continue;
        std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
        touched.clear();
        done_cols.clear();
        // relax the rows of column j at distance dj
        auto relax = [&](int j, double dj) {
            for (int p = Ap[j]; p < Ap[j + 1]; p++) {
                if (cost[p] == INF) continue;
                const int i = Ai[p];
                if (seen[i] == j0) continue;                 // finalised
                // reduced costs are >= 0 up to rounding (the potentials keep them so)
                const double d = dj + std::max(0.0, cost[p] + pc[j] - pr[i]);
                if (d < dr[i]) {
                    if (dr[i] == INF) touched.push_back(i);
                    dr[i] = d;
                    via[i] = j;
                    pq.push({d, i});
                }
            }
        };
        std::vector<std::pair<int, double>> fin;             // finalised rows and their distances
        std::vector<double> dcol;                            // distances of the columns reached
        done_cols.push_back(j0);
        dcol.push_back(0.0);
        relax(j0, 0.0);
        int ifree = -1;
        double delta = INF;
        while (!pq.empty()) {
            const QE t = pq.top();
            pq.pop();
            const int i = t.second;
            if (seen[i] == j0 || t.first > dr[i]) continue;
            seen[i] = j0;
            fin.push_back({i, t.first});
            if (col_of_row[i] < 0) { ifree = i; delta = t.first; break; }
            const int jn = col_of_row[i];
            done_cols.push_back(jn);
            dcol.push_back(t.first);
            relax(jn, t.first);
        }
        if (ifree < 0) return false;                         // no augmenting path: no perfect matching
        // potentials pi += min(d, delta) (Johnson's rule, truncated at the path length), shifted
        // by -delta: nodes reached at d < delta move by d - delta, the others stay
        for (auto &f : fin) if (f.second < delta) pr[f.first] -= delta - f.second;
        for (size_t q = 0; q < done_cols.size(); q++) if (dcol[q] < delta) pc[done_cols[q]] -= delta - dcol[q];
        // augment along via[]
        int i = ifree;
        while (true) {
            const int j = via[i];
            const int iprev = match_of_col[j];
            match_of_col[j] = i;
            col_of_row[i] = j;
            if (j == j0) break;
            i = iprev;
        }
        for (int r : touched) dr[r] = INF;
    }
    lnr.resize(n);
    lnc.resize(n);
    for (int i = 0; i < n; i++) lnr[i] = pr[i];
    for (int j = 0; j < n; j++) lnc[j] = -pc[j] - lnmax[j];
    return true;
}

int run_analysis(Analysis &an, int n, const int32_t *colptr, const int32_t *rowind,
                 int ordering, int transversal, const double *values, int static_pivoting) {
    int rc = validate_csc(n, colptr, rowind);
    if (rc != CKTLU_OK) return rc;
    an = Analysis();
    an.n = n;
    an.nnz = colptr[n];
    an.Ap.assign(colptr, colptr + n + 1);
    an.Ai.assign(rowind, rowind + an.nnz);
    // transversal: B(i, j) = A(match[i], j) has a zero-free diagonal; with values and static
    // pivoting, the one that maximises the product of the diagonal magnitudes (and the scaling)
    std::vector<int> match(n);
    an.rscale.clear();
    an.cscale.clear();
    bool matched = false;
    if (values && static_pivoting > 0) {
        std::vector<double> lnr, lnc;
        matched = max_product_matching(n, an.Ap, an.Ai, values, match, lnr, lnc);
        an.static_pivoting_used = matched ? static_pivoting : 0;
        if (matched && static_pivoting == 2) {
            an.rscale.resize(n);
            an.cscale.resize(n);
            for (int i = 0; i < n; i++) an.rscale[i] = std::exp(lnr[i]);
            for (int j = 0; j < n; j++) an.cscale[j] = std::exp(lnc[j]);
        }
    }
    if (!matched) {
        if (transversal) {
            if (!max_transversal(n, an.Ap, an.Ai, match)) return CKTLU_E_STRUCT_SINGULAR;
        } else {
            std::iota(match.begin(), match.end(), 0);
        }
    }
    std::vector<int> browof(n);            // A row -> B row
    for (int i = 0; i < n; i++) browof[match[i]] = i;
    // ordering of B + B'
    std::vector<int> q(n);
    an.ordering_used = CKTLU_ORDER_NATURAL;
    if (ordering != CKTLU_ORDER_NATURAL) {
        std::vector<int> cnt(n + 1, 0);
        for (int j = 0; j < n; j++)
            for (int p = an.Ap[j]; p < an.Ap[j + 1]; p++) {
                int i = browof[an.Ai[p]];
                if (i != j) { cnt[i + 1]++; cnt[j + 1]++; }
            }
        for (int i = 0; i < n; i++) cnt[i + 1] += cnt[i];
        std::vector<int> Si(cnt[n]), fill(cnt.begin(), cnt.end() - 1);
        for (int j = 0; j < n; j++)
            for (int p = an.Ap[j]; p < an.Ap[j + 1]; p++) {
                int i = browof[an.Ai[p]];
                if (i != j) { Si[fill[i]++] = j; Si[fill[j]++] = i; }
            }
        // sort + dedupe each adjacency list
        std::vector<int> Sp(n + 1, 0), Sd;
        Sd.reserve(Si.size());
        for (int i = 0; i < n; i++) {
            std::sort(Si.begin() + cnt[i], Si.begin() + cnt[i + 1]);
            int prevv = -1;
            for (int p = cnt[i]; p < cnt[i + 1]; p++)
                if (Si[p] != prevv) { Sd.push_back(Si[p]); prevv = Si[p]; }
            Sp[i + 1] = (int)Sd.size();
        }
        // the combined ordering (Section III-A): each method, keep the one with less fill
        const bool autom = ordering == CKTLU_ORDER_AUTO;
        std::vector<int> qm;
        int64_t best = -1;
        const int methods[4] = {CKTLU_ORDER_AMD, CKTLU_ORDER_AMF, CKTLU_ORDER_ND, CKTLU_ORDER_ND_CAMD};
        for (int m : methods) {
            if (!autom && ordering != m) continue;
            if (m == CKTLU_ORDER_ND) nd_order(n, Sp, Sd, qm, kNdLeaf);
            else if (m == CKTLU_ORDER_ND_CAMD) nd_camd_order(n, Sp, Sd, qm, kNdLeaf);
            else amd_order(n, Sp, Sd, qm, m == CKTLU_ORDER_AMF);
            if ((int)qm.size() != n) return CKTLU_E_ARG;
            if (!autom) { q.swap(qm); an.ordering_used = m; break; }
            const int64_t f = symbolic_cholesky_nnz(n, Sp, Sd, qm);
            (m == CKTLU_ORDER_AMD ? an.fill_amd : m == CKTLU_ORDER_AMF ? an.fill_amf
                                              : m == CKTLU_ORDER_ND ? an.fill_nd : an.fill_ndc) = f;
            if (best < 0 || f < best) { best = f; q.swap(qm); an.ordering_used = m; }   // ties keep the earlier
        }
    } else {
        std::iota(q.begin(), q.end(), 0);
    }
    an.rowperm_pre.resize(n);
    an.colperm.resize(n);
    an.rowinv_pre.resize(n);
    an.colinv.resize(n);
    for (int i = 0; i < n; i++) {
        an.rowperm_pre[i] = match[q[i]];
        an.colperm[i] = q[i];
    }
    for (int i = 0; i < n; i++) {
        an.rowinv_pre[an.rowperm_pre[i]] = i;
        an.colinv[an.colperm[i]] = i;
    }
    // A_hat pattern, rows sorted, with the source nonzero of each entry
    an.Hp.assign(n + 1, 0);
    an.Hi.resize(an.nnz);
    an.Hsrc.resize(an.nnz);
    std::vector<std::pair<int, int>> tmp;
    for (int j = 0; j < n; j++) {
        int c = an.colperm[j];
        tmp.clear();
        for (int p = an.Ap[c]; p < an.Ap[c + 1]; p++) tmp.emplace_back(an.rowinv_pre[an.Ai[p]], p);
        std::sort(tmp.begin(), tmp.end());
        an.Hp[j + 1] = an.Hp[j] + (int)tmp.size();
        for (size_t t = 0; t < tmp.size(); t++) {
            an.Hi[an.Hp[j] + t] = tmp[t].first;
            an.Hsrc[an.Hp[j] + t] = tmp[t].second;
        }
    }
    column_etree(n, an.Hp, an.Hi, an.parent);
    std::vector<int> depth(n, 0);
    int h = 0;
    for (int j = n - 1; j >= 0; j--) {
        depth[j] = an.parent[j] < 0 ? 1 : depth[an.parent[j]] + 1;
        h = std::max(h, depth[j]);
    }
    an.etree_height = h;
    return CKTLU_OK;
}

}  // namespace cktlu
