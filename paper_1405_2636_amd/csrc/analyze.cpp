// Host symbolic analysis of the supernodal solver (Section III of the paper):
// nested-dissection ordering, elimination tree, column counts, fundamental
// supernodes, amalgamation under a fill budget, final postorder, vertical
// splitting of wide supernodes, block layout, update pairs and dependency
// counts, plus the maps the device path needs (assembly destinations and the
// symmetric residual pattern).  Integer work only.
//
// Algorithms (chosen for speed on million-unknown grids):
//   * nested dissection on compacted induced subgraphs with an explicit task
//     stack, writing every separator at the end of its range;
//   * elimination tree by Liu's ancestor algorithm with path compression;
//   * column counts by row-subtree traversal of the postordered tree;
//   * supernode row sets by walking row subtrees over the supernodal tree
//     (each row lands in ascending order, so no sorting is needed).
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>
#include <stdexcept>
#include <utility>

namespace spx {

namespace {

// Symmetrized adjacency of A + A^T without the diagonal, sorted rows.
void build_graph(int32_t n, const int64_t* colptr, const int32_t* rowind,
                 std::vector<int64_t>& xadj, std::vector<int32_t>& adj)
{
    std::vector<int64_t> cnt(static_cast<size_t>(n) + 1, 0);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            int32_t i = rowind[p];
            if (i != j) { ++cnt[i + 1]; ++cnt[j + 1]; }
        }
    for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    std::vector<int32_t> tmp(static_cast<size_t>(cnt[n]));
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            int32_t i = rowind[p];
            if (i != j) { tmp[pos[i]++] = j; tmp[pos[j]++] = i; }
        }
    xadj.assign(static_cast<size_t>(n) + 1, 0);
    adj.clear();
    adj.reserve(tmp.size());
    for (int32_t v = 0; v < n; ++v) {
        auto b = tmp.begin() + cnt[v], e = tmp.begin() + cnt[v + 1];
        std::sort(b, e);
        auto last = std::unique(b, e);
        adj.insert(adj.end(), b, last);
        xadj[v + 1] = static_cast<int64_t>(adj.size());
    }
}

// ---------------------------------------------------------------- ordering
// Compact induced subgraph: vertices sorted by global id, local CSR.
struct SubGraph {
    std::vector<int32_t> gid;     // local -> global, ascending
    std::vector<int64_t> ptr;
    std::vector<int32_t> nb;      // local neighbour indices
};

class Dissector {
public:
    Dissector(int32_t n, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj, int32_t leaf)
        : n_(n), xadj_(xadj), adj_(adj), leaf_(std::max(leaf, 1)), loc_(static_cast<size_t>(n), -1) {}

    std::vector<int32_t> run()
    {
        std::vector<int32_t> order(static_cast<size_t>(n_));
        struct Task { std::vector<int32_t> verts; int32_t start; };
        std::vector<Task> stack;
        std::vector<int32_t> all(static_cast<size_t>(n_));
        std::iota(all.begin(), all.end(), 0);
        stack.push_back({std::move(all), 0});
        while (!stack.empty()) {
            Task t = std::move(stack.back());
            stack.pop_back();
            // the set is split into connected components, laid out by ascending min id
            SubGraph g = induce(t.verts);
            std::vector<int32_t> comp_of;
            std::vector<std::vector<int32_t>> comps = components(g, std::vector<char>(), comp_of);
            int32_t at = t.start;
            for (auto& c : comps) {   // c: local ids, ascending
                const int32_t sz = static_cast<int32_t>(c.size());
                if (sz <= leaf_) {
                    for (int32_t q = 0; q < sz; ++q) order[at + q] = g.gid[c[q]];
                } else {
                    std::vector<int32_t> sep, rest;
                    split_component(g, c, sep, rest);
                    const int32_t ns = static_cast<int32_t>(sep.size());
                    for (int32_t q = 0; q < ns; ++q) order[at + sz - ns + q] = sep[q];
                    stack.push_back({std::move(rest), at});
                }
                at += sz;
            }
        }
        return order;
    }

private:
    int32_t n_;
    const std::vector<int64_t>& xadj_;
    const std::vector<int32_t>& adj_;
    int32_t leaf_;
    std::vector<int32_t> loc_;

    SubGraph induce(std::vector<int32_t>& verts)
    {
        SubGraph g;
        std::sort(verts.begin(), verts.end());
        g.gid = verts;
        const int32_t m = static_cast<int32_t>(verts.size());
        for (int32_t q = 0; q < m; ++q) loc_[verts[q]] = q;
        g.ptr.assign(static_cast<size_t>(m) + 1, 0);
        for (int32_t q = 0; q < m; ++q) {
            int32_t v = verts[q];
            for (int64_t p = xadj_[v]; p < xadj_[v + 1]; ++p)
                if (loc_[adj_[p]] >= 0) g.nb.push_back(loc_[adj_[p]]);
            g.ptr[q + 1] = static_cast<int64_t>(g.nb.size());
        }
        for (int32_t q = 0; q < m; ++q) loc_[verts[q]] = -1;
        return g;
    }

    // connected components of g minus the vertices flagged in `removed`
    std::vector<std::vector<int32_t>> components(const SubGraph& g, const std::vector<char>& removed,
                                                 std::vector<int32_t>& comp_of)
    {
        const int32_t m = static_cast<int32_t>(g.gid.size());
        comp_of.assign(static_cast<size_t>(m), -1);
        std::vector<std::vector<int32_t>> out;
        std::vector<int32_t> q;
        for (int32_t s = 0; s < m; ++s) {
            if (comp_of[s] >= 0 || (!removed.empty() && removed[s])) continue;
            const int32_t id = static_cast<int32_t>(out.size());
            q.assign(1, s);
            comp_of[s] = id;
            for (size_t h = 0; h < q.size(); ++h) {
                int32_t v = q[h];
                for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; ++p) {
                    int32_t u = g.nb[p];
                    if (comp_of[u] < 0 && (removed.empty() || !removed[u])) { comp_of[u] = id; q.push_back(u); }
                }
            }
            std::sort(q.begin(), q.end());
            out.push_back(q);
        }
        return out;
    }

    // BFS distances inside component `inc` (flag per local vertex); returns eccentricity
    int32_t levels(const SubGraph& g, const std::vector<int32_t>& comp_of, int32_t cid, int32_t root,
                   std::vector<int32_t>& dist)
    {
        std::vector<int32_t> q;
        q.reserve(1024);
        q.push_back(root);
        dist[root] = 0;
        int32_t ecc = 0;
        std::vector<int32_t> touched{root};
        for (size_t h = 0; h < q.size(); ++h) {
            int32_t v = q[h];
            for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; ++p) {
                int32_t u = g.nb[p];
                if (comp_of[u] == cid && dist[u] < 0) {
                    dist[u] = dist[v] + 1;
                    ecc = std::max(ecc, dist[u]);
                    q.push_back(u);
                }
            }
        }
        return ecc;
    }

    void split_component(const SubGraph& g, const std::vector<int32_t>& c, std::vector<int32_t>& sep,
                         std::vector<int32_t>& rest)
    {
        const int32_t m = static_cast<int32_t>(g.gid.size());
        // component membership of this call
        std::vector<int32_t> member(static_cast<size_t>(m), -1);
        for (int32_t v : c) member[v] = 0;
        auto inner_degree = [&](int32_t v) {
            int32_t d = 0;
            for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; ++p) d += member[g.nb[p]] == 0;
            return d;
        };
        std::vector<int32_t> dist(static_cast<size_t>(m), -1);
        auto reset = [&]() { for (int32_t v : c) dist[v] = -1; };
        int32_t root = c.front();  // smallest global id (local ids ascend with global ids)
        int32_t ecc = levels(g, member, 0, root, dist);
        while (true) {
            int32_t best = -1, bdeg = 0;
            for (int32_t v : c)
                if (dist[v] == ecc) {
                    int32_t d = inner_degree(v);
                    if (best < 0 || d < bdeg || (d == bdeg && v < best)) { best = v; bdeg = d; }
                }
            reset();
            int32_t e2 = levels(g, member, 0, best, dist);
            if (e2 > ecc) { root = best; ecc = e2; continue; }
            reset();
            levels(g, member, 0, root, dist);
            break;
        }
        std::vector<int64_t> width(static_cast<size_t>(ecc) + 1, 0);
        for (int32_t v : c) ++width[dist[v]];
        const int64_t half = (static_cast<int64_t>(c.size()) + 1) / 2;
        int32_t lev = 0;
        int64_t acc = 0;
        for (; lev <= ecc; ++lev) { acc += width[lev]; if (acc >= half) break; }
        if (lev == ecc) lev = ecc - 1;
        for (int32_t v : c) {
            bool s = false;
            if (dist[v] == lev)
                for (int64_t p = g.ptr[v]; p < g.ptr[v + 1] && !s; ++p) {
                    int32_t u = g.nb[p];
                    s = member[u] == 0 && dist[u] == lev + 1;
                }
            if (s) sep.push_back(g.gid[v]); else rest.push_back(g.gid[v]);
        }
        // c ascends in local id == global id order, so sep is ascending already
    }
};

// Elimination tree of P A P^T, perm new -> old (Liu, with path compression).
std::vector<int32_t> etree_liu(int32_t n, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                               const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm)
{
    std::vector<int32_t> parent(static_cast<size_t>(n), -1), anc(static_cast<size_t>(n), -1);
    for (int32_t i = 0; i < n; ++i) {
        int32_t oi = perm[i];
        for (int64_t p = xadj[oi]; p < xadj[oi + 1]; ++p) {
            int32_t k = iperm[adj[p]];
            if (k >= i) continue;
            // climb from k to the root of its current subtree, compressing toward i
            while (k != -1 && k != i) {
                int32_t next = anc[k];
                anc[k] = i;
                if (next == -1) { parent[k] = i; break; }
                k = next;
            }
        }
    }
    return parent;
}

// children ascending, roots ascending, node after its children
std::vector<int32_t> postorder_forest(const std::vector<int32_t>& parent)
{
    const int32_t n = static_cast<int32_t>(parent.size());
    std::vector<int32_t> first(static_cast<size_t>(n), -1), sib(static_cast<size_t>(n), -1);
    for (int32_t v = n - 1; v >= 0; --v)
        if (parent[v] >= 0) { sib[v] = first[parent[v]]; first[parent[v]] = v; }
    std::vector<int32_t> post;
    post.reserve(static_cast<size_t>(n));
    std::vector<std::pair<int32_t, int32_t>> st;
    for (int32_t r = 0; r < n; ++r) {
        if (parent[r] >= 0) continue;
        st.emplace_back(r, first[r]);
        while (!st.empty()) {
            auto& top = st.back();
            if (top.second >= 0) {
                int32_t ch = top.second;
                top.second = sib[ch];
                st.emplace_back(ch, first[ch]);
            } else {
                post.push_back(top.first);
                st.pop_back();
            }
        }
    }
    if (static_cast<int32_t>(post.size()) != n) throw std::runtime_error("elimination tree is not a forest");
    return post;
}

}  // namespace

void analyze_pattern(int32_t n, const int64_t* colptr, const int32_t* rowind, const Options& opt, Plan& P)
{
    if (n < 0) throw InvalidArgument("n must be >= 0");
    if (opt.split_width < 1 || opt.split_width > kMaxWidth)
        throw InvalidArgument("split_width must be in [1, 256]");
    if (opt.amalg_pct < 0) throw InvalidArgument("amalg_pct must be >= 0");
    if (colptr[0] != 0) throw InvalidArgument("colptr[0] must be 0");
    for (int32_t j = 0; j < n; ++j) {
        if (colptr[j + 1] < colptr[j]) throw InvalidArgument("colptr is decreasing");
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            if (rowind[p] < 0 || rowind[p] >= n) throw InvalidArgument("row index out of range");
            if (p > colptr[j] && rowind[p] <= rowind[p - 1]) throw InvalidArgument("rows unsorted or duplicated");
        }
    }
    P = Plan();
    P.n = n;
    P.nnz_a = colptr[n];
    std::vector<int64_t> xadj;
    std::vector<int32_t> adj;
    build_graph(n, colptr, rowind, xadj, adj);

    // ---- ordering
    std::vector<int32_t> ord;
    if (opt.user_perm) {
        ord.assign(opt.user_perm, opt.user_perm + n);
        std::vector<char> hit(static_cast<size_t>(n), 0);
        for (int32_t v : ord) {
            if (v < 0 || v >= n || hit[v]) throw InvalidArgument("user_perm is not a permutation");
            hit[v] = 1;
        }
    } else {
        ord = Dissector(n, xadj, adj, opt.leaf_size).run();
    }
    std::vector<int32_t> iord(static_cast<size_t>(n));
    for (int32_t k = 0; k < n; ++k) iord[ord[k]] = k;

    // ---- elimination tree + postorder: relabel so that labels are a postorder
    std::vector<int32_t> par0 = etree_liu(n, xadj, adj, ord, iord);
    std::vector<int32_t> post = postorder_forest(par0);
    std::vector<int32_t> rank(static_cast<size_t>(n));
    for (int32_t k = 0; k < n; ++k) rank[post[k]] = k;
    std::vector<int32_t> pa(static_cast<size_t>(n)), q(static_cast<size_t>(n)), iq(static_cast<size_t>(n));
    for (int32_t k = 0; k < n; ++k) {
        int32_t old = post[k];
        q[k] = ord[old];
        pa[k] = par0[old] < 0 ? -1 : rank[par0[old]];
    }
    for (int32_t k = 0; k < n; ++k) iq[q[k]] = k;

    // ---- column counts by row subtrees (postordered labels)
    std::vector<int64_t> colcount(static_cast<size_t>(n), 1);
    {
        std::vector<int32_t> visited(static_cast<size_t>(n), -1);
        for (int32_t i = 0; i < n; ++i) {
            visited[i] = i;
            int32_t oi = q[i];
            for (int64_t p = xadj[oi]; p < xadj[oi + 1]; ++p) {
                int32_t k = iq[adj[p]];
                if (k >= i) continue;
                for (; visited[k] != i; k = pa[k]) { visited[k] = i; ++colcount[k]; }
            }
        }
    }
    int64_t nnz_exact = 0;
    double flops_alg = 0.0, flops_alg_lu = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        nnz_exact += colcount[j];
        const double e = static_cast<double>(colcount[j]);
        flops_alg += e * e;
        flops_alg_lu += 2.0 * (e - 1.0) * (e - 1.0) + (e - 1.0);
    }

    // ---- fundamental supernodes
    std::vector<int32_t> nkids(static_cast<size_t>(n), 0);
    for (int32_t j = 0; j < n; ++j) if (pa[j] >= 0) ++nkids[pa[j]];
    std::vector<int32_t> sstart;  // first column of each fundamental supernode
    std::vector<int32_t> sof(static_cast<size_t>(n));
    for (int32_t j = 0; j < n; ++j) {
        bool extend = j > 0 && pa[j - 1] == j && nkids[j] == 1 && colcount[j - 1] == colcount[j] + 1;
        if (!extend) sstart.push_back(j);
        sof[j] = static_cast<int32_t>(sstart.size()) - 1;
    }
    const int32_t nf = static_cast<int32_t>(sstart.size());
    sstart.push_back(n);
    std::vector<int32_t> sparent(static_cast<size_t>(nf));
    for (int32_t s = 0; s < nf; ++s) {
        int32_t last = sstart[s + 1] - 1;
        sparent[s] = pa[last] < 0 ? -1 : sof[pa[last]];
    }
    // row sets R_s: every row i is appended to the supernodes of its row subtree
    std::vector<std::vector<int32_t>> R(static_cast<size_t>(nf));
    {
        std::vector<int32_t> seen(static_cast<size_t>(nf), -1);
        for (int32_t i = 0; i < n; ++i) {
            int32_t si = sof[i];
            int32_t oi = q[i];
            for (int64_t p = xadj[oi]; p < xadj[oi + 1]; ++p) {
                int32_t k = iq[adj[p]];
                if (k >= i) continue;
                for (int32_t s = sof[k]; s != si && seen[s] != i; s = sparent[s]) {
                    seen[s] = i;
                    R[s].push_back(i);
                }
            }
        }
    }
    for (int32_t s = 0; s < nf; ++s)
        if (static_cast<int64_t>(R[s].size()) != colcount[sstart[s + 1] - 1] - 1)
            throw std::runtime_error("inconsistent supernode structure");

    // ---- amalgamation: cheapest merge first, (cost, id) order, stop at the first over budget
    const int64_t budget = (static_cast<int64_t>(opt.amalg_pct) * nnz_exact) / 100;
    std::vector<int64_t> width(static_cast<size_t>(nf)), rcnt(static_cast<size_t>(nf)), cost(static_cast<size_t>(nf), 0);
    std::vector<int32_t> up(sparent);
    std::vector<std::vector<int32_t>> kids(static_cast<size_t>(nf)), members(static_cast<size_t>(nf));
    std::vector<char> dead(static_cast<size_t>(nf), 0);
    for (int32_t s = 0; s < nf; ++s) {
        width[s] = sstart[s + 1] - sstart[s];
        rcnt[s] = static_cast<int64_t>(R[s].size());
        members[s].push_back(s);
        if (up[s] >= 0) kids[up[s]].push_back(s);
    }
    using Entry = std::pair<int64_t, int32_t>;
    std::priority_queue<Entry, std::vector<Entry>, std::greater<Entry>> heap;
    auto merge_cost = [&](int32_t c) { int32_t p = up[c]; return width[c] * (width[p] + rcnt[p] - rcnt[c]); };
    for (int32_t s = 0; s < nf; ++s)
        if (up[s] >= 0) { cost[s] = merge_cost(s); heap.emplace(cost[s], s); }
    int64_t used = 0;
    while (!heap.empty()) {
        Entry e = heap.top();
        heap.pop();
        const int32_t c = e.second;
        if (dead[c] || up[c] < 0 || cost[c] != e.first) continue;
        if (used + e.first > budget) break;
        const int32_t p = up[c];
        used += e.first;
        dead[c] = 1;
        width[p] += width[c];
        members[p].insert(members[p].end(), members[c].begin(), members[c].end());
        members[c].clear();
        auto& pk = kids[p];
        pk.erase(std::find(pk.begin(), pk.end(), c));
        for (int32_t x : kids[c]) { up[x] = p; pk.push_back(x); }
        kids[c].clear();
        if (up[p] >= 0) { cost[p] = merge_cost(p); heap.emplace(cost[p], p); }
        for (int32_t x : pk) { cost[x] = merge_cost(x); heap.emplace(cost[x], x); }
    }

    // ---- final postorder of the amalgamated tree
    std::vector<int32_t> alive;
    std::vector<int32_t> compact(static_cast<size_t>(nf), -1);
    for (int32_t s = 0; s < nf; ++s)
        if (!dead[s]) { compact[s] = static_cast<int32_t>(alive.size()); alive.push_back(s); }
    const int32_t nsn = static_cast<int32_t>(alive.size());
    std::vector<int32_t> apar(static_cast<size_t>(nsn));
    for (int32_t a = 0; a < nsn; ++a) apar[a] = up[alive[a]] < 0 ? -1 : compact[up[alive[a]]];
    std::vector<int32_t> apost = postorder_forest(apar);

    P.perm.resize(static_cast<size_t>(n));
    P.iperm.resize(static_cast<size_t>(n));
    P.snptr.resize(static_cast<size_t>(nsn) + 1);
    std::vector<int32_t> relabel(static_cast<size_t>(n));  // postordered label -> final
    std::vector<int32_t> top_of(static_cast<size_t>(nsn));  // fundamental supernode owning R
    std::vector<int32_t> cols;
    int32_t next = 0;
    double flops_exec = 0.0, flops_exec_lu = 0.0;
    for (int32_t t = 0; t < nsn; ++t) {
        const int32_t s = alive[apost[t]];
        top_of[t] = s;
        P.snptr[t] = next;
        cols.clear();
        for (int32_t m : members[s])
            for (int32_t j = sstart[m]; j < sstart[m + 1]; ++j) cols.push_back(j);
        std::sort(cols.begin(), cols.end());
        for (int32_t j : cols) { relabel[j] = next; P.perm[next] = q[j]; ++next; }
        const int64_t w = static_cast<int64_t>(cols.size()), r = rcnt[s];
        for (int64_t i = 0; i < w; ++i) {
            const double e = static_cast<double>(w - i + r);
            flops_exec += e * e;
            flops_exec_lu += 2.0 * (e - 1.0) * (e - 1.0) + (e - 1.0);
        }
    }
    P.snptr[nsn] = next;
    for (int32_t k = 0; k < n; ++k) P.iperm[P.perm[k]] = k;
    P.etree.resize(static_cast<size_t>(n));
    for (int32_t j = 0; j < n; ++j) P.etree[relabel[j]] = pa[j] < 0 ? -1 : relabel[pa[j]];

    // ---- vertical split and blocks
    std::vector<int32_t> cb_sn;
    for (int32_t t = 0; t < nsn; ++t) {
        const int32_t f = P.snptr[t], w = P.snptr[t + 1] - f;
        const int32_t parts = (w + opt.split_width - 1) / opt.split_width;
        const int32_t base = w / parts, wide = w % parts;
        int32_t c0 = f;
        for (int32_t i = 0; i < parts; ++i) {
            const int32_t wi = base + (i < wide ? 1 : 0);
            P.fcol.push_back(c0);
            P.lcol.push_back(c0 + wi - 1);
            cb_sn.push_back(t);
            c0 += wi;
        }
    }
    const int32_t ncblk = static_cast<int32_t>(P.fcol.size());
    std::vector<int32_t> col_cblk(static_cast<size_t>(n));
    for (int32_t k = 0; k < ncblk; ++k)
        for (int32_t j = P.fcol[k]; j <= P.lcol[k]; ++j) col_cblk[j] = k;
    P.bptr.resize(static_cast<size_t>(ncblk) + 1);
    P.stride.resize(static_cast<size_t>(ncblk));
    P.panel_off.resize(static_cast<size_t>(ncblk) + 1);
    P.cparent.resize(static_cast<size_t>(ncblk));
    P.uptr.resize(static_cast<size_t>(ncblk) + 1);
    P.dep.assign(static_cast<size_t>(ncblk), 0);
    std::vector<int32_t> rows;
    int64_t off = 0;
    for (int32_t k = 0; k < ncblk; ++k) {
        const int32_t t = cb_sn[k];
        rows.clear();
        for (int32_t j = P.lcol[k] + 1; j < P.snptr[t + 1]; ++j) rows.push_back(j);
        const size_t tail = rows.size();
        for (int32_t r : R[top_of[t]]) rows.push_back(relabel[r]);
        std::sort(rows.begin() + static_cast<long>(tail), rows.end());
        const int32_t w = P.lcol[k] - P.fcol[k] + 1;
        P.bptr[k] = static_cast<int32_t>(P.frow.size());
        P.frow.push_back(P.fcol[k]);
        P.lrow.push_back(P.lcol[k]);
        P.fcblk.push_back(k);
        P.coefind.push_back(0);
        int32_t h = w;
        size_t a = 0;
        while (a < rows.size()) {
            size_t b = a;
            const int32_t tgt = col_cblk[rows[a]];
            while (b + 1 < rows.size() && rows[b + 1] == rows[b] + 1 && col_cblk[rows[b + 1]] == tgt) ++b;
            P.frow.push_back(rows[a]);
            P.lrow.push_back(rows[b]);
            P.fcblk.push_back(tgt);
            P.coefind.push_back(h);
            h += static_cast<int32_t>(b - a + 1);
            a = b + 1;
        }
        P.stride[k] = h;
        P.panel_off[k] = off;
        off += static_cast<int64_t>(h) * w;
        // update pairs: distinct facing cblks, ascending
        P.uptr[k] = static_cast<int32_t>(P.utgt.size());
        for (size_t b = P.bptr[k] + 1; b < P.frow.size(); ++b) {
            const int32_t j = P.fcblk[b];
            if (P.utgt.size() == static_cast<size_t>(P.uptr[k]) || P.utgt.back() != j) {
                P.utgt.push_back(j);
                ++P.dep[j];
            }
        }
        P.cparent[k] = P.utgt.size() > static_cast<size_t>(P.uptr[k]) ? P.utgt[P.uptr[k]] : -1;
    }
    P.bptr[ncblk] = static_cast<int32_t>(P.frow.size());
    P.uptr[ncblk] = static_cast<int32_t>(P.utgt.size());
    P.panel_off[ncblk] = off;
    P.ncblk = ncblk;
    P.nblok = static_cast<int32_t>(P.frow.size());
    P.nsnode = nsn;
    P.nsn_fund = nf;
    P.nnz_exact = nnz_exact;
    P.zeros_used = used;
    P.nnz_stored = nnz_exact + used;
    P.panel_entries = off;
    P.flops_alg = flops_alg;
    P.flops_exec = flops_exec;
    P.flops_alg_lu = flops_alg_lu;
    P.flops_exec_lu = flops_exec_lu;
    P.col_cblk = std::move(col_cblk);

    build_device_maps(colptr, rowind, P, opt.lu);
}

// Position, inside cblk k's panel, of the row r of its structure (binary search over blocks).
int32_t panel_row(const Plan& P, int32_t k, int32_t r)
{
    int32_t lo = P.bptr[k], hi = P.bptr[k + 1] - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) / 2;
        if (P.frow[mid] <= r) lo = mid; else hi = mid - 1;
    }
    if (P.frow[lo] > r || P.lrow[lo] < r) return -1;
    return P.coefind[lo] + (r - P.frow[lo]);
}

void build_device_maps(const int64_t* colptr, const int32_t* rowind, Plan& P, bool lu)
{
    const int32_t n = P.n;
    const int64_t nnz = colptr[n];
    P.amap.assign(static_cast<size_t>(nnz), -1);
    if (lu) {
        // L U: an entry (a, b) of P A P^T with a >= b goes to the L panel of
        // column b (row a); with a < b to the square diagonal block of the
        // L panel when b is a column of a's block, else to the U^T panel of
        // column a (row b)
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
                const int32_t a = P.iperm[rowind[p]], b = P.iperm[j];
                if (a >= b) {
                    const int32_t k = P.col_cblk[b];
                    const int32_t pos = panel_row(P, k, a);
                    if (pos < 0) throw std::runtime_error("entry outside the symbolic structure");
                    P.amap[p] = P.panel_off[k] + static_cast<int64_t>(b - P.fcol[k]) * P.stride[k] + pos;
                } else {
                    const int32_t k = P.col_cblk[a];
                    if (b <= P.lcol[k]) {
                        P.amap[p] = P.panel_off[k] + static_cast<int64_t>(b - P.fcol[k]) * P.stride[k] + (a - P.fcol[k]);
                    } else {
                        const int32_t pos = panel_row(P, k, b);
                        if (pos < 0) throw std::runtime_error("entry outside the symbolic structure");
                        P.amap[p] = P.panel_entries + P.panel_off[k] +
                                    static_cast<int64_t>(a - P.fcol[k]) * P.stride[k] + pos;
                    }
                }
            }
        // row lists of A itself for the residual: row i lists (column, value
        // index) of every entry (i, j)
        std::vector<int64_t> cnt(static_cast<size_t>(n) + 1, 0);
        for (int64_t p = 0; p < nnz; ++p) ++cnt[rowind[p] + 1];
        for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
        P.rptr = cnt;
        P.rcol.assign(static_cast<size_t>(nnz), 0);
        P.rval.assign(static_cast<size_t>(nnz), 0);
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
                const int32_t i = rowind[p];
                P.rcol[pos[i]] = j;
                P.rval[pos[i]++] = p;
            }
        return;
    }
    // assembly destinations of the lower-triangle entries
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            const int32_t i = rowind[p];
            if (i < j) continue;
            const int32_t a = P.iperm[i], b = P.iperm[j];
            const int32_t r = std::max(a, b), c = std::min(a, b);
            const int32_t k = P.col_cblk[c];
            const int32_t pos = panel_row(P, k, r);
            if (pos < 0) throw std::runtime_error("entry outside the symbolic structure");
            P.amap[p] = P.panel_off[k] + static_cast<int64_t>(c - P.fcol[k]) * P.stride[k] + pos;
        }
    // symmetric row pattern for the residual: row i lists (column, value
    // index) of every lower entry (i, j) and its mirror (j, i)
    std::vector<int64_t> cnt(static_cast<size_t>(n) + 1, 0);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            const int32_t i = rowind[p];
            if (i < j) continue;
            ++cnt[i + 1];
            if (i != j) ++cnt[j + 1];
        }
    for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    P.rptr = cnt;
    P.rcol.assign(static_cast<size_t>(cnt[n]), 0);
    P.rval.assign(static_cast<size_t>(cnt[n]), 0);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            const int32_t i = rowind[p];
            if (i < j) continue;
            P.rcol[pos[i]] = j;
            P.rval[pos[i]++] = p;
            if (i != j) { P.rcol[pos[j]] = i; P.rval[pos[j]++] = p; }
        }
}

}  // namespace spx
