// Symbolic analysis, once per sparsity pattern (the pattern is fixed across
// NCL iterations because only the objective changes, Section IV-A).
//
// Per block template (all contingency blocks share one):
//   exact minimum degree on the template graph (its vertices plus the
//   border vertices it touches): the non-border vertex of smallest current
//   degree goes next (ties: smallest layout index), its neighbours become a
//   clique, border vertices are never eliminated -- or a caller-given
//   elimination sequence instead; the elimination forest's DFS postorder
//   (children and roots by elimination position) is the block order (a
//   topological relabelling of the same elimination: the fill and the
//   factor's entries are those of the sequence); then the symbolic
//   factorisation, the fundamental supernodes (at most kMaxW columns) and
//   relaxed amalgamation.
// The border (first-stage variables) follows all blocks in layout order;
// its structure collects the border rows of every block root.
#include <algorithm>
#include <set>

#include "ncl_internal.h"

namespace ncl {

namespace {

// Elimination on the explicit elimination graph.  adj: block vertices
// 0..n-1, border vertices n.. .  With given == nullptr the next vertex is
// the one of smallest current degree (exact minimum degree, ties to the
// smallest index); otherwise given[0..n) is the elimination sequence.
// Returns the sequence and, per vertex, the block neighbours it had when it
// was eliminated.
void eliminate(int n, std::vector<std::vector<int32_t>> &adj, const int32_t *given, std::vector<int32_t> &seq,
               std::vector<std::vector<int32_t>> &bnbr) {
    std::set<std::pair<int32_t, int32_t>> pq;
    std::vector<char> gone(n, 0);
    for (int v = 0; v < n; v++) pq.insert({int32_t(adj[v].size()), v});
    seq.clear();
    bnbr.assign(n, {});
    std::vector<int32_t> merged;
    while (!pq.empty()) {
        int v;
        if (given) {
            v = given[seq.size()];
            pq.erase({int32_t(adj[v].size()), v});
        } else {
            v = pq.begin()->second;
            pq.erase(pq.begin());
        }
        gone[v] = 1;
        seq.push_back(v);
        const std::vector<int32_t> nv = adj[v];   // remaining neighbours (sorted)
        for (int32_t u : nv)
            if (u < n) bnbr[v].push_back(u);
        for (int32_t u : nv) {
            if (u >= n) continue;                 // border rows are never needed for decisions
            std::vector<int32_t> &au = adj[u];
            pq.erase({int32_t(au.size()), u});
            merged.clear();
            std::set_union(au.begin(), au.end(), nv.begin(), nv.end(), std::back_inserter(merged));
            merged.erase(std::remove_if(merged.begin(), merged.end(), [&](int32_t x) { return x == u || x == v; }),
                         merged.end());
            au.swap(merged);
            pq.insert({int32_t(au.size()), u});
        }
        adj[v].clear();
    }
}

}  // namespace

int analyze_template(Template &t, int nbd, int maxw, int znum, int zden, const int32_t *order) {
    const int n = t.n;
    // undirected adjacency of the template (border as n + b)
    std::vector<std::vector<int32_t>> adj(n);
    for (int c = 0; c < n; c++)
        for (int64_t p = t.colptr[c]; p < t.colptr[c + 1]; p++) {
            int32_t r = t.rowind[p];
            if (r == c) continue;
            adj[c].push_back(r);
            if (r < n) adj[r].push_back(c);
        }
    for (auto &a : adj) {
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    std::vector<int32_t> seq;
    std::vector<std::vector<int32_t>> bnbr;
    if (order) {
        std::vector<char> seen(n, 0);
        for (int j = 0; j < n; j++) {
            if (order[j] < 0 || order[j] >= n || seen[order[j]]) return NCL_ERR_ARG;
            seen[order[j]] = 1;
        }
    }
    eliminate(n, adj, order, seq, bnbr);
    std::vector<int32_t> epos(n);
    for (int s = 0; s < n; s++) epos[seq[s]] = s;
    std::vector<int32_t> mpar(n, -1);
    for (int v = 0; v < n; v++) {
        int32_t best = -1;
        for (int32_t u : bnbr[v])
            if (best < 0 || epos[u] < epos[best]) best = u;
        mpar[v] = best;
    }
    // children lists in increasing elimination position, then DFS postorder
    std::vector<std::vector<int32_t>> kids(n);
    for (int s = 0; s < n; s++)
        if (mpar[seq[s]] >= 0) kids[mpar[seq[s]]].push_back(seq[s]);
    t.perm.clear();
    t.perm.reserve(n);
    std::vector<std::pair<int32_t, size_t>> stk;
    for (int s = 0; s < n; s++) {
        int32_t r = seq[s];
        if (mpar[r] >= 0) continue;
        stk.push_back({r, 0});
        while (!stk.empty()) {
            auto &top = stk.back();
            if (top.second < kids[top.first].size()) {
                int32_t c = kids[top.first][top.second++];
                stk.push_back({c, 0});
            } else {
                t.perm.push_back(top.first);
                stk.pop_back();
            }
        }
    }
    if (int(t.perm.size()) != n) return NCL_ERR_ARG;
    t.iperm.assign(n, 0);
    for (int j = 0; j < n; j++) t.iperm[t.perm[j]] = j;

    // symbolic factorisation in factor numbering
    std::vector<std::vector<int32_t>> low(n);
    for (int c = 0; c < n; c++)
        for (int64_t p = t.colptr[c]; p < t.colptr[c + 1]; p++) {
            int32_t r = t.rowind[p];
            if (r == c) continue;
            int32_t a = r < n ? t.iperm[r] : r, b = t.iperm[c];
            if (a > b) low[b].push_back(a);
            else low[a].push_back(b);
        }
    t.parent.assign(n, -1);
    t.colcount.assign(n, 1);
    t.lp.assign(n + 1, 0);
    t.li.clear();
    std::vector<int32_t> mark(n + nbd, -1), head(n, -1), next(n, -1), buf;
    for (int j = 0; j < n; j++) {
        buf.clear();
        mark[j] = j;
        for (int32_t i : low[j])
            if (mark[i] != j) { mark[i] = j; buf.push_back(i); }
        for (int32_t c = head[j]; c >= 0; c = next[c])
            for (int32_t p = t.lp[c]; p < t.lp[c + 1]; p++) {
                int32_t i = t.li[p];
                if (i > j && mark[i] != j) { mark[i] = j; buf.push_back(i); }
            }
        std::sort(buf.begin(), buf.end());
        t.li.insert(t.li.end(), buf.begin(), buf.end());
        t.lp[j + 1] = int32_t(t.li.size());
        t.colcount[j] = int64_t(buf.size()) + 1;
        if (!buf.empty() && buf[0] < n) {
            t.parent[j] = buf[0];
            next[j] = head[buf[0]];
            head[buf[0]] = j;
        }
    }
    // the elimination forest of the ordering must be this tree (relabelled)
    for (int v = 0; v < n; v++) {
        int32_t want = mpar[v] >= 0 ? t.iperm[mpar[v]] : -1;
        if (t.parent[t.iperm[v]] != want) return NCL_ERR_ARG;
    }
    std::vector<int32_t> nchild(n, 0);
    for (int j = 0; j < n; j++)
        if (t.parent[j] >= 0) nchild[t.parent[j]]++;
    // fundamental supernodes
    std::vector<int32_t> fs{0};
    int run = 1;
    for (int j = 0; j + 1 < n; j++) {
        bool join = t.parent[j] == j + 1 && t.colcount[j] == t.colcount[j + 1] + 1 && nchild[j + 1] == 1 && run < kMaxW;
        if (join) run++;
        else { fs.push_back(j + 1); run = 1; }
    }
    fs.push_back(n);
    // relaxed amalgamation (left to right, the current supernode absorbs the next)
    t.sup.clear();
    std::vector<int32_t> rmark(n + nbd, -1);
    int stamp = 0;
    int32_t cf = fs[0], cl = fs[1] - 1;
    for (size_t q = 1; q + 1 < fs.size(); q++) {
        int32_t pf = fs[q], pl = fs[q + 1] - 1;
        int64_t w = pl - cf + 1;
        bool ok = t.parent[cl] == pf && w <= maxw && w <= kMaxW;
        if (ok) {
            stamp++;
            int64_t off = 0, truenz = 0;
            for (int32_t j = cf; j <= pl; j++) {
                truenz += t.colcount[j];
                for (int32_t p = t.lp[j]; p < t.lp[j + 1]; p++) {
                    int32_t i = t.li[p];
                    if (i > pl && rmark[i] != stamp) { rmark[i] = stamp; off++; }
                }
            }
            int64_t entries = w * (w + 1) / 2 + w * off;
            ok = int64_t(zden) * (entries - truenz) <= int64_t(znum) * entries;
        }
        if (ok) cl = pl;
        else {
            t.sup.push_back(cf);
            cf = pf;
            cl = pl;
        }
    }
    t.sup.push_back(cf);
    t.sup.push_back(n);
    // panel rows
    const int ns = int(t.sup.size()) - 1;
    t.srp.assign(ns + 1, 0);
    t.sri.clear();
    for (int s = 0; s < ns; s++) {
        int32_t f = t.sup[s], l = t.sup[s + 1] - 1;
        for (int32_t j = f; j <= l; j++) t.sri.push_back(j);
        size_t c0 = t.sri.size();
        stamp++;
        for (int32_t j = f; j <= l; j++)
            for (int32_t p = t.lp[j]; p < t.lp[j + 1]; p++) {
                int32_t i = t.li[p];
                if (i > l && rmark[i] != stamp) { rmark[i] = stamp; t.sri.push_back(i); }
            }
        std::sort(t.sri.begin() + c0, t.sri.end());
        t.srp[s + 1] = int32_t(t.sri.size());
    }
    return NCL_OK;
}

int analyze_border(Handle &h, Inst &I, int maxw, int znum, int zden) {
    const int nbd = I.nbd;
    I.bparent.assign(nbd, -1);
    I.bcolcount.assign(nbd, 1);
    I.blp.assign(nbd + 1, 0);
    I.bli.clear();
    I.bsup.clear();
    if (nbd == 0) return NCL_OK;
    // border rows of each template's roots, and how many blocks use each template
    std::vector<int> uses(h.tmpl.size(), 0);
    for (int b = I.blk0; b < I.blk0 + I.nblk; b++) uses[h.block_tmpl[b]]++;
    std::vector<std::vector<std::vector<int32_t>>> rootrows(h.tmpl.size());   // per template, per root
    std::vector<std::vector<int32_t>> root_kids(nbd);      // (template, root) -> child of border column
    std::vector<int64_t> nchild(nbd, 0);
    std::vector<std::vector<std::pair<int, int>>> kids(nbd);
    for (size_t ti = size_t(I.t0); ti < size_t(I.t0 + I.nt); ti++) {
        const Template &t = h.tmpl[ti];
        for (int j = 0; j < t.n; j++) {
            if (t.parent[j] >= 0) continue;
            std::vector<int32_t> rows;
            for (int32_t p = t.lp[j]; p < t.lp[j + 1]; p++)
                if (t.li[p] >= t.n) rows.push_back(t.li[p] - t.n);
            if (rows.empty()) continue;
            int idx = int(rootrows[ti].size());
            rootrows[ti].push_back(rows);
            kids[rows[0]].push_back({int(ti), idx});
            nchild[rows[0]] += uses[ti];
        }
    }
    std::vector<int32_t> mark(nbd, -1), head(nbd, -1), next(nbd, -1), buf;
    for (int b = 0; b < nbd; b++) {
        buf.clear();
        mark[b] = b;
        for (int64_t p = I.bcolptr[b]; p < I.bcolptr[b + 1]; p++) {
            int32_t i = I.browind[p];
            if (i > b && mark[i] != b) { mark[i] = b; buf.push_back(i); }
        }
        for (auto &k : kids[b])
            for (int32_t i : rootrows[k.first][k.second])
                if (i > b && mark[i] != b) { mark[i] = b; buf.push_back(i); }
        for (int32_t c = head[b]; c >= 0; c = next[c])
            for (int32_t p = I.blp[c]; p < I.blp[c + 1]; p++) {
                int32_t i = I.bli[p];
                if (i > b && mark[i] != b) { mark[i] = b; buf.push_back(i); }
            }
        std::sort(buf.begin(), buf.end());
        I.bli.insert(I.bli.end(), buf.begin(), buf.end());
        I.blp[b + 1] = int32_t(I.bli.size());
        I.bcolcount[b] = int64_t(buf.size()) + 1;
        if (!buf.empty()) {
            I.bparent[b] = buf[0];
            next[b] = head[buf[0]];
            head[buf[0]] = b;
            nchild[buf[0]]++;
        }
    }
    std::vector<int32_t> fs{0};
    int run = 1;
    for (int j = 0; j + 1 < nbd; j++) {
        bool join = I.bparent[j] == j + 1 && I.bcolcount[j] == I.bcolcount[j + 1] + 1 && nchild[j + 1] == 1 && run < kMaxW;
        if (join) run++;
        else { fs.push_back(j + 1); run = 1; }
    }
    fs.push_back(nbd);
    std::vector<int32_t> rmark(nbd, -1);
    int stamp = 0;
    int32_t cf = fs[0], cl = fs[1] - 1;
    for (size_t q = 1; q + 1 < fs.size(); q++) {
        int32_t pf = fs[q], pl = fs[q + 1] - 1;
        int64_t w = pl - cf + 1;
        bool ok = I.bparent[cl] == pf && w <= maxw && w <= kMaxW;
        if (ok) {
            stamp++;
            int64_t off = 0, truenz = 0;
            for (int32_t j = cf; j <= pl; j++) {
                truenz += I.bcolcount[j];
                for (int32_t p = I.blp[j]; p < I.blp[j + 1]; p++) {
                    int32_t i = I.bli[p];
                    if (i > pl && rmark[i] != stamp) { rmark[i] = stamp; off++; }
                }
            }
            int64_t entries = w * (w + 1) / 2 + w * off;
            ok = int64_t(zden) * (entries - truenz) <= int64_t(znum) * entries;
        }
        if (ok) cl = pl;
        else {
            I.bsup.push_back(cf);
            cf = pf;
            cl = pl;
        }
    }
    I.bsup.push_back(cf);
    I.bsup.push_back(nbd);
    return NCL_OK;
}

}  // namespace ncl
