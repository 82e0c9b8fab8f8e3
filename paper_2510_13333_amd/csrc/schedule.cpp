// Schedules for the numeric kernels, built once per template from the
// supernode partition.
//
// Factor (left-looking, one workgroup per block): supernodes are grouped
// by level (leaves 0; a parent is above all its children), and every panel
// row of a supernode is one "row task".  A row task of target supernode t
// gathers, in increasing order of d, the contribution of every descendant
// supernode d whose panel holds both that row and one of t's columns:
//     P_t[row, c] -= sum_{k in cols(d)} L_d[row, k] d_k L_d[c, k].
// The task's K entries seed its accumulator first.
#include <algorithm>

#include "ncl_internal.h"

namespace ncl {

int64_t panel_entries(const Template &t) {
    int64_t e = 0;
    const int ns = int(t.sup.size()) - 1;
    for (int s = 0; s < ns; s++) e += int64_t(t.srp[s + 1] - t.srp[s]) * (t.sup[s + 1] - t.sup[s]);
    return e;
}

int build_schedule(Template &t, int nbd) {
    const int n = t.n;
    const int ns = int(t.sup.size()) - 1;
    std::vector<int32_t> col2sup(n);
    for (int s = 0; s < ns; s++)
        for (int j = t.sup[s]; j < t.sup[s + 1]; j++) col2sup[j] = s;
    t.panel_off.assign(ns + 1, 0);
    for (int s = 0; s < ns; s++) {
        int64_t sz = int64_t(t.srp[s + 1] - t.srp[s]) * (t.sup[s + 1] - t.sup[s]);
        int64_t nx = int64_t(t.panel_off[s]) + sz;
        if (nx >= (int64_t(1) << 31)) return NCL_ERR_ARG;
        t.panel_off[s + 1] = int32_t(nx);
        if (t.srp[s + 1] - t.srp[s] > 65535) return NCL_ERR_ARG;
    }
    // supernodal tree and levels
    std::vector<int32_t> spar(ns, -1), level(ns, 0);
    for (int s = 0; s < ns; s++) {
        int32_t p = t.parent[t.sup[s + 1] - 1];
        spar[s] = p >= 0 ? col2sup[p] : -1;
    }
    for (int s = 0; s < ns; s++)
        if (spar[s] >= 0) level[spar[s]] = std::max(level[spar[s]], level[s] + 1);
    int nlev = 0;
    for (int s = 0; s < ns; s++) nlev = std::max(nlev, level[s] + 1);
    t.nlev = nlev;
    t.lev_sup_ptr.assign(nlev + 1, 0);
    for (int s = 0; s < ns; s++) t.lev_sup_ptr[level[s] + 1]++;
    for (int l = 0; l < nlev; l++) t.lev_sup_ptr[l + 1] += t.lev_sup_ptr[l];
    t.lev_sup.assign(ns, 0);
    {
        std::vector<int32_t> fill(t.lev_sup_ptr.begin(), t.lev_sup_ptr.end() - 1);
        for (int s = 0; s < ns; s++) t.lev_sup[fill[level[s]]++] = s;
    }
    // row tasks, grouped by level then supernode
    std::vector<int32_t> task_base(ns, 0);
    t.task_s.clear();
    t.task_p.clear();
    t.lev_task_ptr.assign(nlev + 1, 0);
    t.lev_dtask_ptr.assign(nlev + 1, 0);
    t.dtask.clear();
    for (int l = 0; l < nlev; l++) {
        for (int q = t.lev_sup_ptr[l]; q < t.lev_sup_ptr[l + 1]; q++) {
            int s = t.lev_sup[q];
            task_base[s] = int32_t(t.task_s.size());
            int r = t.srp[s + 1] - t.srp[s], w = t.sup[s + 1] - t.sup[s];
            for (int p = 0; p < r; p++) {
                if (p < w) t.dtask.push_back(int32_t(t.task_s.size()));
                t.task_s.push_back(s);
                t.task_p.push_back(p);
            }
        }
        t.lev_task_ptr[l + 1] = int32_t(t.task_s.size());
        t.lev_dtask_ptr[l + 1] = int32_t(t.dtask.size());
    }
    const int ntask = int(t.task_s.size());
    auto pos_in = [&](int s, int32_t row) -> int32_t {
        auto b = t.sri.begin() + t.srp[s], e = t.sri.begin() + t.srp[s + 1];
        auto it = std::lower_bound(b, e, row);
        if (it == e || *it != row) return -1;
        return int32_t(it - b);
    };
    // gather items: for each descendant d (ascending), each target supernode
    // touched by its off-diagonal rows, each row of the tail
    std::vector<std::vector<GItem>> items(ntask);
    t.crel.clear();
    for (int d = 0; d < ns; d++) {
        const int r = t.srp[d + 1] - t.srp[d], w = t.sup[d + 1] - t.sup[d];
        const int32_t *R = &t.sri[t.srp[d]];
        int q = w;
        while (q < r && R[q] < n) {
            int tgt = col2sup[R[q]];
            int q0 = q;
            while (q < r && R[q] < n && col2sup[R[q]] == tgt) q++;
            int nc = q - q0;
            int32_t croff = int32_t(t.crel.size());
            for (int a = q0; a < q0 + nc; a++) t.crel.push_back(uint8_t(R[a] - t.sup[tgt]));
            GItem g;
            g.coff = t.panel_off[d] + q0;
            g.dcol = t.sup[d];
            g.crel = croff;
            g.meta = int32_t(uint32_t(r) | (uint32_t(w) << 16) | (uint32_t(nc) << 24));
            for (int a = q0; a < r; a++) {
                int32_t pt = pos_in(tgt, R[a]);
                if (pt < 0) return NCL_ERR_ARG;      // not a valid supernodal structure
                g.ioff = t.panel_off[d] + a;
                items[task_base[tgt] + pt].push_back(g);
            }
        }
    }
    t.task_gptr.assign(ntask + 1, 0);
    for (int k = 0; k < ntask; k++) t.task_gptr[k + 1] = t.task_gptr[k] + int32_t(items[k].size());
    t.gitems.clear();
    t.gitems.reserve(t.task_gptr[ntask]);
    for (auto &v : items) t.gitems.insert(t.gitems.end(), v.begin(), v.end());
    // K entries of each row task
    std::vector<std::vector<AEnt>> ae(ntask);
    for (int c = 0; c < n; c++)
        for (int64_t p = t.colptr[c]; p < t.colptr[c + 1]; p++) {
            int32_t r = t.rowind[p];
            int32_t a = r < n ? t.iperm[r] : r, b = t.iperm[c];
            int32_t col = std::min(a, b), row = std::max(a, b);
            int s = col2sup[col];
            int32_t pr = pos_in(s, row);
            if (pr < 0) return NCL_ERR_ARG;
            ae[task_base[s] + pr].push_back(AEnt{int32_t(p), col - t.sup[s]});
        }
    t.task_aptr.assign(ntask + 1, 0);
    for (int k = 0; k < ntask; k++) t.task_aptr[k + 1] = t.task_aptr[k] + int32_t(ae[k].size());
    t.aents.clear();
    for (auto &v : ae) t.aents.insert(t.aents.end(), v.begin(), v.end());
    // every offset a kernel dereferences stays inside its panel / value range
    const int64_t nnzk = t.colptr[n];
    for (int k = 0; k < ntask; k++) {
        const int s = t.task_s[k];
        const int ws = t.sup[s + 1] - t.sup[s];
        for (int e = t.task_gptr[k]; e < t.task_gptr[k + 1]; e++) {
            const GItem &g = t.gitems[e];
            const int ld = g.meta & 0xffff, wd = (g.meta >> 16) & 0xff, nc = (g.meta >> 24) & 0xff;
            const int d = (g.dcol >= 0 && g.dcol < n) ? col2sup[g.dcol] : -1;
            if (d < 0 || t.sup[d] != g.dcol || wd != t.sup[d + 1] - t.sup[d] || ld != t.srp[d + 1] - t.srp[d]) return NCL_ERR_ARG;
            const int64_t lim = t.panel_off[d + 1];
            if (g.ioff < t.panel_off[d] || g.ioff + int64_t(wd - 1) * ld >= lim) return NCL_ERR_ARG;
            if (g.coff < t.panel_off[d] || g.coff + (nc - 1) + int64_t(wd - 1) * ld >= lim || nc < 1) return NCL_ERR_ARG;
            for (int q = 0; q < nc; q++)
                if (t.crel[g.crel + q] >= ws) return NCL_ERR_ARG;
        }
        for (int e = t.task_aptr[k]; e < t.task_aptr[k + 1]; e++)
            if (t.aents[e].kpos < 0 || t.aents[e].kpos >= nnzk || t.aents[e].crel < 0 || t.aents[e].crel >= ws)
                return NCL_ERR_ARG;
        if (t.task_p[k] >= t.srp[s + 1] - t.srp[s]) return NCL_ERR_ARG;
    }
    // border rows: the supernodes whose panel holds them
    t.bpath_ptr.assign(nbd + 1, 0);
    std::vector<std::vector<std::pair<int32_t, int32_t>>> bp(nbd);
    for (int s = 0; s < ns; s++)
        for (int p = t.srp[s]; p < t.srp[s + 1]; p++)
            if (t.sri[p] >= n) bp[t.sri[p] - n].push_back({s, p - t.srp[s]});
    t.bpath_s.clear();
    t.bpath_pos.clear();
    for (int b = 0; b < nbd; b++) {
        for (auto &x : bp[b]) {
            t.bpath_s.push_back(x.first);
            t.bpath_pos.push_back(x.second);
        }
        t.bpath_ptr[b + 1] = int32_t(t.bpath_s.size());
    }
    return NCL_OK;
}

}  // namespace ncl
