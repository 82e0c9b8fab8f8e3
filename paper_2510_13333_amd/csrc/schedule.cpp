// Schedules of the numeric kernels, built once per pattern.
//
// Factor, left-looking over supernodes grouped by level (leaves 0; a parent
// sits above all its children).  Every entry (row, column c) of a panel in
// the lower triangle is seeded with its K value and gathers, in increasing
// order of d, the contribution of every descendant supernode d whose panel
// holds both the row and the column c:
//     P[row, c] -= sum_{k in cols(d)} L_d[row, k] d_k L_d[c, k].
// Each level then factors the diagonal blocks of its wide supernodes and
// solves the off-diagonal rows.  All blocks of a template run the same
// schedule, one block per lane.
#include <algorithm>

#include "ncl_internal.h"

namespace ncl {

// Full symmetric rows of a template's K for the residual b - Kx: the lower
// CSC entry (r, c) at position p counts in row r (times x_c) and, off the
// diagonal, in row c (times x_r); a border row r = n + b collects the
// block's entries of that row separately (its sum runs over the blocks).
static void build_residual_rows(Template &t, int nbd) {
    const int n = t.n;
    std::vector<std::vector<int32_t>> rows(n), brows(nbd);
    for (int c = 0; c < n; c++)
        for (int64_t p = t.colptr[c]; p < t.colptr[c + 1]; p++) {
            const int32_t r = t.rowind[p];
            if (r < n) {
                rows[r].push_back(int32_t(p));
                rows[r].push_back(c);
                if (r != c) {
                    rows[c].push_back(int32_t(p));
                    rows[c].push_back(r);
                }
            } else {
                rows[c].push_back(int32_t(p));
                rows[c].push_back(r);
                brows[r - n].push_back(int32_t(p));
                brows[r - n].push_back(c);
            }
        }
    t.rr_ptr.assign(1, 0);
    t.rr_ent.clear();
    for (auto &r : rows) {
        t.rr_ent.insert(t.rr_ent.end(), r.begin(), r.end());
        t.rr_ptr.push_back(int32_t(t.rr_ent.size() / 2));
    }
    t.rb_ptr.assign(1, 0);
    t.rb_ent.clear();
    for (auto &r : brows) {
        t.rb_ent.insert(t.rb_ent.end(), r.begin(), r.end());
        t.rb_ptr.push_back(int32_t(t.rb_ent.size() / 2));
    }
}

int build_template_schedule(Template &t, int nbd) {
    const int n = t.n;
    build_residual_rows(t, nbd);
    const int ns = int(t.sup.size()) - 1;
    std::vector<int32_t> col2sup(n);
    for (int s = 0; s < ns; s++)
        for (int j = t.sup[s]; j < t.sup[s + 1]; j++) col2sup[j] = s;
    t.panel_off.assign(ns + 1, 0);
    for (int s = 0; s < ns; s++) {
        const int64_t sz = int64_t(t.srp[s + 1] - t.srp[s]) * (t.sup[s + 1] - t.sup[s]);
        const int64_t nx = int64_t(t.panel_off[s]) + sz;
        if (nx >= (int64_t(1) << 31) || t.srp[s + 1] - t.srp[s] > 65535) return NCL_ERR_ARG;
        t.panel_off[s + 1] = int32_t(nx);
    }
    // supernodal tree levels
    t.level.assign(ns, 0);
    for (int s = 0; s < ns; s++) {
        const int32_t p = t.parent[t.sup[s + 1] - 1];
        if (p >= 0) {
            const int ps = col2sup[p];
            t.level[ps] = std::max(t.level[ps], t.level[s] + 1);
        }
    }
    t.nlev = 0;
    for (int s = 0; s < ns; s++) t.nlev = std::max(t.nlev, t.level[s] + 1);
    // row tasks by level, supernode, row
    t.lev_tasks.assign(t.nlev, {});
    std::vector<std::vector<int32_t>> bylev(t.nlev);
    for (int s = 0; s < ns; s++) bylev[t.level[s]].push_back(s);
    std::vector<int32_t> task_base(ns, 0);
    t.task_s.clear();
    t.task_p.clear();
    t.task_cbase.assign(1, 0);
    for (int l = 0; l < t.nlev; l++)
        for (int s : bylev[l]) {
            task_base[s] = int32_t(t.task_s.size());
            const int r = t.srp[s + 1] - t.srp[s], w = t.sup[s + 1] - t.sup[s];
            for (int p = 0; p < r; p++) {
                t.lev_tasks[l].push_back(int32_t(t.task_s.size()));
                t.task_s.push_back(s);
                t.task_p.push_back(p);
                t.task_cbase.push_back(t.task_cbase.back() + w);
            }
        }
    const int ntask = int(t.task_s.size());
    const int nent = t.task_cbase[ntask];
    auto pos_in = [&](int s, int32_t row) -> int32_t {
        auto b = t.sri.begin() + t.srp[s], e = t.sri.begin() + t.srp[s + 1];
        auto it = std::lower_bound(b, e, row);
        if (it == e || *it != row) return -1;
        return int32_t(it - b);
    };
    // panel element of every entry (row p, column c of supernode s)
    t.ent_out.assign(nent, 0);
    for (int k = 0; k < ntask; k++) {
        const int s = t.task_s[k], p = t.task_p[k];
        const int r = t.srp[s + 1] - t.srp[s];
        for (int c = 0; c < t.task_cbase[k + 1] - t.task_cbase[k]; c++)
            t.ent_out[t.task_cbase[k] + c] = t.panel_off[s] + c * r + p;
    }
    // K value of every panel entry
    t.ent_kpos.assign(nent, -1);
    for (int c = 0; c < n; c++)
        for (int64_t p = t.colptr[c]; p < t.colptr[c + 1]; p++) {
            const int32_t r = t.rowind[p];
            const int32_t a = r < n ? t.iperm[r] : r, b = t.iperm[c];
            const int32_t col = std::min(a, b), row = std::max(a, b);
            const int s = col2sup[col];
            const int32_t pr = pos_in(s, row);
            if (pr < 0) return NCL_ERR_ARG;
            t.ent_kpos[t.task_cbase[task_base[s] + pr] + (col - t.sup[s])] = int32_t(p);
        }
    // gather items of every panel entry, descendants in increasing order
    std::vector<std::vector<CItem>> items(nent);
    for (int d = 0; d < ns; d++) {
        const int r = t.srp[d + 1] - t.srp[d], w = t.sup[d + 1] - t.sup[d];
        const int32_t *R = &t.sri[t.srp[d]];
        int q = w;
        while (q < r && R[q] < n) {
            const int tgt = col2sup[R[q]];
            const int q0 = q;
            while (q < r && R[q] < n && col2sup[R[q]] == tgt) q++;
            for (int a = q0; a < r; a++) {
                const int32_t pt = pos_in(tgt, R[a]);
                if (pt < 0) return NCL_ERR_ARG;   // not a valid supernodal structure
                const int tk = task_base[tgt] + pt;
                for (int qc = q0; qc < q; qc++) {
                    if (R[qc] > R[a]) break;          // upper triangle of the diagonal block
                    CItem g;
                    g.ioff = t.panel_off[d] + a;
                    g.coff = t.panel_off[d] + qc;
                    g.dcol = t.sup[d];
                    g.meta = int32_t(uint32_t(r) | (uint32_t(w) << 16));
                    items[t.task_cbase[tk] + (R[qc] - t.sup[tgt])].push_back(g);
                }
            }
        }
    }
    std::vector<CItem> citems;
    for (auto &v : items) citems.insert(citems.end(), v.begin(), v.end());
    // every element a kernel dereferences stays inside its panel
    for (const CItem &g : citems) {
        const int ld = g.meta & 0xffff, wd = (g.meta >> 16) & 0xff;
        const int d = (g.dcol >= 0 && g.dcol < n) ? col2sup[g.dcol] : -1;
        if (d < 0 || t.sup[d] != g.dcol || wd != t.sup[d + 1] - t.sup[d] || ld != t.srp[d + 1] - t.srp[d])
            return NCL_ERR_ARG;
        const int64_t lo = t.panel_off[d], hi = t.panel_off[d + 1];
        if (g.ioff < lo || g.ioff + int64_t(wd - 1) * ld >= hi) return NCL_ERR_ARG;
        if (g.coff < lo || g.coff + int64_t(wd - 1) * ld >= hi) return NCL_ERR_ARG;
    }
    for (int e = 0; e < nent; e++)
        if (t.ent_kpos[e] >= int64_t(t.colptr[n])) return NCL_ERR_ARG;
    // flatten: one term per (descendant, column of the descendant)
    const int64_t kTermMax = INT32_MAX;
    t.ent_tptr.assign(nent + 1, 0);
    t.terms.clear();
    for (int e = 0; e < nent; e++) {
        for (const CItem &g : items[e]) {
            const int ld = g.meta & 0xffff, wd = (g.meta >> 16) & 0xff;
            for (int k = 0; k < wd; k++) t.terms.push_back(Term{g.ioff + k * ld, g.coff + k * ld, g.dcol + k, 0});
        }
        if (int64_t(t.terms.size()) > kTermMax) return NCL_ERR_ARG;
        t.ent_tptr[e + 1] = int32_t(t.terms.size());
    }
    items.clear();
    items.shrink_to_fit();
    // border rows: the supernodes whose panel holds them, ascending
    std::vector<std::vector<std::pair<int32_t, int32_t>>> bp(nbd);
    for (int s = 0; s < ns; s++)
        for (int p = t.srp[s]; p < t.srp[s + 1]; p++)
            if (t.sri[p] >= n) bp[t.sri[p] - n].push_back({s, p - t.srp[s]});
    auto push_cols = [&](std::vector<Term> &out, int s, int pi, int pj) {
        const int r = t.srp[s + 1] - t.srp[s], w = t.sup[s + 1] - t.sup[s];
        for (int k = 0; k < w; k++)
            out.push_back(Term{t.panel_off[s] + pi + k * r, t.panel_off[s] + pj + k * r, t.sup[s] + k, 0});
    };
    // border right-hand side terms: L[b, k] over the columns k of those panels
    t.bterm_ptr.assign(nbd + 1, 0);
    t.bterms.clear();
    for (int b = 0; b < nbd; b++) {
        for (auto &x : bp[b]) push_cols(t.bterms, x.first, x.second, x.second);
        if (int64_t(t.bterms.size()) > kTermMax) return NCL_ERR_ARG;
        t.bterm_ptr[b + 1] = int32_t(t.bterms.size());
    }
    // backward solve: block rows of each panel (border rows come last)
    t.sup_rnb.assign(ns, 0);
    t.col_sup = col2sup;
    for (int s = 0; s < ns; s++) {
        int rnb = t.srp[s + 1] - t.srp[s];
        while (rnb > 0 && t.sri[t.srp[s] + rnb - 1] >= n) rnb--;
        if (rnb < t.sup[s + 1] - t.sup[s]) return NCL_ERR_ARG;
        t.sup_rnb[s] = rnb;
    }
    // border rows of each supernode (the border Schur items are built per
    // instance, over a permutation of the border shared by its templates)
    t.brow.assign(ns, {});
    for (int b = 0; b < nbd; b++)
        for (auto &x : bp[b]) t.brow[x.first].push_back({b, x.second});
    return NCL_OK;
}

int build_schedule(Handle &h) {
    Schedule &S = h.sched;
    S = Schedule();
    h.t_kbase.assign(h.tmpl.size(), 0);
    h.t_lbase.assign(h.tmpl.size(), 0);
    h.t_dbase.assign(h.tmpl.size(), 0);
    h.t_abase.assign(h.tmpl.size(), 0);
    h.t_awbase.assign(h.tmpl.size(), 0);
    h.t_tile0.assign(h.tmpl.size(), 0);
    h.t_rwbase.assign(h.tmpl.size(), 0);
    h.kint = h.lint = h.dint = h.asm_threads = h.asm_wthreads = h.tiles = h.rows_waves = 0;
    for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
        const Template &t = h.tmpl[ti];
        const int64_t nb = int64_t(t.blocks.size());
        // kernels address a template's panels, pivots and vectors with 32-bit
        // byte offsets from the template's base
        if (int64_t(t.n) * nb >= (int64_t(1) << 29) || int64_t(t.panel_off.back()) * nb >= (int64_t(1) << 29) ||
            int64_t(t.colptr[t.n]) * nb >= (int64_t(1) << 29))
            return NCL_ERR_ARG;
        h.t_kbase[ti] = h.kint;
        h.t_lbase[ti] = h.lint;
        h.t_dbase[ti] = h.dint;
        h.t_abase[ti] = h.asm_threads;
        h.t_awbase[ti] = h.asm_wthreads;
        h.t_tile0[ti] = h.tiles;
        h.t_rwbase[ti] = h.rows_waves;
        h.rows_waves += int64_t(t.n) * ((nb + 63) / 64);
        h.tiles += int64_t((t.n + kTileJ - 1) / kTileJ) * ((nb + kTileB - 1) / kTileB);
        h.kint += t.colptr[t.n] * nb;
        h.lint += int64_t(t.panel_off.back()) * nb;
        h.dint += int64_t(t.n) * nb;
        if (h.from_network) {
            h.asm_threads += nb * (h.inst[t.inst].nb + h.inst[t.inst].ng);
            h.asm_wthreads += (nb + 63) / 64 * 64 * (h.inst[t.inst].nb + h.inst[t.inst].ng);
        }
        S.nlev = std::max(S.nlev, t.nlev);
    }
    if (h.tmpl.size() > 32767) return NCL_ERR_ARG;
    auto groups = [](const Template &t, int per) { return (int(t.blocks.size()) + per - 1) / per; };
    auto tg = [](size_t ti, int g) { return int32_t((uint32_t(ti) << 16) | uint32_t(g)); };
    S.a_ptr.assign(1, 0);
    S.b_ptr.assign(1, 0);
    S.c_ptr.assign(1, 0);
    S.f_ptr.assign(1, 0);
    S.d_ptr.assign(1, 0);
    S.sn_ptr.assign(1, 0);
    S.sn_nar.clear();
    S.sn_wmax.clear();
    S.sn.clear();
    // backward border step: every supernode of every template and group,
    // narrow ones first
    S.sb.clear();
    for (int wide = 0; wide < 2; wide++) {
        for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
            const Template &t = h.tmpl[ti];
            for (int g = 0; g < groups(t, 64); g++)
                for (int j = 0; j < t.n; j++) {
                    const int s = t.col_sup[j];
                    const bool wd = t.srp[s + 1] - t.srp[s] - t.sup_rnb[s] > kSolBorderWideRows;
                    if (wd != (wide == 1)) continue;
                    S.sb.push_back(Work{tg(ti, g), j | (wd ? kWideFlag : 0)});
                }
        }
        if (!wide) S.sb_nar = int32_t(S.sb.size());
    }
    // Work lists are group-major: within a (level, template) every item of
    // one block group comes before the next group's, so that contiguous runs
    // of a list share the same blocks' panels.  The list kernels map
    // contiguous workgroup ranges to one XCD each, so such a run is served
    // by one L2.
    for (int l = 0; l < S.nlev; l++) {
        // solve items: the level's narrow supernodes of every template and
        // group, then the wide ones
        int wmax = 1;
        for (int wide = 0; wide < 2; wide++) {
            for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
                const Template &t = h.tmpl[ti];
                if (l >= t.nlev) continue;
                const int ng64 = groups(t, 64);
                for (int g = 0; g < ng64; g++) {
                    int last_s = -1;
                    for (int32_t k : t.lev_tasks[l]) {
                        const int s = t.task_s[k];
                        if (s == last_s) continue;
                        last_s = s;
                        const int w = t.sup[s + 1] - t.sup[s];
                        const bool wd = w > kNarrowW || t.sup_rnb[s] - w > kSolWideRows;
                        if (wd != (wide == 1)) continue;
                        S.sn.push_back(Work{tg(ti, g), s | (wd ? kWideFlag : 0)});
                        wmax = std::max(wmax, w);
                    }
                }
            }
            if (!wide) S.sn_nar.push_back(int32_t(S.sn.size()) - S.sn_ptr.back());
        }
        S.sn_ptr.push_back(int32_t(S.sn.size()));
        S.sn_wmax.push_back(wmax);
        for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
            const Template &t = h.tmpl[ti];
            if (l >= t.nlev) continue;
            const int ng64 = groups(t, 64), ng2 = groups(t, 2);
            if (ng64 > 65535 || ng2 > 65535) return NCL_ERR_ARG;
            for (int g = 0; g < ng64; g++) {
                int last_s = -1;
                for (int32_t k : t.lev_tasks[l]) {
                    const int s = t.task_s[k], p = t.task_p[k];
                    const int w = t.sup[s + 1] - t.sup[s];
                    const int cend = p < w ? p + 1 : w;     // lower triangle of the diagonal block
                    for (int c = 0; c < cend; c++) S.a.push_back(Work{tg(ti, g), t.task_cbase[k] + c});
                    if (w > 1 && p >= w) S.c.push_back(Work{tg(ti, g), k});
                    // forward solve: the diagonal entry's terms are exactly the
                    // descendants holding this row
                    if (p < w && t.ent_tptr[t.task_cbase[k] + p + 1] > t.ent_tptr[t.task_cbase[k] + p])
                        S.f.push_back(Work{tg(ti, g), k});
                    if (w > 1 && s != last_s) S.d.push_back(Work{tg(ti, g), s});
                    last_s = s;
                }
            }
            // diagonal blocks: width-1 pivots and narrow blocks per 64-block
            // group (a block per lane), wide ones per 2-block group (a block
            // per half wavefront)
            for (int g = 0; g < ng64; g++) {
                int last_s = -1;
                for (int32_t k : t.lev_tasks[l]) {
                    const int s = t.task_s[k];
                    const int w = t.sup[s + 1] - t.sup[s];
                    if (w == 1 && s != last_s) S.b.push_back(Work{tg(ti, g), s | kPivotFlag});
                    if (w > 1 && w <= kNarrowW && s != last_s) S.b.push_back(Work{tg(ti, g), s | kNarrowFlag});
                    last_s = s;
                }
            }
            for (int g = 0; g < ng2; g++) {
                int last_s = -1;
                for (int32_t k : t.lev_tasks[l]) {
                    const int s = t.task_s[k];
                    const int w = t.sup[s + 1] - t.sup[s];
                    if (w > kNarrowW && s != last_s) S.b.push_back(Work{tg(ti, g), s});
                    last_s = s;
                }
            }
        }
        S.a_ptr.push_back(int32_t(S.a.size()));
        S.f_ptr.push_back(int32_t(S.f.size()));
        S.d_ptr.push_back(int32_t(S.d.size()));
        S.b_ptr.push_back(int32_t(S.b.size()));
        S.c_ptr.push_back(int32_t(S.c.size()));

    }
    for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
        const Template &t = h.tmpl[ti];
        const int nbd = h.inst[t.inst].nbd;
        const int ng64 = groups(t, 64);
        for (int g = 0; g < ng64; g++)
            for (int b = 0; b < nbd; b++) S.bpart.push_back(Work{tg(ti, g), b});
    }
    // border Schur items of each instance.  The border rows are placed in
    // tiles of kMT in the order of the first supernode (elimination order)
    // of the instance's largest template that holds them, so that the rows
    // of a supernode share few tiles; then per pair of tiles (I >= J), one
    // item per supernode (every template in order) holding rows of both.
    // The wavefront slices: per pair, per chunk of kMC blocks, the items of
    // the templates with blocks in the chunk cut (never across a template)
    // into runs of about kMSlice instructions, an item counting kMItemCost
    // more for its dependent loads.
    for (Inst &I : h.inst) {
        I.mitems.clear();
        I.mdesc.clear();
        I.mdesc_ptr.assign(1, 0);
        const int nbd = I.nbd;
        int tbig = I.t0, maxnb = 0;
        for (int ti = I.t0; ti < I.t0 + I.nt; ti++)
            if (int(h.tmpl[ti].blocks.size()) > maxnb) {
                maxnb = int(h.tmpl[ti].blocks.size());
                tbig = ti;
            }
        std::vector<int32_t> first(nbd, INT32_MAX);
        if (nbd) {
            const Template &t = h.tmpl[tbig];
            for (size_t s = 0; s < t.brow.size(); s++)
                for (auto &y : t.brow[s]) first[y.first] = std::min(first[y.first], int32_t(s));
        }
        I.bperm.resize(nbd);
        for (int b = 0; b < nbd; b++) I.bperm[b] = b;
        std::stable_sort(I.bperm.begin(), I.bperm.end(), [&](int32_t x, int32_t y) { return first[x] < first[y]; });
        std::vector<int32_t> tpos(nbd);
        for (int q = 0; q < nbd; q++) tpos[I.bperm[q]] = q;
        const int nmt = (nbd + kMT - 1) / kMT;
        I.npair = nmt * (nmt + 1) / 2;
        std::vector<std::vector<MItem>> pairs(size_t(I.npair) * I.nt);   // [pair][template]
        for (int q = 0; q < I.nt; q++) {
            const Template &t = h.tmpl[I.t0 + q];
            for (size_t s = 0; s < t.brow.size(); s++) {
                if (t.brow[s].empty()) continue;
                std::vector<int> tiles;
                for (auto &y : t.brow[s]) tiles.push_back(tpos[y.first] / kMT);
                std::sort(tiles.begin(), tiles.end());
                tiles.erase(std::unique(tiles.begin(), tiles.end()), tiles.end());
                const int r = t.srp[s + 1] - t.srp[s], w = t.sup[s + 1] - t.sup[s];
                if (r > INT16_MAX) return NCL_ERR_ARG;
                for (int TI : tiles)
                    for (int TJ : tiles) {
                        if (TJ > TI) break;
                        MItem it{};
                        it.tmpl = I.t0 + q;
                        it.poff = t.panel_off[s];
                        it.r = r;
                        it.w = w;
                        for (int u = 0; u < kMT; u++) it.ri[u] = it.rj[u] = -1;
                        for (auto &y : t.brow[s]) {
                            const int tp = tpos[y.first];
                            if (tp / kMT == TI) it.ri[tp % kMT] = int16_t(y.second);
                            if (tp / kMT == TJ) it.rj[tp % kMT] = int16_t(y.second);
                        }
                        pairs[(size_t(TI) * (TI + 1) / 2 + TJ) * I.nt + q].push_back(it);
                    }
            }
        }
        const int nch = (maxnb + kMC - 1) / kMC;
        for (int pq = 0; pq < I.npair; pq++) {
            std::vector<std::pair<int32_t, int32_t>> trange;      // per template: item range
            for (int q = 0; q < I.nt; q++) {
                const int32_t ib = int32_t(I.mitems.size());
                const auto &v = pairs[size_t(pq) * I.nt + q];
                I.mitems.insert(I.mitems.end(), v.begin(), v.end());
                trange.push_back({ib, int32_t(I.mitems.size())});
            }
            if (I.mitems.size() > size_t(INT32_MAX)) return NCL_ERR_ARG;
            for (int c = 0; c < nch; c++)
                for (int q = 0; q < I.nt; q++) {
                    const int nb = int(h.tmpl[I.t0 + q].blocks.size()), cs = std::min(kMC, nb - kMC * c);
                    if (cs <= 0) continue;
                    int32_t ib = trange[q].first;
                    int64_t cost = 0;
                    for (int32_t it = trange[q].first; it < trange[q].second; it++) {
                        const int64_t ci = (int64_t(I.mitems[it].w) * cs + 3) / 4 + kMItemCost;
                        if (it > ib && cost + ci > kMSlice) {
                            I.mdesc.push_back(MDesc{pq, c, ib, it});
                            ib = it;
                            cost = 0;
                        }
                        cost += ci;
                    }
                    if (ib < trange[q].second) I.mdesc.push_back(MDesc{pq, c, ib, trange[q].second});
                }
            if (I.mdesc.size() > size_t(INT32_MAX)) return NCL_ERR_ARG;
            I.mdesc_ptr.push_back(int32_t(I.mdesc.size()));
        }
    }
    return NCL_OK;
}

}  // namespace ncl
