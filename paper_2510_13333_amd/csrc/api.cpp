// C ABI of libnclkkt: handle life cycle, workspace binding, launches and the
// host-side views of the symbolic result.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "kernels.h"

using ncl::Handle;
using ncl::Template;

namespace {

constexpr size_t kAlign = 256;

void kernel_model(Handle &h);

int relax_params(const ncl_analyze_opts *o, int &maxw, int &znum, int &zden) {
    maxw = 16;
    znum = 1;
    zden = 4;
    if (o) {
        if (o->relax_maxw) maxw = o->relax_maxw;
        if (o->relax_zden) { znum = o->relax_znum; zden = o->relax_zden; }
        if (maxw < 1 || zden <= 0 || znum < 0) return NCL_ERR_ARG;
        if (o->ordering != NCL_ORDER_MD && o->ordering != NCL_ORDER_USER) return NCL_ERR_ARG;
        if (o->ordering == NCL_ORDER_USER && !o->user_perm) return NCL_ERR_ARG;
    }
    return NCL_OK;
}

// The local elimination order of template t from a caller's permutation of
// its instance (new -> layout index, instance-local), checked to respect
// the block structure: every block of the template takes the same local
// order over its own columns, and the instance's border maps to itself.
int user_order(const Handle &h, const Template &t, const int32_t *perm, std::vector<int32_t> &order) {
    const ncl::Inst &I = h.inst[t.inst];
    const int n = t.n;
    order.assign(n, -1);
    for (size_t q = 0; q < t.blocks.size(); q++) {
        const int b = t.blocks[q];
        const int64_t o = h.block_col0[b] - I.col0;
        for (int j = 0; j < n; j++) {
            const int64_t v = int64_t(perm[o + j]) - o;
            if (v < 0 || v >= n) return NCL_ERR_ARG;
            if (q == 0) order[j] = int32_t(v);
            else if (order[j] != v) return NCL_ERR_ARG;
        }
    }
    const int64_t bs = I.bstart - I.col0;
    for (int j = 0; j < I.nbd; j++)
        if (perm[bs + j] != bs + j) return NCL_ERR_ARG;
    return NCL_OK;
}

// opts: nullptr (defaults), one set for every instance (nopts == 1) or one per instance.
int finish_analyze(Handle &h, const ncl_analyze_opts *opts, int nopts) {
    const int ninst = int(h.inst.size());
    auto opts_of = [&](int i) -> const ncl_analyze_opts * {
        if (!opts) return nullptr;
        return nopts == 1 ? opts : opts + i;
    };
    for (const auto &I : h.inst)
        if (I.nbd > NCL_MAX_BORDER) return NCL_ERR_ARG;
    h.block_bl.assign(h.nblk, 0);
    for (auto &t : h.tmpl) t.blocks.clear();
    for (int b = 0; b < h.nblk; b++) {
        Template &t = h.tmpl[h.block_tmpl[b]];
        h.block_bl[b] = int32_t(t.blocks.size());
        t.blocks.push_back(b);
    }
    for (auto &t : h.tmpl) {
        int maxw, znum, zden;
        int rc = relax_params(opts_of(t.inst), maxw, znum, zden);
        if (rc) return rc;
        const ncl_analyze_opts *o = opts_of(t.inst);
        std::vector<int32_t> order;
        if (o && o->ordering == NCL_ORDER_USER) {
            rc = user_order(h, t, o->user_perm, order);
            if (rc) return rc;
        }
        rc = ncl::analyze_template(t, h.inst[t.inst].nbd, maxw, znum, zden, order.empty() ? nullptr : order.data());
        if (rc) return rc;
        rc = ncl::build_template_schedule(t, h.inst[t.inst].nbd);
        if (rc) return rc;
    }
    for (int i = 0; i < ninst; i++) {
        int maxw, znum, zden;
        int rc = relax_params(opts_of(i), maxw, znum, zden);
        if (!rc) rc = ncl::analyze_border(h, h.inst[i], maxw, znum, zden);
        if (rc) return rc;
        // full symmetric rows of K_bb (residual of the border rows)
        ncl::Inst &I = h.inst[i];
        std::vector<std::vector<int32_t>> br(I.nbd);
        for (int c = 0; c < I.nbd; c++)
            for (int64_t p = I.bcolptr[c]; p < I.bcolptr[c + 1]; p++) {
                const int32_t r = I.browind[p];
                br[r].push_back(int32_t(p));
                br[r].push_back(c);
                if (r != c) {
                    br[c].push_back(int32_t(p));
                    br[c].push_back(r);
                }
            }
        I.kbr_ptr.assign(1, 0);
        I.kbr_ent.clear();
        for (auto &r : br) {
            I.kbr_ent.insert(I.kbr_ent.end(), r.begin(), r.end());
            I.kbr_ptr.push_back(int32_t(I.kbr_ent.size() / 2));
        }
    }
    int rc = ncl::build_schedule(h);
    if (rc) return rc;
    h.nnzL = 0;
    h.nsuper = 0;
    h.npanel = 0;
    for (int b = 0; b < h.nblk; b++) {
        const Template &t = h.tmpl[h.block_tmpl[b]];
        h.nnzL += t.lp[t.n];
        h.nsuper += int64_t(t.sup.size()) - 1;
        h.npanel += int64_t(t.sri.size());
    }
    h.nbd_tot = h.nbb_tot = h.npk_tot = h.sp_tot = h.cp_tot = h.gp_tot = h.mw_tot = h.pe_tot = 0;
    h.max_nbd = 0;
    for (auto &I : h.inst) {
        I.kbb0 = h.nbb_tot;
        I.sbb0 = h.npk_tot;
        I.bd0 = h.nbd_tot;
        I.sp0 = h.sp_tot;
        I.cp0 = h.cp_tot;
        I.npk0 = h.npk_tot;
        I.gp0 = h.gp_tot;
        h.nbb_tot += I.nbb();
        h.npk_tot += I.npk();
        h.nbd_tot += I.nbd;
        I.mw0 = h.mw_tot;
        h.mw_tot += int64_t(I.mdesc.size());
        I.pe0 = h.pe_tot;
        h.pe_tot += int64_t(I.npair) * ncl::kMT * ncl::kMT;
        h.sp_tot += int64_t(I.mdesc.size()) * ncl::kMT * ncl::kMT;
        h.cp_tot += int64_t(I.nbd) * I.nblk;
        if (I.nbd) h.gp_tot += I.ng;
        h.max_nbd = std::max(h.max_nbd, I.nbd);
        if (!I.nbd) continue;
        h.nnzL += I.blp[I.nbd];
        h.nsuper += int64_t(I.bsup.size()) - 1;
        std::vector<int32_t> mk(I.nbd, -1);
        for (size_t s = 0; s + 1 < I.bsup.size(); s++) {
            int f = I.bsup[s], l = I.bsup[s + 1] - 1;
            h.npanel += l - f + 1;
            for (int j = f; j <= l; j++)
                for (int p = I.blp[j]; p < I.blp[j + 1]; p++)
                    if (I.bli[p] > l && mk[I.bli[p]] != int(s)) { mk[I.bli[p]] = int(s); h.npanel++; }
        }
    }
    kernel_model(h);
    return NCL_OK;
}

// Workspace layout: schedule tables first, then the numeric arrays.  The
// same walk sizes the workspace and, with a staging buffer, copies the
// tables for upload.
struct WsLayout {
    size_t off = 0;
    std::vector<uint8_t> *stage = nullptr;
    size_t take(const void *src, size_t bytes) {
        const size_t o = off;
        off = (off + bytes + kAlign - 1) & ~(kAlign - 1);
        if (stage) {
            if (stage->size() < off) stage->resize(off, 0);
            if (bytes && src) std::memcpy(stage->data() + o, src, bytes);
        }
        return o;
    }
    template <class T>
    size_t vec(const std::vector<T> &v) { return take(v.data(), v.size() * sizeof(T)); }
};

struct Plan {
    std::vector<std::vector<size_t>> toff;   // per template, in TemplDev pointer order
    std::vector<std::vector<size_t>> ioff;   // per instance: kbb_pos, border_pg, gen_c2, br_r, br_x, ..., gen_alpha
    size_t tdev = 0, bdev = 0, idev = 0, work = 0, bprim = 0, pg_col = 0, row_pq = 0, tables_end = 0;
    size_t kval = 0, lpan = 0, upan = 0, dval = 0, spart = 0, sbb = 0, lbb = 0, ybuf = 0, cpart = 0, zint = 0, sint = 0, stat = 0,
           xint = 0, bint = 0, rint = 0, rbuf = 0, epart = 0, total = 0;
};

// Workgroups of the backward-error kernels (their partial maxima).
int64_t berr_partials(const Handle &h) { return (h.rows_waves + 3) / 4 + (h.nbd_tot + 3) / 4; }

std::vector<uint8_t> col_primal(const Template &t) {
    std::vector<uint8_t> cp(t.n);
    for (int j = 0; j < t.n; j++) cp[j] = t.is_primal[t.perm[j]];
    return cp;
}

std::vector<ncl::Work> all_work(Handle &h) {
    const ncl::Schedule &S = h.sched;
    std::vector<ncl::Work> w;
    auto app = [&](const std::vector<ncl::Work> &v, size_t &off) {
        off = w.size();
        w.insert(w.end(), v.begin(), v.end());
    };
    app(S.a, h.w_a);
    app(S.b, h.w_b);
    app(S.c, h.w_c);
    app(S.f, h.w_f);
    app(S.d, h.w_d);
    app(S.sn, h.w_sn);
    app(S.sb, h.w_sb);
    app(S.bpart, h.w_bpart);
    return w;
}

// Dispatch-map tables of a single network without PV/PQ rows (empty
// otherwise): the global column of each generator's pg, and the global P and
// Q rows of every bus in every block.
void dispatch_tables(Handle &h, std::vector<int64_t> &pgc, std::vector<int64_t> &rows) {
    h.ng_disp = h.nbus_disp = 0;
    if (!h.from_network || h.inst.size() != 1 || (h.inst[0].flags & (NCL_PVPQ | NCL_AGC))) return;
    const ncl::Inst &I = h.inst[0];
    for (int b = I.blk0; b < I.blk0 + I.nblk; b++) {
        const Template &t = h.tmpl[h.block_tmpl[b]];
        std::vector<int64_t> rp, rq;
        for (int j = 0; j < t.n; j++) {
            const int64_t c = h.block_col0[b] + j;
            if (t.lkind[j] == ncl::LK_PG) pgc.push_back(c);
            if (t.lkind[j] == ncl::LK_ROWP) rp.push_back(c);
            if (t.lkind[j] == ncl::LK_ROWQ) rq.push_back(c);
        }
        if (int(rp.size()) != I.nb || int(rq.size()) != I.nb) {
            pgc.clear();
            rows.clear();
            return;
        }
        for (int i = 0; i < I.nb; i++) {
            rows.push_back(rp[i]);
            rows.push_back(rq[i]);
        }
    }
    for (int j = 0; j < std::min(I.nbd, I.ng); j++) pgc.push_back(I.bstart + j);
    if (int(pgc.size()) != I.ng) {
        pgc.clear();
        rows.clear();
        return;
    }
    h.ng_disp = I.ng;
    h.nbus_disp = I.nb;
}

Plan plan_ws(Handle &h, int64_t nrhs, std::vector<uint8_t> *stage) {
    Plan p;
    WsLayout L;
    L.stage = stage;
    p.toff.resize(h.tmpl.size());
    for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
        const Template &t = h.tmpl[ti];
        std::vector<size_t> &o = p.toff[ti];
        o.push_back(L.vec(t.blocks));
        o.push_back(L.vec(t.sup));
        o.push_back(L.vec(t.srp));
        o.push_back(L.vec(t.sri));
        o.push_back(L.vec(t.panel_off));
        o.push_back(L.vec(t.task_s));
        o.push_back(L.vec(t.task_p));
        o.push_back(L.vec(t.task_cbase));
        o.push_back(L.vec(t.ent_kpos));
        o.push_back(L.vec(t.ent_out));
        o.push_back(L.vec(t.ent_tptr));
        o.push_back(L.vec(t.terms));
        o.push_back(L.vec(t.bterm_ptr));
        o.push_back(L.vec(t.bterms));
        o.push_back(L.vec(t.bus_idx));
        o.push_back(L.vec(t.bus_slot));
        o.push_back(L.vec(t.bus_adj_ptr));
        o.push_back(L.vec(t.bus_adj));
        o.push_back(L.vec(t.br_slot));
        o.push_back(L.vec(t.br_idx));
        o.push_back(L.vec(t.gen_idx));
        o.push_back(L.vec(t.gen_slot));
        o.push_back(L.vec(t.perm));
        o.push_back(L.vec(col_primal(t)));
        o.push_back(L.vec(t.bus_gen));
        o.push_back(L.vec(t.lkind));
        o.push_back(L.vec(t.iperm));
        o.push_back(L.vec(t.rr_ptr));
        o.push_back(L.vec(t.rr_ent));
        o.push_back(L.vec(t.rb_ptr));
        o.push_back(L.vec(t.rb_ent));
        o.push_back(L.vec(t.sup_rnb));
        o.push_back(L.vec(t.col_sup));
    }
    p.tdev = L.take(nullptr, sizeof(ncl::TemplDev) * h.tmpl.size());
    p.bdev = L.take(nullptr, sizeof(ncl::BlockDev) * size_t(h.nblk));
    p.idev = L.take(nullptr, sizeof(ncl::InstDev) * h.inst.size());
    p.work = L.vec(all_work(h));
    p.ioff.resize(h.inst.size());
    // expected sign of every pivot in the order of the pivots (the blocks'
    // interleaved by template, then each instance's border), for the pivot
    // report's coalesced reads
    std::vector<uint8_t> bprim(size_t(h.dint));
    for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
        const Template &t = h.tmpl[ti];
        const std::vector<uint8_t> cp = col_primal(t);
        const int64_t nb = int64_t(t.blocks.size());
        for (int j = 0; j < t.n; j++)
            std::fill_n(bprim.begin() + (h.t_dbase[ti] + int64_t(j) * nb), nb, cp[j]);
    }
    for (size_t i = 0; i < h.inst.size(); i++) {
        const ncl::Inst &I = h.inst[i];
        p.ioff[i] = {L.vec(I.kbb_pos), L.vec(I.border_pg), L.vec(I.gen_c2), L.vec(I.br_r), L.vec(I.br_x),
                     L.vec(I.kbr_ptr), L.vec(I.kbr_ent), L.vec(I.mdesc_ptr), L.vec(I.mdesc), L.vec(I.mitems),
                     L.vec(I.bperm), L.vec(I.gen_alpha)};
        bprim.insert(bprim.end(), I.border_primal.begin(), I.border_primal.end());
    }
    p.bprim = L.vec(bprim);
    {
        std::vector<int64_t> pgc, rows;
        dispatch_tables(h, pgc, rows);
        p.pg_col = L.vec(pgc);
        p.row_pq = L.vec(rows);
    }
    p.tables_end = L.off;
    L.stage = nullptr;
    p.kval = L.take(nullptr, sizeof(double) * size_t(h.kint + h.nbb_tot));
    p.lpan = L.take(nullptr, sizeof(double) * size_t(h.lint));
    p.upan = L.take(nullptr, sizeof(double) * size_t(h.lint));
    p.dval = L.take(nullptr, sizeof(double) * size_t(h.dint + h.nbd_tot));
    p.spart = L.take(nullptr, sizeof(double) * size_t(h.sp_tot));
    p.sbb = L.take(nullptr, sizeof(double) * size_t(h.npk_tot));
    p.lbb = L.take(nullptr, sizeof(double) * size_t(h.npk_tot));
    p.ybuf = L.take(nullptr, sizeof(double) * size_t(h.dint + h.nbd_tot) * size_t(nrhs));
    p.cpart = L.take(nullptr, sizeof(double) * size_t(nrhs) * size_t(h.cp_tot));
    p.zint = L.take(nullptr, sizeof(double) * size_t(h.dint + h.nbd_tot));
    p.sint = L.take(nullptr, sizeof(double) * size_t(h.dint + h.nbd_tot));
    p.xint = L.take(nullptr, sizeof(double) * size_t(h.dint + h.nbd_tot));
    p.bint = L.take(nullptr, sizeof(double) * size_t(h.dint + h.nbd_tot));
    p.rint = L.take(nullptr, sizeof(double) * size_t(h.dint + h.nbd_tot));
    p.rbuf = L.take(nullptr, sizeof(double) * size_t(h.N));
    p.epart = L.take(nullptr, sizeof(double) * 8 * size_t(berr_partials(h)));
    p.stat = L.take(nullptr, sizeof(int64_t) * ncl::kStatWords * ncl::kStatStride);
    p.total = L.off;
    return p;
}

ncl::DevArgs dev_args(const Handle &h) {
    ncl::DevArgs a{};
    a.tmpls = h.d.tmpl;
    a.blks = h.d.blk;
    a.insts = h.d.inst;
    a.ntmpl = int(h.tmpl.size());
    a.nblk = h.nblk;
    a.ninst = int(h.inst.size());
    a.max_nbd = h.max_nbd;
    a.N = h.N;
    a.kint = h.kint;
    a.dint = h.dint;
    a.nbd_tot = h.nbd_tot;
    a.nbb_tot = h.nbb_tot;
    a.npk_tot = h.npk_tot;
    a.asm_threads = h.asm_threads;
    a.asm_wthreads = h.asm_wthreads;
    a.gp_tot = h.gp_tot;
    a.mw_tot = h.mw_tot;
    a.pe_tot = h.pe_tot;
    a.tiles = h.tiles;
    a.zint = h.d.zint;
    a.sint = h.d.sint;
    a.kval = h.d.kval;
    a.lpan = h.d.lpan;
    a.upan = h.d.upan;
    a.dval = h.d.dval;
    a.spart = h.d.spart;
    a.sbb = h.d.sbb;
    a.lbb = h.d.lbb;
    a.ybuf = h.d.ybuf;
    a.cpart = h.d.cpart;
    a.stat = h.d.stat;
    a.bprim = h.d.bprim;
    a.rows_waves = h.rows_waves;
    a.nprimal = h.nprimal;
    a.xint = h.d.xint;
    a.bint = h.d.bint;
    a.rint = h.d.rint;
    a.rbuf = h.d.rbuf;
    a.epart = h.d.epart;
    a.rows_wg = int((h.rows_waves + 3) / 4);
    a.pg_col = h.d.pg_col;
    a.row_pq = h.d.row_pq;
    a.ng_disp = h.ng_disp;
    a.nbus_disp = h.nbus_disp;
    return a;
}

// The largest border of an instance too large for the register factor (0: none).

// Launches and algorithmic bytes per step of every kernel kind: each
// distinct element a launch reads or writes counts once per launch.
// The largest border over kBorderRegMax rows (0 if none): the blocked path.
int big_border(const Handle &h) {
    int m = 0;
    for (const ncl::Inst &I : h.inst)
        if (I.nbd > ncl::kBorderRegMax && I.nbd > m) m = I.nbd;
    return m;
}

void kernel_model(Handle &h) {
    constexpr int64_t D = sizeof(double);
    h.km_launch.assign(NCL_K_COUNT, 0);
    h.km_bytes.assign(NCL_K_COUNT, 0);
    auto &L = h.km_launch;
    auto &B = h.km_bytes;
    const ncl::Schedule &S = h.sched;
    auto levels = [&](int kind, const std::vector<int32_t> &ptr) {
        for (size_t l = 0; l + 1 < ptr.size(); l++)
            if (ptr[l + 1] > ptr[l]) L[kind]++;
    };
    levels(NCL_K_FAC_GATHER, S.a_ptr);
    levels(NCL_K_FAC_DIAG, S.b_ptr);
    levels(NCL_K_FAC_ROWS, S.c_ptr);
    levels(NCL_K_SOL_FWD_GATHER, S.f_ptr);
    levels(NCL_K_SOL_FWD_DIAG, S.d_ptr);
    levels(NCL_K_SOL_BWD, S.sn_ptr);
    L[NCL_K_SOL_BWD_BORDER] = S.sb.empty() ? 0 : 1;
    for (const Template &t : h.tmpl) {
        const int64_t nb = int64_t(t.blocks.size());
        const int n = t.n;
        std::vector<int32_t> mp(size_t(t.panel_off.back()), -1), mk(size_t(n) + h.max_nbd + 1, -1);
        int stamp = 0;
        std::vector<int32_t> mu(size_t(t.panel_off.back()), -1);
        // factor updates read U[a] L[c]: distinct U and L elements
        auto uniq_ul = [&](const ncl::Term &q, int64_t &uu, int64_t &ul) {
            if (mu[q.a] != stamp) { mu[q.a] = stamp; uu++; }
            if (mp[q.c] != stamp) { mp[q.c] = stamp; ul++; }
        };
        for (int l = 0; l < t.nlev; l++) {
            // factor: gather (A), diagonal blocks and width-1 pivots (B), rows (C)
            int64_t ents = 0, kr = 0, up = 0, uk = 0, bdiag = 0, rows = 0;
            stamp++;
            int last_s = -1;
            for (int32_t k : t.lev_tasks[l]) {
                const int s = t.task_s[k], p = t.task_p[k];
                const int w = t.sup[s + 1] - t.sup[s];
                const int cend = p < w ? p + 1 : w;
                for (int c = 0; c < cend; c++) {
                    const int e = t.task_cbase[k] + c;
                    ents++;
                    if (t.ent_kpos[e] >= 0) kr++;
                    for (int q = t.ent_tptr[e]; q < t.ent_tptr[e + 1]; q++) uniq_ul(t.terms[q], up, uk);
                }
                if (w == 1) bdiag += p > 0 ? 3 : 2;              // entry read, L and U (or d) written
                else if (p >= w) rows += 3 * w;
                if (w > 1 && s != last_s) {
                    bdiag += int64_t(w) * (w + 1) + w;            // diagonal block read and written, pivots
                    rows += int64_t(w) * (w - 1) / 2 + w;         // the block and pivots the rows read
                }
                last_s = s;
            }
            B[NCL_K_FAC_GATHER] += nb * D * (ents + kr + up + uk);
            B[NCL_K_FAC_DIAG] += nb * D * bdiag;
            B[NCL_K_FAC_ROWS] += nb * D * rows;
            // forward solve: gathers of the diagonal rows (F), diagonal solves (D)
            int64_t fr = 0, fup = 0, fuy = 0, dd = 0;
            stamp++;
            last_s = -1;
            for (int32_t k : t.lev_tasks[l]) {
                const int s = t.task_s[k], p = t.task_p[k];
                const int w = t.sup[s + 1] - t.sup[s];
                if (p >= w) continue;
                const int e = t.task_cbase[k] + p;
                if (t.ent_tptr[e + 1] > t.ent_tptr[e]) {
                    fr += 2;
                    for (int q = t.ent_tptr[e]; q < t.ent_tptr[e + 1]; q++) {
                        const ncl::Term &tm = t.terms[q];
                        if (mp[tm.a] != stamp) { mp[tm.a] = stamp; fup++; }
                        if (mk[tm.k] != stamp) { mk[tm.k] = stamp; fuy++; }
                    }
                }
                if (w > 1 && s != last_s) dd += int64_t(w) * (w - 1) / 2 + 2 * w - 1;
                last_s = s;
            }
            B[NCL_K_SOL_FWD_GATHER] += nb * D * (fr + fup + fuy);
            B[NCL_K_SOL_FWD_DIAG] += nb * D * dd;
            // backward, per supernode of the level: its diagonal block and the
            // block rows below it read once, its y read and written, the
            // solution of the distinct block rows below read
            int64_t sb = 0, rowsx = 0;
            stamp++;
            last_s = -1;
            for (int32_t k : t.lev_tasks[l]) {
                const int s = t.task_s[k];
                if (s == last_s) continue;
                last_s = s;
                const int w = t.sup[s + 1] - t.sup[s], rnb = t.sup_rnb[s];
                sb += int64_t(w) * (w - 1) / 2 + int64_t(rnb - w) * w + 2 * w;
                for (int i = t.srp[s] + w; i < t.srp[s] + rnb; i++) {
                    const int row = t.sri[i];
                    if (mk[row] != stamp) { mk[row] = stamp; rowsx++; }
                }
            }
            B[NCL_K_SOL_BWD] += nb * D * (sb + rowsx);
        }
        // backward border step: every column's y and d read and y written,
        // the border rows of every panel read
        {
            int64_t bb = 0;
            const int ns = int(t.sup.size()) - 1;
            for (int s = 0; s < ns; s++) {
                const int w = t.sup[s + 1] - t.sup[s];
                bb += 3 * int64_t(w) + int64_t(t.srp[s + 1] - t.srp[s] - t.sup_rnb[s]) * w;
            }
            B[NCL_K_SOL_BWD_BORDER] += nb * D * bb;
        }
        const ncl::Inst &I = h.inst[t.inst];
        if (I.nbd) {
            // border Schur products: the tile rows each item holds, over its
            // columns and the template's blocks
            int64_t el = 0;
            for (const ncl::MItem &it : I.mitems) {
                if (it.tmpl != int(&t - h.tmpl.data())) continue;
                int cnt = 0;
                for (int q = 0; q < ncl::kMT; q++) cnt += (it.ri[q] >= 0) + (it.rj[q] >= 0);
                el += int64_t(it.w) * cnt;
            }
            B[NCL_K_BORDER_SCHUR] += nb * D * el;
            int64_t up = 0, uk = 0;
            up = uk = 0;
            stamp++;
            for (const ncl::Term &q : t.bterms) {
                if (mp[q.a] != stamp) { mp[q.a] = stamp; up++; }
                if (mk[q.k] != stamp) { mk[q.k] = stamp; uk++; }
            }
            B[NCL_K_SOL_BPART] += nb * D * (I.nbd + up + uk);
        }
    }
    L[NCL_K_INTERLEAVE] = L[NCL_K_ASSEMBLE] = h.from_network ? 1 : 0;
    B[NCL_K_INTERLEAVE] = h.from_network ? D * 4 * (h.dint + h.nbd_tot) : 0;
    B[NCL_K_ASSEMBLE] = h.from_network ? D * (2 * h.N + h.kint + h.nbb_tot) : 0;
    L[NCL_K_STATUS_INIT] = 1;
    B[NCL_K_STATUS_INIT] = D * 6;
    L[NCL_K_STATUS] = 1;
    B[NCL_K_STATUS] = (D + 1) * (h.dint + h.nbd_tot);   // each pivot and its expected sign
    L[NCL_K_SOL_LOAD] = L[NCL_K_SOL_STORE] = 1;
    B[NCL_K_SOL_LOAD] = B[NCL_K_SOL_STORE] = D * 2 * h.dint;
    if (h.nbd_tot) {
        L[NCL_K_BORDER_SCHUR] = L[NCL_K_BORDER_SUM] = 1;
        L[NCL_K_SOL_BPART] = L[NCL_K_SOL_BORDER] = 1;
        B[NCL_K_BORDER_SCHUR] += D * h.sp_tot;     // the partial tiles written
        B[NCL_K_BORDER_SUM] = D * (h.sp_tot + h.nbb_tot + h.npk_tot);
        const int bb = big_border(h);
        L[NCL_K_BORDER_FACTOR] = 1 + (bb + ncl::kBorderBlock - 1) / ncl::kBorderBlock;
        B[NCL_K_BORDER_FACTOR] = 0;
        for (const ncl::Inst &I : h.inst) {
            const int64_t n = I.nbd;
            if (n <= ncl::kBorderRegMax) {
                B[NCL_K_BORDER_FACTOR] += D * (n * (n + 1) + n);     // the packed matrix read, L written, pivots
                continue;
            }
            // blocked: per column block (bs x bs tiles) every trailing tile
            // reads the block's factor and the block column rows of its two
            // tile rows (one on the diagonal), reads and writes itself; the
            // diagonal tiles write L; the diagonal blocks and pivots once
            const int64_t bs = ncl::kBorderBlock, nb = (n + bs - 1) / bs, t2 = bs * bs;
            for (int64_t b = 0; b < nb; b++) {
                const int64_t rem = nb - b - 1, tiles = rem * (rem + 1) / 2;
                B[NCL_K_BORDER_FACTOR] += D * (t2 * tiles + t2 * (2 * tiles - rem) + 2 * t2 * tiles + t2 * rem + t2 + bs);
            }
        }
        B[NCL_K_SOL_BORDER] = D * (h.cp_tot + h.npk_tot + 4 * h.nbd_tot);
    } else {
        B[NCL_K_BORDER_SCHUR] = B[NCL_K_SOL_BPART] = 0;
    }
}

// Whether a launch of this kind with these arguments runs a kernel.
bool nonempty(int kind, const ncl::DevArgs &a, const ncl::LaunchArgs &l) {
    switch (kind) {
        case NCL_K_ASSEMBLE: return a.asm_threads + a.gp_tot > 0;
        case NCL_K_VALUES: return a.kint + a.nbb_tot > 0;
        case NCL_K_BORDER_SUM: return a.pe_tot > 0;
        case NCL_K_BORDER_SCHUR: return a.mw_tot > 0;
        case NCL_K_BORDER_FACTOR:
        case NCL_K_SOL_BORDER: return a.max_nbd > 0;
        case NCL_K_STATUS_INIT:
        case NCL_K_STATUS: return true;
        case NCL_K_SOL_LOAD:
        case NCL_K_SOL_STORE: return a.dint > 0;
        case NCL_K_RESIDUAL: return a.asm_threads + a.gp_tot > 0;
        case NCL_K_INTERLEAVE: return a.tiles + a.nbd_tot > 0;
        case NCL_K_MAX_STEP: return true;
        case NCL_K_BERR_ROWS: return a.rows_waves > 0;
        case NCL_K_BERR_BORDER: return a.nbd_tot > 0;
        case NCL_K_BERR_FINAL: return true;
        default: return l.nw > 0;
    }
}

// Launch one kernel; bracket it with events when its kind is being profiled.
hipError_t run(Handle &h, int kind, const ncl::DevArgs &a, const ncl::LaunchArgs &l, hipStream_t st) {
    if (kind != h.prof_kind || !nonempty(kind, a, l)) return ncl::launch(kind, a, l, st);
    if (h.prof_seen++ % h.prof_stride != 0) return ncl::launch(kind, a, l, st);
    if (2 * h.ev_used + 2 > h.ev.size()) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return hipErrorOutOfMemory;
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return hipErrorOutOfMemory;
        }
        h.ev.push_back(e0);
        h.ev.push_back(e1);
    }
    hipEvent_t e0 = static_cast<hipEvent_t>(h.ev[2 * h.ev_used]), e1 = static_cast<hipEvent_t>(h.ev[2 * h.ev_used + 1]);
    hipError_t e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = ncl::launch(kind, a, l, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) h.ev_used++;
    return e;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? NCL_OK : NCL_ERR_HIP; }

}  // namespace

extern "C" {

const char *ncl_status_string(int s) {
    switch (s) {
        case NCL_OK: return "ok";
        case NCL_ERR_ARG: return "invalid argument";
        case NCL_ERR_ALLOC: return "host allocation failed";
        case NCL_ERR_HIP: return "HIP runtime error";
        case NCL_ERR_STATE: return "call out of order";
        case NCL_ERR_ZERO_PIVOT: return "zero pivot";
        case NCL_ERR_INERTIA: return "pivot of the wrong sign (inertia)";
        case NCL_ERR_NONFINITE: return "non-finite pivot";
        case NCL_ERR_NOT_CONVERGED: return "Newton method did not converge";
        default: return "unknown status";
    }
}

int ncl_kkt_analyze(const ncl_network *net, const ncl_analyze_opts *opts, ncl_kkt **out) {
    if (!out) return NCL_ERR_ARG;
    *out = nullptr;
    ncl_kkt *k = new (std::nothrow) ncl_kkt;
    if (!k) return NCL_ERR_ALLOC;
    try {
        std::string err;
        int rc = ncl::build_network_model(net, k->h, err);
        if (!rc) rc = finish_analyze(k->h, opts, opts ? 1 : 0);
        if (rc) { delete k; return rc; }
    } catch (const std::bad_alloc &) {
        delete k;
        return NCL_ERR_ALLOC;
    }
    *out = k;
    return NCL_OK;
}

int ncl_kkt_analyze_pattern(int64_t N, int32_t nblk, const int64_t *block_off, const int64_t *colptr,
                            const int32_t *rowind, const uint8_t *is_primal, const ncl_analyze_opts *opts,
                            ncl_kkt **out) {
    if (!out) return NCL_ERR_ARG;
    *out = nullptr;
    ncl_kkt *k = new (std::nothrow) ncl_kkt;
    if (!k) return NCL_ERR_ALLOC;
    try {
        std::string err;
        int rc = ncl::build_pattern_model(N, nblk, block_off, colptr, rowind, is_primal, k->h, err);
        if (!rc) rc = finish_analyze(k->h, opts, opts ? 1 : 0);
        if (rc) { delete k; return rc; }
    } catch (const std::bad_alloc &) {
        delete k;
        return NCL_ERR_ALLOC;
    }
    *out = k;
    return NCL_OK;
}

int ncl_kkt_analyze_batch(const ncl_network *nets, int32_t count, const ncl_analyze_opts *opts, int32_t nopts,
                          ncl_kkt **out) {
    if (!out || !nets || count < 1 || (opts && nopts != 1 && nopts != count) || (!opts && nopts != 0))
        return NCL_ERR_ARG;
    *out = nullptr;
    ncl_kkt *k = new (std::nothrow) ncl_kkt;
    if (!k) return NCL_ERR_ALLOC;
    try {
        std::string err;
        int rc = NCL_OK;
        for (int i = 0; i < count && !rc; i++) rc = ncl::build_network_model(nets + i, k->h, err);
        if (!rc && k->h.tmpl.size() > 32767) rc = NCL_ERR_ARG;
        if (!rc) rc = finish_analyze(k->h, opts, nopts);
        if (rc) { delete k; return rc; }
    } catch (const std::bad_alloc &) {
        delete k;
        return NCL_ERR_ALLOC;
    }
    *out = k;
    return NCL_OK;
}

int ncl_kkt_instances(const ncl_kkt *k, int32_t *count) {
    if (!k || !count) return NCL_ERR_ARG;
    *count = int32_t(k->h.inst.size());
    return NCL_OK;
}

int ncl_kkt_instance(const ncl_kkt *k, int32_t i, int64_t *col0, int64_t *n, int64_t *nprimal, int32_t *nblk,
                     int32_t *nbd) {
    if (!k || i < 0 || i >= int32_t(k->h.inst.size())) return NCL_ERR_ARG;
    const ncl::Inst &I = k->h.inst[i];
    if (col0) *col0 = I.col0;
    if (n) *n = I.N;
    if (nprimal) *nprimal = I.nprimal;
    if (nblk) *nblk = I.nblk;
    if (nbd) *nbd = I.nbd;
    return NCL_OK;
}

void ncl_kkt_destroy(ncl_kkt *k) { delete k; }

int ncl_kkt_dims(const ncl_kkt *k, int64_t *N, int64_t *nprimal, int64_t *nnzK, int64_t *nnzL, int64_t *nsuper,
                 int64_t *npanel) {
    if (!k) return NCL_ERR_ARG;
    const Handle &h = k->h;
    if (N) *N = h.N;
    if (nprimal) *nprimal = h.nprimal;
    if (nnzK) *nnzK = h.nnzK;
    if (nnzL) *nnzL = h.nnzL;
    if (nsuper) *nsuper = h.nsuper;
    if (npanel) *npanel = h.npanel;
    return NCL_OK;
}

int ncl_kkt_symbolic(const ncl_kkt *k, int32_t *perm, int32_t *etree, int64_t *colcount, int64_t *super_ptr,
                     int64_t *lcolptr, int32_t *lrowind, int64_t *srowptr, int32_t *srowind) {
    if (!k) return NCL_ERR_ARG;
    const Handle &h = k->h;
    int64_t lq = 0, sq = 0, pq = 0;
    if (lcolptr) lcolptr[0] = 0;
    if (srowptr) srowptr[0] = 0;
    for (const ncl::Inst &I : h.inst) {
        const int64_t bstart = I.bstart;
        for (int b = I.blk0; b < I.blk0 + I.nblk; b++) {
            const Template &t = h.tmpl[h.block_tmpl[b]];
            const int64_t o = h.block_col0[b];
            auto gmap = [&](int32_t i) -> int32_t { return int32_t(i < t.n ? o + i : bstart + (i - t.n)); };
            for (int j = 0; j < t.n; j++) {
                if (perm) perm[o + j] = int32_t(o + t.perm[j]);
                if (colcount) colcount[o + j] = t.colcount[j];
                if (etree) {
                    int32_t par = -1;
                    if (t.parent[j] >= 0) par = int32_t(o + t.parent[j]);
                    else if (t.lp[j + 1] > t.lp[j]) par = gmap(t.li[t.lp[j]]);
                    etree[o + j] = par;
                }
                for (int p = t.lp[j]; p < t.lp[j + 1]; p++) {
                    if (lrowind) lrowind[lq] = gmap(t.li[p]);
                    lq++;
                }
                if (lcolptr) lcolptr[o + j + 1] = lq;
            }
            const int ns = int(t.sup.size()) - 1;
            for (int s = 0; s < ns; s++) {
                if (super_ptr) super_ptr[sq] = o + t.sup[s];
                for (int p = t.srp[s]; p < t.srp[s + 1]; p++) {
                    if (srowind) srowind[pq] = gmap(t.sri[p]);
                    pq++;
                }
                sq++;
                if (srowptr) srowptr[sq] = pq;
            }
        }
        std::vector<int32_t> mk(I.nbd, -1), buf;
        for (int j = 0; j < I.nbd; j++) {
            const int64_t g = bstart + j;
            if (perm) perm[g] = int32_t(g);
            if (colcount) colcount[g] = I.bcolcount[j];
            if (etree) etree[g] = I.bparent[j] >= 0 ? int32_t(bstart + I.bparent[j]) : -1;
            for (int p = I.blp[j]; p < I.blp[j + 1]; p++) {
                if (lrowind) lrowind[lq] = int32_t(bstart + I.bli[p]);
                lq++;
            }
            if (lcolptr) lcolptr[g + 1] = lq;
        }
        for (size_t s = 0; s + 1 < I.bsup.size(); s++) {
            const int f = I.bsup[s], l = I.bsup[s + 1] - 1;
            if (super_ptr) super_ptr[sq] = bstart + f;
            buf.clear();
            for (int j = f; j <= l; j++) buf.push_back(j);
            size_t c0 = buf.size();
            for (int j = f; j <= l; j++)
                for (int p = I.blp[j]; p < I.blp[j + 1]; p++)
                    if (I.bli[p] > l && mk[I.bli[p]] != int(s)) { mk[I.bli[p]] = int(s); buf.push_back(I.bli[p]); }
            std::sort(buf.begin() + c0, buf.end());
            for (int32_t r : buf) {
                if (srowind) srowind[pq] = int32_t(bstart + r);
                pq++;
            }
            sq++;
            if (srowptr) srowptr[sq] = pq;
        }
    }
    if (super_ptr) super_ptr[sq] = h.N;
    return NCL_OK;
}

int ncl_kkt_pattern(const ncl_kkt *k, int64_t *colptr, int32_t *rowind) {
    if (!k || !colptr || !rowind) return NCL_ERR_ARG;
    const Handle &h = k->h;
    colptr[0] = 0;
    for (const ncl::Inst &I : h.inst) {
        const int64_t bstart = I.bstart;
        for (int b = I.blk0; b < I.blk0 + I.nblk; b++) {
            const Template &t = h.tmpl[h.block_tmpl[b]];
            const int64_t o = h.block_col0[b];
            for (int c = 0; c < t.n; c++) {
                colptr[o + c + 1] = h.kbase[b] + t.colptr[c + 1];
                for (int64_t p = t.colptr[c]; p < t.colptr[c + 1]; p++) {
                    int32_t r = t.rowind[p];
                    rowind[h.kbase[b] + p] = int32_t(r < t.n ? o + r : bstart + (r - t.n));
                }
            }
        }
        for (int c = 0; c < I.nbd; c++) {
            colptr[bstart + c + 1] = I.kcsc_border + I.bcolptr[c + 1];
            for (int64_t p = I.bcolptr[c]; p < I.bcolptr[c + 1]; p++)
                rowind[I.kcsc_border + p] = int32_t(bstart + I.browind[p]);
        }
    }
    return NCL_OK;
}

int ncl_kkt_workspace_bytes(const ncl_kkt *k, int32_t nrhs_max, size_t *bytes) {
    if (!k || !bytes || nrhs_max < 1) return NCL_ERR_ARG;
    *bytes = plan_ws(const_cast<Handle &>(k->h), nrhs_max, nullptr).total;
    return NCL_OK;
}

int ncl_kkt_bind_workspace(ncl_kkt *k, void *dptr, size_t bytes, int32_t nrhs_max, void *stream) {
    if (!k || !dptr || nrhs_max < 1 || (reinterpret_cast<uintptr_t>(dptr) & (kAlign - 1))) return NCL_ERR_ARG;
    Handle &h = k->h;
    std::vector<uint8_t> buf;
    Plan p = plan_ws(h, nrhs_max, &buf);
    if (bytes < p.total) return NCL_ERR_ARG;
    buf.resize(p.tables_end, 0);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *base = static_cast<uint8_t *>(dptr);
    std::vector<ncl::TemplDev> tdev(h.tmpl.size());
    for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
        const Template &t = h.tmpl[ti];
        const std::vector<size_t> &o = p.toff[ti];
        ncl::TemplDev &d = tdev[ti];
        auto at = [&](int q) { return base + o[q]; };
        d.n = t.n;
        d.nsup = int32_t(t.sup.size()) - 1;
        d.nblk = int32_t(t.blocks.size());
        const ncl::Inst &I = h.inst[t.inst];
        d.nbd = I.nbd;
        d.inst = t.inst;
        d.nbus = I.nb;
        d.ngen = I.ng;
        d.abase = h.t_abase[ti];
        d.awbase = h.t_awbase[ti];
        d.tile0 = h.t_tile0[ti];
        d.bd0 = I.bd0;
        d.br_r = reinterpret_cast<const double *>(base + p.ioff[t.inst][3]);
        d.br_x = reinterpret_cast<const double *>(base + p.ioff[t.inst][4]);
        d.gen_c2 = reinterpret_cast<const double *>(base + p.ioff[t.inst][2]);
        d.gen_alpha = reinterpret_cast<const double *>(base + p.ioff[t.inst][11]);
        d.kbase = h.t_kbase[ti];
        d.lbase = h.t_lbase[ti];
        d.dbase = h.t_dbase[ti];
        d.nnz = int32_t(t.colptr[t.n]);
        d.pvpq_rows = t.pvpq_rows;
        d.has_pg_local = t.pg_local;
        d.agc_rows = t.agc_rows;
        d.blocks = reinterpret_cast<const int32_t *>(at(0));
        d.sup_first = reinterpret_cast<const int32_t *>(at(1));
        d.sup_rowptr = reinterpret_cast<const int32_t *>(at(2));
        d.sup_rows = reinterpret_cast<const int32_t *>(at(3));
        d.panel_off = reinterpret_cast<const int32_t *>(at(4));
        d.task_s = reinterpret_cast<const int32_t *>(at(5));
        d.task_p = reinterpret_cast<const int32_t *>(at(6));
        d.task_cbase = reinterpret_cast<const int32_t *>(at(7));
        d.ent_kpos = reinterpret_cast<const int32_t *>(at(8));
        d.ent_out = reinterpret_cast<const int32_t *>(at(9));
        d.ent_tptr = reinterpret_cast<const int32_t *>(at(10));
        d.terms = reinterpret_cast<const ncl::Term *>(at(11));
        d.bterm_ptr = reinterpret_cast<const int32_t *>(at(12));
        d.bterms = reinterpret_cast<const ncl::Term *>(at(13));
        d.bus_idx = reinterpret_cast<const int32_t *>(at(14));
        d.bus_slot = reinterpret_cast<const int32_t *>(at(15));
        d.bus_adj_ptr = reinterpret_cast<const int32_t *>(at(16));
        d.bus_adj = reinterpret_cast<const int32_t *>(at(17));
        d.br_slot = reinterpret_cast<const int32_t *>(at(18));
        d.br_idx = reinterpret_cast<const int32_t *>(at(19));
        d.gen_idx = reinterpret_cast<const int32_t *>(at(20));
        d.gen_slot = reinterpret_cast<const int32_t *>(at(21));
        d.perm = reinterpret_cast<const int32_t *>(at(22));
        d.col_primal = reinterpret_cast<const uint8_t *>(at(23));
        d.bus_gen = reinterpret_cast<const int32_t *>(at(24));
        d.lkind = reinterpret_cast<const uint8_t *>(at(25));
        d.iperm = reinterpret_cast<const int32_t *>(at(26));
        d.rr_ptr = reinterpret_cast<const int32_t *>(at(27));
        d.rr_ent = reinterpret_cast<const int32_t *>(at(28));
        d.rb_ptr = reinterpret_cast<const int32_t *>(at(29));
        d.rb_ent = reinterpret_cast<const int32_t *>(at(30));
        d.sup_rnb = reinterpret_cast<const int32_t *>(at(31));
        d.col_sup = reinterpret_cast<const int32_t *>(at(32));
        d.rwbase = h.t_rwbase[ti];
    }
    std::memcpy(buf.data() + p.tdev, tdev.data(), sizeof(ncl::TemplDev) * tdev.size());
    std::vector<ncl::BlockDev> bdev(h.nblk);
    for (int b = 0; b < h.nblk; b++) {
        bdev[b].tmpl = h.block_tmpl[b];
        bdev[b].bl = h.block_bl[b];
        bdev[b].outage = h.block_outage[b];
        bdev[b].col0 = h.block_col0[b];
        bdev[b].kcsc = h.kbase[b];
    }
    std::memcpy(buf.data() + p.bdev, bdev.data(), sizeof(ncl::BlockDev) * bdev.size());
    std::vector<ncl::InstDev> idev(h.inst.size());
    for (size_t i = 0; i < h.inst.size(); i++) {
        const ncl::Inst &I = h.inst[i];
        ncl::InstDev &d = idev[i];
        d.nbd = I.nbd;
        d.nblk = I.nblk;
        d.blk0 = I.blk0;
        d.ng = I.ng;
        d.bstart = I.bstart;
        d.kbb0 = I.kbb0;
        d.sbb0 = I.sbb0;
        d.bd0 = I.bd0;
        d.sp0 = I.sp0;
        d.cp0 = I.cp0;
        d.npk0 = I.npk0;
        d.gp0 = I.gp0;
        d.kcsc_border = I.kcsc_border;
        d.nbb = I.nbb();
        d.kbb_pos = reinterpret_cast<const int32_t *>(base + p.ioff[i][0]);
        d.border_pg = reinterpret_cast<const int32_t *>(base + p.ioff[i][1]);
        d.gen_c2 = reinterpret_cast<const double *>(base + p.ioff[i][2]);
        d.kbr_ptr = reinterpret_cast<const int32_t *>(base + p.ioff[i][5]);
        d.kbr_ent = reinterpret_cast<const int32_t *>(base + p.ioff[i][6]);
        d.mdesc_ptr = reinterpret_cast<const int32_t *>(base + p.ioff[i][7]);
        d.mdesc = reinterpret_cast<const ncl::MDesc *>(base + p.ioff[i][8]);
        d.mitems = reinterpret_cast<const ncl::MItem *>(base + p.ioff[i][9]);
        d.bperm = reinterpret_cast<const int32_t *>(base + p.ioff[i][10]);
        d.mw0 = I.mw0;
        d.pe0 = I.pe0;
        d.npair = I.npair;
        d.t0 = I.t0;
        d.nt = I.nt;
    }
    std::memcpy(buf.data() + p.idev, idev.data(), sizeof(ncl::InstDev) * idev.size());
    if (hipMemcpyAsync(base, buf.data(), buf.size(), hipMemcpyHostToDevice, st) != hipSuccess) return NCL_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return NCL_ERR_HIP;
    h.ws = dptr;
    h.ws_bytes = bytes;
    h.nrhs_max = nrhs_max;
    h.d.tmpl = reinterpret_cast<ncl::TemplDev *>(base + p.tdev);
    h.d.blk = reinterpret_cast<ncl::BlockDev *>(base + p.bdev);
    h.d.inst = reinterpret_cast<ncl::InstDev *>(base + p.idev);
    h.d.work = reinterpret_cast<ncl::Work *>(base + p.work);
    h.d.bprim = reinterpret_cast<const uint8_t *>(base + p.bprim);
    h.d.kval = reinterpret_cast<double *>(base + p.kval);
    h.d.lpan = reinterpret_cast<double *>(base + p.lpan);
    h.d.upan = reinterpret_cast<double *>(base + p.upan);
    h.d.dval = reinterpret_cast<double *>(base + p.dval);
    h.d.spart = reinterpret_cast<double *>(base + p.spart);
    h.d.sbb = reinterpret_cast<double *>(base + p.sbb);
    h.d.lbb = reinterpret_cast<double *>(base + p.lbb);
    h.d.ybuf = reinterpret_cast<double *>(base + p.ybuf);
    h.d.cpart = reinterpret_cast<double *>(base + p.cpart);
    h.d.zint = reinterpret_cast<double *>(base + p.zint);
    h.d.sint = reinterpret_cast<double *>(base + p.sint);
    h.d.stat = reinterpret_cast<int64_t *>(base + p.stat);
    h.d.xint = reinterpret_cast<double *>(base + p.xint);
    h.d.bint = reinterpret_cast<double *>(base + p.bint);
    h.d.rint = reinterpret_cast<double *>(base + p.rint);
    h.d.rbuf = reinterpret_cast<double *>(base + p.rbuf);
    h.d.epart = reinterpret_cast<double *>(base + p.epart);
    h.d.pg_col = reinterpret_cast<const int64_t *>(base + p.pg_col);
    h.d.row_pq = reinterpret_cast<const int64_t *>(base + p.row_pq);
    h.bound = true;
    h.factored = false;
    h.blocks_done = false;
    h.values_set = false;
    h.factor_failed = false;
    return NCL_OK;
}

int ncl_kkt_assemble(ncl_kkt *k, const ncl_kkt_point *pt, void *stream) {
    if (!k || !pt || !pt->z || !pt->sigma || !(pt->rho > 0)) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.from_network) return NCL_ERR_STATE;
    if (pt->flags & ~NCL_NO_SHIFT) return NCL_ERR_ARG;
    ncl::LaunchArgs l;
    l.z = pt->z;
    l.sig = pt->sigma;
    l.rho = pt->rho;
    l.flags = pt->flags;
    const ncl::DevArgs a = dev_args(h);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    l.zdst = h.d.zint;
    l.sdst = h.d.sint;
    if (run(h, NCL_K_INTERLEAVE, a, l, st) != hipSuccess) return NCL_ERR_HIP;
    if (run(h, NCL_K_ASSEMBLE, a, l, st) != hipSuccess) return NCL_ERR_HIP;
    h.values_set = true;
    return NCL_OK;
}

int ncl_kkt_set_values(ncl_kkt *k, const double *dvals, void *stream) {
    if (!k || !dvals) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound) return NCL_ERR_STATE;
    ncl::LaunchArgs l;
    l.src = dvals;
    l.dst = h.d.kval;
    l.to_internal = true;
    if (run(h, NCL_K_VALUES, dev_args(h), l, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return NCL_ERR_HIP;
    h.values_set = true;
    return NCL_OK;
}

int ncl_kkt_get_values(ncl_kkt *k, double *dvals, void *stream) {
    if (!k || !dvals) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound) return NCL_ERR_STATE;
    ncl::LaunchArgs l;
    l.src = h.d.kval;
    l.dst = dvals;
    l.to_internal = false;
    return hip_rc(run(h, NCL_K_VALUES, dev_args(h), l, reinterpret_cast<hipStream_t>(stream)));
}

// The blocks' factorisation: per level the gathers, diagonal blocks and rows.
static int factor_levels(Handle &h, const ncl::DevArgs &a, hipStream_t st) {
    const ncl::Schedule &S = h.sched;
    const ncl::Work *W = h.d.work;
    auto list = [&](int kind, size_t off, const std::vector<int32_t> &ptr, int l) {
        ncl::LaunchArgs la;
        la.wl = W + off + ptr[l];
        la.nw = ptr[l + 1] - ptr[l];
        return run(h, kind, a, la, st);
    };
    for (int l = 0; l < S.nlev; l++) {
        if (list(NCL_K_FAC_GATHER, h.w_a, S.a_ptr, l) != hipSuccess) return NCL_ERR_HIP;
        if (list(NCL_K_FAC_DIAG, h.w_b, S.b_ptr, l) != hipSuccess) return NCL_ERR_HIP;
        if (list(NCL_K_FAC_ROWS, h.w_c, S.c_ptr, l) != hipSuccess) return NCL_ERR_HIP;
    }
    return NCL_OK;
}

// One level of the blocks' factorisation (the combined call's pipeline).
static int factor_level(Handle &h, const ncl::DevArgs &a, int l, hipStream_t st) {
    const ncl::Schedule &S = h.sched;
    const ncl::Work *W = h.d.work;
    auto list = [&](int kind, size_t off, const std::vector<int32_t> &ptr) {
        ncl::LaunchArgs la;
        la.wl = W + off + ptr[l];
        la.nw = ptr[l + 1] - ptr[l];
        return run(h, kind, a, la, st);
    };
    if (list(NCL_K_FAC_GATHER, h.w_a, S.a_ptr) != hipSuccess || list(NCL_K_FAC_DIAG, h.w_b, S.b_ptr) != hipSuccess ||
        list(NCL_K_FAC_ROWS, h.w_c, S.c_ptr) != hipSuccess)
        return NCL_ERR_HIP;
    return NCL_OK;
}

// The border: the Schur products (schur = true), their sum and the dense
// border factor.
static int border_launches(Handle &h, const ncl::DevArgs &a, bool schur, hipStream_t st) {
    const ncl::LaunchArgs none;
    if (schur && run(h, NCL_K_BORDER_SCHUR, a, none, st) != hipSuccess) return NCL_ERR_HIP;
    if (run(h, NCL_K_BORDER_SUM, a, none, st) != hipSuccess) return NCL_ERR_HIP;
    // the register path for borders of up to kBorderRegMax rows, then one
    // launch per column block of the largest larger border
    {
        ncl::LaunchArgs l;
        l.b0 = -2;
        if (run(h, NCL_K_BORDER_FACTOR, a, l, st) != hipSuccess) return NCL_ERR_HIP;
    }
    const int nbk = (big_border(h) + ncl::kBorderBlock - 1) / ncl::kBorderBlock;
    for (int b = -1; b < nbk - 1; b++) {
        ncl::LaunchArgs l;
        l.b0 = b;
        if (run(h, NCL_K_BORDER_FACTOR, a, l, st) != hipSuccess) return NCL_ERR_HIP;
    }
    return NCL_OK;
}

int ncl_kkt_factor_blocks(ncl_kkt *k, void *stream) {
    if (!k) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.values_set) return NCL_ERR_STATE;
    // the factors are overwritten from here on: no solve until the border is done
    h.blocks_done = false;
    h.factored = false;
    h.factor_failed = false;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ncl::DevArgs a = dev_args(h);
    int rc = factor_levels(h, a, st);
    if (rc) return rc;
    if (h.nbd_tot && run(h, NCL_K_BORDER_SCHUR, a, ncl::LaunchArgs{}, st) != hipSuccess) return NCL_ERR_HIP;
    h.blocks_done = true;
    return NCL_OK;
}

int ncl_kkt_factor_border(ncl_kkt *k, void *stream) {
    if (!k) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.blocks_done) return NCL_ERR_STATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ncl::DevArgs a = dev_args(h);
    const ncl::LaunchArgs none;
    if (h.nbd_tot) {
        const int rc = border_launches(h, a, false, st);
        if (rc) return rc;
    }
    for (int kind : {NCL_K_STATUS_INIT, NCL_K_STATUS})
        if (run(h, kind, a, none, st) != hipSuccess) return NCL_ERR_HIP;
    h.factored = true;
    return NCL_OK;
}

int ncl_kkt_factor(ncl_kkt *k, void *stream) {
    int rc = ncl_kkt_factor_blocks(k, stream);
    return rc ? rc : ncl_kkt_factor_border(k, stream);
}

int ncl_kkt_info(ncl_kkt *k, ncl_kkt_report *rep, void *stream) {
    if (!k || !rep) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.factored) return NCL_ERR_STATE;
    int64_t sw[ncl::kStatWords * ncl::kStatStride], s[ncl::kStatWords];
    if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return NCL_ERR_HIP;
    if (hipMemcpy(sw, h.d.stat, sizeof(sw), hipMemcpyDeviceToHost) != hipSuccess) return NCL_ERR_HIP;
    for (int q = 0; q < ncl::kStatWords; q++) s[q] = sw[q * ncl::kStatStride];
    rep->npos = s[0];
    rep->nneg = s[1];
    rep->nzero = s[2];
    double mn, mx;
    std::memcpy(&mn, &s[4], sizeof(double));
    std::memcpy(&mx, &s[5], sizeof(double));
    rep->min_absd = s[4] == INT64_MAX ? INFINITY : mn;
    rep->max_absd = mx;
    if (s[3] == INT64_MAX) {
        rep->first_bad = -1;
        rep->status = NCL_OK;
    } else {
        rep->first_bad = s[3] / 8;
        const int code = int(s[3] % 8);
        rep->status = code == 1 ? NCL_ERR_INERTIA : code == 2 ? NCL_ERR_ZERO_PIVOT : NCL_ERR_NONFINITE;
    }
    rep->nnonfinite = s[6];
    // the same test k_sol_load makes on the device
    rep->solvable = (s[2] == 0 && s[6] == 0 && s[0] == h.nprimal) ? 1 : 0;
    h.factor_failed = !rep->solvable;
    return NCL_OK;
}

int ncl_kkt_get_factors(ncl_kkt *k, double *lx, double *dd, void *stream) {
    if (!k) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.factored) return NCL_ERR_STATE;
    if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return NCL_ERR_HIP;
    std::vector<double> pan(size_t(h.lint)), dv(size_t(h.dint + h.nbd_tot));
    std::vector<double> sbb(static_cast<size_t>(h.npk_tot));
    if (!pan.empty() && hipMemcpy(pan.data(), h.d.lpan, sizeof(double) * pan.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return NCL_ERR_HIP;
    if (!dv.empty() && hipMemcpy(dv.data(), h.d.dval, sizeof(double) * dv.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return NCL_ERR_HIP;
    if (!sbb.empty() && hipMemcpy(sbb.data(), h.d.lbb, sizeof(double) * sbb.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return NCL_ERR_HIP;
    int64_t q = 0;
    for (const ncl::Inst &I : h.inst) {
        for (int b = I.blk0; b < I.blk0 + I.nblk; b++) {
            const int ti = h.block_tmpl[b];
            const Template &t = h.tmpl[ti];
            const int64_t nb = int64_t(t.blocks.size()), bl = h.block_bl[b];
            const double *P = pan.data() + h.t_lbase[ti] + bl;
            if (dd)
                for (int j = 0; j < t.n; j++) dd[h.block_col0[b] + j] = dv[size_t(h.t_dbase[ti] + int64_t(j) * nb + bl)];
            if (!lx) continue;
            const int ns = int(t.sup.size()) - 1;
            for (int s = 0; s < ns; s++) {
                const int f = t.sup[s], w = t.sup[s + 1] - f, r = t.srp[s + 1] - t.srp[s];
                const int32_t *R = &t.sri[t.srp[s]];
                for (int c = 0; c < w; c++) {
                    const int j = f + c;
                    for (int p = t.lp[j]; p < t.lp[j + 1]; p++) {
                        const int pos = int(std::lower_bound(R, R + r, t.li[p]) - R);
                        lx[q++] = P[(int64_t(t.panel_off[s]) + int64_t(c) * r + pos) * nb];
                    }
                }
            }
        }
        if (dd)
            for (int j = 0; j < I.nbd; j++) dd[I.bstart + j] = dv[size_t(h.dint + I.bd0 + j)];
        if (lx)
            for (int j = 0; j < I.nbd; j++)
                for (int p = I.blp[j]; p < I.blp[j + 1]; p++) {
                    const int i = I.bli[p];
                    lx[q++] = sbb[size_t(I.sbb0) + size_t(i) * (i + 1) / 2 + j];
                }
    }
    return NCL_OK;
}

// nrhs right-hand sides (columns ld apart) through the factors, every
// launch covering all of them.  refine: one column whose right-hand side is
// the residual the backward-error kernels left (blocks interleaved in rint,
// the border in rbuf); its solution is added into x.
// The solve in two halves.  The first (right-hand side in, forward
// substitution of the blocks, the blocks' parts of the border right-hand
// side) needs only the blocks' factors; the second (the border solve, the
// backward substitution, the solution out) needs the border's factor and
// the factorisation status.  check = false: the load does not consult the
// status (the combined factor+solve computes it between the halves; the
// store writes NaN for an unusable factorisation either way).
static ncl::LaunchArgs solve_args(Handle &h, const double *b, double *x, int nrhs, int64_t ld, bool refine) {
    ncl::LaunchArgs v;
    v.b = refine ? h.d.rbuf : b;
    v.x = x;
    v.y = h.d.ybuf;
    v.cpart = h.d.cpart;
    v.src = refine ? h.d.rint : nullptr;
    v.accumulate = refine;
    v.nrhs = nrhs;
    v.bld = ld;
    v.ys = h.dint + h.nbd_tot;
    v.cps = h.cp_tot;
    return v;
}

// The first half of a solve: the right-hand side loaded into the
// interleaved order (without the factor's status check in the combined
// call, whose status comes later), the forward substitution level by level,
// and the border rows' partial sums.
static int solve_load(Handle &h, const ncl::DevArgs &a, const ncl::LaunchArgs &v, hipStream_t st, bool check = false) {
    ncl::LaunchArgs la = v;
    la.nocheck = !check;
    return run(h, NCL_K_SOL_LOAD, a, la, st) != hipSuccess ? NCL_ERR_HIP : NCL_OK;
}

static int solve_forward_level(Handle &h, const ncl::DevArgs &a, const ncl::LaunchArgs &v, int l, hipStream_t st) {
    const ncl::Schedule &S = h.sched;
    const ncl::Work *W = h.d.work;
    auto list = [&](int kind, size_t off, const std::vector<int32_t> &ptr) {
        ncl::LaunchArgs la = v;
        la.wl = W + off + ptr[l];
        la.nw = ptr[l + 1] - ptr[l];
        return run(h, kind, a, la, st);
    };
    if (list(NCL_K_SOL_FWD_GATHER, h.w_f, S.f_ptr) != hipSuccess || list(NCL_K_SOL_FWD_DIAG, h.w_d, S.d_ptr) != hipSuccess)
        return NCL_ERR_HIP;
    return NCL_OK;
}

static int solve_border_partials(Handle &h, const ncl::DevArgs &a, const ncl::LaunchArgs &v, hipStream_t st) {
    if (!h.nbd_tot) return NCL_OK;
    ncl::LaunchArgs la = v;
    la.wl = h.d.work + h.w_bpart;
    la.nw = int(h.sched.bpart.size());
    return run(h, NCL_K_SOL_BPART, a, la, st) != hipSuccess ? NCL_ERR_HIP : NCL_OK;
}

static int solve_first_half(Handle &h, const ncl::DevArgs &a, const ncl::LaunchArgs &v, bool check, hipStream_t st) {
    int rc = solve_load(h, a, v, st, check);
    for (int l = 0; !rc && l < h.sched.nlev; l++) rc = solve_forward_level(h, a, v, l, st);
    return rc ? rc : solve_border_partials(h, a, v, st);
}

static int solve_second_half(Handle &h, const ncl::DevArgs &a, const ncl::LaunchArgs &v, hipStream_t st) {
    const ncl::Schedule &S = h.sched;
    const ncl::Work *W = h.d.work;
    if (h.nbd_tot && run(h, NCL_K_SOL_BORDER, a, v, st) != hipSuccess) return NCL_ERR_HIP;
    {
        ncl::LaunchArgs la = v;
        la.wl = W + h.w_sb;
        la.nw = int(S.sb.size());
        la.nnar = S.sb_nar;
        if (run(h, NCL_K_SOL_BWD_BORDER, a, la, st) != hipSuccess) return NCL_ERR_HIP;
    }
    for (int l = S.nlev - 1; l >= 0; l--) {
        ncl::LaunchArgs la = v;
        la.wl = W + h.w_sn + S.sn_ptr[l];
        la.nw = S.sn_ptr[l + 1] - S.sn_ptr[l];
        la.nnar = S.sn_nar[l];
        la.wmax = S.sn_wmax[l];
        if (run(h, NCL_K_SOL_BWD, a, la, st) != hipSuccess) return NCL_ERR_HIP;
    }
    if (run(h, NCL_K_SOL_STORE, a, v, st) != hipSuccess) return NCL_ERR_HIP;
    return NCL_OK;
}

static int solve_columns(Handle &h, const ncl::DevArgs &a, const double *b, double *x, int nrhs, int64_t ld, bool refine,
                         hipStream_t st) {
    const ncl::LaunchArgs v = solve_args(h, b, x, nrhs, ld, refine);
    const int rc = solve_first_half(h, a, v, true, st);
    return rc ? rc : solve_second_half(h, a, v, st);
}

// The library's second stream and its fork and join events, created on
// first use (on the device current then).
static int side_stream(Handle &h) {
    if (h.side) return NCL_OK;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return NCL_ERR_HIP;
    if (hipEventCreateWithFlags(&e0, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipStreamDestroy(s);
        return NCL_ERR_HIP;
    }
    h.side = s;
    h.ev_fork = e0;
    h.ev_join = e1;
    return NCL_OK;
}

// one event per factor level (created once per handle)
static int level_events(Handle &h) {
    while (int(h.ev_lev.size()) < h.sched.nlev) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return NCL_ERR_HIP;
        h.ev_lev.push_back(e);
    }
    return NCL_OK;
}

static int do_solve(ncl_kkt *k, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream) {
    if (!k || !db || !dx || nrhs < 1) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.factored || h.factor_failed) return NCL_ERR_STATE;
    if (nrhs > h.nrhs_max || ld < h.N) return NCL_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ncl::DevArgs a = dev_args(h);
    return solve_columns(h, a, db, dx, nrhs, ld, false, st);
}

// r = b - K x of one column into rint (blocks) and rbuf (border), and the
// partial maxima of the backward error; with derr, its final (eta, omega).
static int residual_column(Handle &h, const ncl::DevArgs &a, const double *b, const double *x, double *derr,
                           hipStream_t st) {
    ncl::LaunchArgs l;
    l.z = x;
    l.sig = b;
    l.zdst = a.xint;
    l.sdst = a.bint;
    if (run(h, NCL_K_INTERLEAVE, a, l, st) != hipSuccess) return NCL_ERR_HIP;
    if (run(h, NCL_K_BERR_ROWS, a, l, st) != hipSuccess) return NCL_ERR_HIP;
    if (run(h, NCL_K_BERR_BORDER, a, l, st) != hipSuccess) return NCL_ERR_HIP;
    if (derr) {
        l.dst = derr;
        if (run(h, NCL_K_BERR_FINAL, a, l, st) != hipSuccess) return NCL_ERR_HIP;
    }
    return NCL_OK;
}

int ncl_kkt_layout_kinds(const ncl_kkt *k, uint8_t *kinds) {
    if (!k || !kinds) return NCL_ERR_ARG;
    const Handle &h = k->h;
    if (!h.from_network) return NCL_ERR_ARG;
    static_assert(int(ncl::LK_VM) == NCL_L_VM && int(ncl::LK_FLOW) == NCL_L_FLOW && int(ncl::LK_NUP) == NCL_L_NUP &&
                      int(ncl::LK_CLO) == NCL_L_CLO && int(ncl::LK_VM0) == NCL_L_VM0,
                  "kind codes");
    for (const ncl::Inst &I : h.inst) {
        for (int b = I.blk0; b < I.blk0 + I.nblk; b++) {
            const Template &t = h.tmpl[h.block_tmpl[b]];
            std::memcpy(kinds + h.block_col0[b], t.lkind.data(), size_t(t.n));
        }
        for (int j = 0; j < I.nbd; j++) kinds[I.bstart + j] = j < I.ng ? NCL_L_PG : NCL_L_VM0;
    }
    return NCL_OK;
}

static int nlp_check(const Handle &h, const ncl_nlp *p) {
    if (!p || !p->pd || !(p->mu > 0) || !(p->rho > 0) || !(p->vmax > p->vmin) || !(p->qmax > 0) || !(p->pmax > 0) ||
        !(p->smax2 > 0) || p->eps < 0)
        return NCL_ERR_ARG;
    if (!h.from_network || h.inst.size() != 1 || (h.inst[0].flags & (NCL_PVPQ | NCL_SCREEN | NCL_AGC))) return NCL_ERR_ARG;
    if (!h.bound) return NCL_ERR_STATE;
    return NCL_OK;
}

int ncl_kkt_residual(ncl_kkt *k, const ncl_nlp *p, const double *z, double *F, double *sigma, void *stream) {
    if (!k || !z || !F || !sigma || F == z || sigma == z || F == sigma) return NCL_ERR_ARG;
    Handle &h = k->h;
    const int rc = nlp_check(h, p);
    if (rc) return rc;
    ncl::LaunchArgs l;
    l.z = z;
    l.nlp = *p;
    l.rho = p->rho;
    l.F = F;
    l.sigma_out = sigma;
    return hip_rc(run(h, NCL_K_RESIDUAL, dev_args(h), l, reinterpret_cast<hipStream_t>(stream)));
}

int ncl_kkt_max_step(ncl_kkt *k, const ncl_nlp *p, const double *z, const double *dz, double tau, double *alpha,
                     void *stream) {
    if (!k || !z || !dz || !alpha || !(tau > 0 && tau < 1)) return NCL_ERR_ARG;
    Handle &h = k->h;
    const int rc = nlp_check(h, p);
    if (rc) return rc;
    ncl::LaunchArgs l;
    l.z = z;
    l.dz = dz;
    l.nlp = *p;
    l.tau = tau;
    l.alpha = alpha;
    return hip_rc(run(h, NCL_K_MAX_STEP, dev_args(h), l, reinterpret_cast<hipStream_t>(stream)));
}

// ---------------------------------------------------------------- inertia correction

namespace {

// Assemble the exact K (no diagonal shift) at (z, sig) and factor it; ok:
// the inertia (n, m) of the Newton matrix of a minimum, no zero or
// non-finite pivot (single pivots may carry the other sign).
// assembled: K at (z, sig) without the shift is already in the handle
int factor_exact(Handle &h, ncl_kkt *k, const double *z, const double *sig, double rho, bool &ok, hipStream_t st,
                 bool assembled = false) {
    ncl_kkt_point pt{z, sig, rho, NCL_NO_SHIFT};
    int rc = assembled ? NCL_OK : ncl_kkt_assemble(k, &pt, st);
    if (!rc) rc = ncl_kkt_factor(k, st);
    ncl_kkt_report rep{};
    if (!rc) rc = ncl_kkt_info(k, &rep, st);
    if (rc) return rc;
    ok = (rep.status == NCL_OK || rep.status == NCL_ERR_INERTIA) && rep.nzero == 0 && rep.nnonfinite == 0 &&
         rep.npos == h.nprimal && rep.nneg == h.N - h.nprimal;
    return NCL_OK;
}

// The inertia correction of Section V-C as a primal shift: the exact K,
// then sig + dw on the primal positions with dw from a third of the last
// accepted shift (or 1e-4), growing x8 below 1e12.  sgs: N doubles.
int inertia_loop(Handle &h, ncl_kkt *k, const double *z, const double *sig, double rho, double &dw_last, int &nfac,
                 double *sgs, hipStream_t st, bool first_assembled = false) {
    const ncl::DevArgs a = dev_args(h);
    bool ok = false;
    nfac = 1;
    int rc = factor_exact(h, k, z, sig, rho, ok, st, first_assembled);
    if (rc) return rc;
    if (ok) {
        dw_last = 0.0;
        return NCL_OK;
    }
    for (double dw = dw_last > 0 ? dw_last / 3.0 : 1e-4; dw < 1e12; dw *= 8.0) {
        if (ncl::launch_ipm_point(a, ncl::IpmArgs{}, ncl::IPM_SHIFT, sig, dw, sgs, nullptr, nullptr, nullptr, st) !=
            hipSuccess)
            return NCL_ERR_HIP;
        nfac++;
        if ((rc = factor_exact(h, k, z, sgs, rho, ok, st))) return rc;
        if (ok) {
            dw_last = dw;
            return NCL_OK;
        }
    }
    return NCL_ERR_INERTIA;
}

}  // namespace

// ---------------------------------------------------------------- dispatch map: Newton and adjoint

namespace {

struct Disp {
    Handle &h;
    ncl_kkt *k;
    hipStream_t st;
    ncl::DevArgs a;
    double *sc;          // device scalars: norm, step excess, alpha
    bool sync_read(const double *d, double &v) {
        return hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, st) == hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    }
    int residual(const ncl_nlp &q, const double *z, double *F, double *sig) {
        ncl::LaunchArgs l;
        l.z = z;
        l.nlp = q;
        l.rho = q.rho;
        l.F = F;
        l.sigma_out = sig;
        return hip_rc(run(h, NCL_K_RESIDUAL, a, l, st));
    }
    int norm2(const double *x, double &v) {
        if (ncl::launch_vec_reduce(h.N, x, nullptr, 0.0, 0, h.d.epart, sc, st) != hipSuccess) return NCL_ERR_HIP;
        return sync_read(sc, v) ? NCL_OK : NCL_ERR_HIP;
    }
    // max_i |dz_i| - tol (1 + |z_i|): <= 0 when every step component is small
    int excess(const double *z, const double *dz, double tol, double &v) {
        if (ncl::launch_vec_reduce(h.N, dz, z, tol, 1, h.d.epart, sc + 1, st) != hipSuccess) return NCL_ERR_HIP;
        return sync_read(sc + 1, v) ? NCL_OK : NCL_ERR_HIP;
    }
    int max_step(const ncl_nlp &q, const double *z, const double *dz, double &al) {
        const int rc = ncl_kkt_max_step(k, &q, z, dz, 0.995, sc + 2, st);
        if (rc) return rc;
        return sync_read(sc + 2, al) ? NCL_OK : NCL_ERR_HIP;
    }
    int axpy(double al, const double *x, const double *y, double *out) {
        return hip_rc(ncl::launch_vec_axpy(h.N, al, x, y, out, st));
    }
    int factor_min(const double *z, const double *sig, double rho, bool &ok) {
        return factor_exact(h, k, z, sig, rho, ok, st);
    }
};

}  // namespace

int ncl_kkt_dispatch_newton(ncl_kkt *k, const ncl_nlp *p, double *dz_state, double *dwork, ncl_newton_opts *o,
                            void *stream) {
    if (!k || !dz_state || !dwork || !o || !(o->step_tol > 0) || !(o->floor_tol > 0) || o->maxit < 1) return NCL_ERR_ARG;
    Handle &h = k->h;
    int rc = nlp_check(h, p);
    if (rc) return rc;
    if (h.ng_disp == 0 || ncl::vec_reduce_partials(h.N) > 8 * berr_partials(h)) return NCL_ERR_ARG;
    const int64_t N = h.N;
    double *F = dwork, *sig = F + N, *dz = sig + N, *zt = dz + N, *Ft = zt + N, *sgt = Ft + N, *sgs = sgt + N;
    Disp D{h, k, reinterpret_cast<hipStream_t>(stream), dev_args(h), sgs + N};
    double *z = dz_state;
    // barrier values: from the default start, 10, 3, 1, 0.3, 0.1, 0.03 down
    // to (and ending at) p->mu; from a given state only p->mu
    static const double kSchedule[] = {10.0, 3.0, 1.0, 0.3, 0.1, 0.03};
    std::vector<double> mus;
    if (o->from_default) {
        if (ncl::launch_disp_point(D.a, *p, nullptr, 0.0, 0, z, D.st) != hipSuccess) return NCL_ERR_HIP;
        for (double m : kSchedule)
            if (m > p->mu) mus.push_back(m);
    }
    mus.push_back(p->mu);
    int total = 0;
    for (double mu : mus) {
        ncl_nlp q = *p;
        q.mu = mu;
        const double tol = mu == p->mu ? o->step_tol : 1e-6;
        double nrm = 0.0;
        if ((rc = D.residual(q, z, F, sig)) || (rc = D.norm2(F, nrm))) return rc;
        bool converged = false;
        for (int it = 0; it < o->maxit && !converged; it++) {
            // Newton matrix with the inertia of a minimum (the inertia correction)
            int nfac = 0;
            if ((rc = inertia_loop(h, k, z, sig, q.rho, o->dw_last, nfac, sgs, D.st))) return rc;
            // dz = -K^{-1} F (the solve is linear and rounding is symmetric
            // under negation, so this equals the solve of -F bit for bit)
            if ((rc = ncl_kkt_solve(k, F, dz, 1, N, D.st))) return rc;
            if ((rc = D.axpy(-1.0, dz, nullptr, dz))) return rc;
            double ex = 0.0, al = 1.0;
            if ((rc = D.excess(z, dz, tol, ex))) return rc;
            if (ex <= 0.0) {
                // converged: take the last (tiny, quadratically accurate) step if it is feasible
                if ((rc = D.max_step(q, z, dz, al))) return rc;
                if (al >= 1.0) {
                    if ((rc = D.axpy(1.0, dz, z, z)) || (rc = D.residual(q, z, F, sig))) return rc;
                }
                converged = true;
                break;
            }
            if ((rc = D.max_step(q, z, dz, al))) return rc;
            double nt = 0.0;
            for (;;) {
                if ((rc = D.axpy(al, dz, z, zt)) || (rc = D.residual(q, zt, Ft, sgt)) || (rc = D.norm2(Ft, nt)))
                    return rc;
                if (nt <= (1.0 - 1e-4 * al) * nrm || al < 1e-10) break;
                al *= 0.5;
            }
            if (al < 1e-10) {
                // |F| at its rounding floor (variables pressed against their
                // bounds make the barrier curvature huge) with a tiny step
                if ((rc = D.excess(z, dz, o->floor_tol, ex))) return rc;
                if (ex <= 0.0) {
                    converged = true;
                    break;
                }
            }
            if (hipMemcpyAsync(z, zt, sizeof(double) * size_t(N), hipMemcpyDeviceToDevice, D.st) != hipSuccess ||
                hipMemcpyAsync(F, Ft, sizeof(double) * size_t(N), hipMemcpyDeviceToDevice, D.st) != hipSuccess ||
                hipMemcpyAsync(sig, sgt, sizeof(double) * size_t(N), hipMemcpyDeviceToDevice, D.st) != hipSuccess)
                return NCL_ERR_HIP;
            nrm = nt;
            total++;
        }
        if (!converged) {
            o->iterations = total;
            return NCL_ERR_NOT_CONVERGED;
        }
    }
    // leave the exact K at the solution factored for the adjoint solves
    bool ok = false;
    if ((rc = D.residual(*p, z, F, sig)) || (rc = D.factor_min(z, sig, p->rho, ok))) return rc;
    o->iterations = total;
    return ok ? NCL_OK : NCL_ERR_INERTIA;
}

int ncl_kkt_dispatch_outputs(ncl_kkt *k, const double *dz, double *dphi, double *dpg, void *stream) {
    if (!k || !dz || !dphi) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound) return NCL_ERR_STATE;
    if (h.ng_disp == 0) return NCL_ERR_ARG;
    return hip_rc(ncl::launch_disp_outputs(dev_args(h), dz, dphi, dpg, reinterpret_cast<hipStream_t>(stream)));
}

int ncl_kkt_dispatch_vjp(ncl_kkt *k, const ncl_nlp *p, const double *dz, const double *dgphi, const double *dgpg,
                         double *dgpd, double *dwork, void *stream) {
    if (!k || !dz || !dgphi || !dgpd || !dwork) return NCL_ERR_ARG;
    Handle &h = k->h;
    int rc = nlp_check(h, p);
    if (rc) return rc;
    if (h.ng_disp == 0) return NCL_ERR_ARG;
    if (!h.factored || h.factor_failed) return NCL_ERR_STATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ncl::DevArgs a = dev_args(h);
    double *g = dwork, *adj = dwork + h.N;
    if (ncl::launch_disp_adjoint(a, dz, dgphi, dgpg, g, st) != hipSuccess) return NCL_ERR_HIP;
    if ((rc = ncl_kkt_solve_adjoint(k, g, adj, 1, h.N, stream))) return rc;
    return hip_rc(ncl::launch_disp_load_grad(a, adj, p->qd_ratio, dgpd, st));
}

// ---------------------------------------------------------------- IPM step

static int ipm_check(const Handle &h, const ncl_ipm_problem *p, const ncl_ipm_state *s) {
    if (!p || !s || !p->pd || !p->lo || !p->hi || !p->y_n || !s->z || !s->rt || !s->s || !s->zl || !s->zu)
        return NCL_ERR_ARG;
    if (!(p->mu > 0) || !(p->rho > 0) || !(p->smax2 > 0) || !(p->qmax > 0) || !(p->pmax > 0) || !(p->eps >= 0) ||
        !std::isfinite(p->qd_ratio) || !std::isfinite(p->mu) || !std::isfinite(p->rho))
        return NCL_ERR_ARG;
    if (!h.from_network || h.inst.size() != 1) return NCL_ERR_ARG;
    const uint32_t fl = h.inst[0].flags;
    if ((fl & NCL_SCREEN) && (!p->pg0 || ((fl & NCL_PVPQ) && !p->vm0))) return NCL_ERR_ARG;
    if (!h.bound) return NCL_ERR_STATE;
    return NCL_OK;
}

static ncl::IpmArgs ipm_args(const ncl_ipm_problem &p, const ncl_ipm_state &s) {
    ncl::IpmArgs q;
    q.pd = p.pd;
    q.lo = p.lo;
    q.hi = p.hi;
    q.yn = p.y_n;
    q.z = s.z;
    q.rt = s.rt;
    q.s = s.s;
    q.zl = s.zl;
    q.zu = s.zu;
    q.pg0 = p.pg0;
    q.vm0 = p.vm0;
    q.qd_ratio = p.qd_ratio;
    q.qmax = p.qmax;
    q.pmax = p.pmax;
    q.smax2 = p.smax2;
    q.eps = p.eps;
    q.mu = p.mu;
    q.rho = p.rho;
    return q;
}

// r = (r1, r2): the multipliers masked to the dual rows (xm), the residual
// xm - K xm, whose primal rows are -J'y, c and grad phi (cg), combined
static int ipm_rhs(Handle &h, const ncl::IpmArgs &q, double *r, double *work, hipStream_t st) {
    const ncl::DevArgs a = dev_args(h);
    double *xm = work, *cg = work + h.N;
    if (ncl::launch_ipm_point(a, q, ncl::IPM_MASK, nullptr, 0.0, xm, nullptr, nullptr, nullptr, st) != hipSuccess)
        return NCL_ERR_HIP;
    int rc = residual_column(h, a, xm, xm, nullptr, st);
    if (rc) return rc;
    if (ncl::launch_ipm_cons(a, q, cg, st) != hipSuccess) return NCL_ERR_HIP;
    return hip_rc(ncl::launch_ipm_point(a, q, ncl::IPM_RHS, cg, 0.0, r, nullptr, nullptr, nullptr, st));
}

int ncl_kkt_ipm_sigma(ncl_kkt *k, const ncl_ipm_problem *p, const ncl_ipm_state *s, double *dsigma, void *stream) {
    if (!k || !dsigma) return NCL_ERR_ARG;
    Handle &h = k->h;
    const int rc = ipm_check(h, p, s);
    if (rc) return rc;
    return hip_rc(ncl::launch_ipm_point(dev_args(h), ipm_args(*p, *s), ncl::IPM_SIGMA, nullptr, 0.0, dsigma, nullptr,
                                        nullptr, nullptr, reinterpret_cast<hipStream_t>(stream)));
}

int ncl_kkt_ipm_rhs(ncl_kkt *k, const ncl_ipm_problem *p, const ncl_ipm_state *s, double *drhs, double *dwork,
                    void *stream) {
    if (!k || !drhs || !dwork) return NCL_ERR_ARG;
    Handle &h = k->h;
    const int rc = ipm_check(h, p, s);
    if (rc) return rc;
    if (!h.values_set) return NCL_ERR_STATE;
    return ipm_rhs(h, ipm_args(*p, *s), drhs, dwork, reinterpret_cast<hipStream_t>(stream));
}

int ncl_kkt_ipm_recover(ncl_kkt *k, const ncl_ipm_problem *p, const ncl_ipm_state *s, const double *ddz,
                        const ncl_ipm_direction *d, void *stream) {
    if (!k || !ddz || !d || !d->drt || !d->ds || !d->dzl || !d->dzu) return NCL_ERR_ARG;
    Handle &h = k->h;
    const int rc = ipm_check(h, p, s);
    if (rc) return rc;
    return hip_rc(ncl::launch_ipm_point(dev_args(h), ipm_args(*p, *s), ncl::IPM_RECOVER, ddz, 0.0, d->drt, d->ds,
                                        d->dzl, d->dzu, reinterpret_cast<hipStream_t>(stream)));
}

int ncl_kkt_factor_inertia(ncl_kkt *k, const double *dz, const double *dsigma, double rho, ncl_inertia_opts *o,
                           double *dwork, void *stream) {
    if (!k || !dz || !dsigma || !o || !dwork || !(rho > 0) || !(o->dw_last >= 0)) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.from_network || h.inst.size() != 1) return NCL_ERR_ARG;
    if (!h.bound) return NCL_ERR_STATE;
    int nfac = 0;
    const int rc = inertia_loop(h, k, dz, dsigma, rho, o->dw_last, nfac, dwork, reinterpret_cast<hipStream_t>(stream));
    o->nfactor = nfac;
    return rc;
}

int ncl_kkt_ipm_step(ncl_kkt *k, const ncl_ipm_problem *p, const ncl_ipm_state *s, const ncl_ipm_direction *d,
                     ncl_inertia_opts *o, double *dwork, void *stream) {
    if (!k || !d || !d->dz || !d->drt || !d->ds || !d->dzl || !d->dzu || !o || !dwork || !(o->dw_last >= 0))
        return NCL_ERR_ARG;
    Handle &h = k->h;
    int rc = ipm_check(h, p, s);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ncl::DevArgs a = dev_args(h);
    const ncl::IpmArgs q = ipm_args(*p, *s);
    const int64_t N = h.N;
    // sigma, then the inertia-corrected factorisation; once factored, the
    // same dwork holds the right-hand side (first N) and its work (2 N)
    double *sg = dwork, *sgs = dwork + N;
    if (ncl::launch_ipm_point(a, q, ncl::IPM_SIGMA, nullptr, 0.0, sg, nullptr, nullptr, nullptr, st) != hipSuccess)
        return NCL_ERR_HIP;
    int nfac = 0;
    rc = inertia_loop(h, k, s->z, sg, p->rho, o->dw_last, nfac, sgs, st);
    o->nfactor = nfac;
    if (rc) return rc;
    double *r = dwork;
    if ((rc = ipm_rhs(h, q, r, dwork + N, st))) return rc;
    if ((rc = ncl_kkt_solve(k, r, d->dz, 1, N, st))) return rc;
    return hip_rc(
        ncl::launch_ipm_point(a, q, ncl::IPM_RECOVER, d->dz, 0.0, d->drt, d->ds, d->dzl, d->dzu, st));
}

namespace {

// The NCL solve's device evaluations: the barrier KKT error at the current
// point (largest |G| at mu and at 0, largest |rt|), the step lengths, the
// update; every reduction deterministic, read back as a few scalars.
struct NclRun {
    Handle &h;
    ncl_kkt *k;
    hipStream_t st;
    ncl::DevArgs a;
    int64_t N;
    double *cg, *e0, *e1, *e2, *sg, *part, *sc;
    double hs[4] = {0, 0, 0, 0};
    int read(int n) {
        if (hipMemcpyAsync(hs, sc, sizeof(double) * size_t(n), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return NCL_ERR_HIP;
        return NCL_OK;
    }
    int reduce_max(const double *x, int slot) {
        return hip_rc(ncl::launch_vec_reduce(N, x, x, 0.0, 1, part, sc + slot, st));
    }
    // at the point: sigma and K (no shift), which is also the first matrix
    // of the step's inertia correction; J'y from K's Jacobian blocks (the
    // primal rows of x - Kx for x = (0, y) do not depend on sigma), c(w) and
    // grad phi, which the step's right-hand side reuses
    int prepare(const ncl_ipm_problem &p, const ncl_ipm_state &s, double rho) {
        const ncl::IpmArgs q = ipm_args(p, s);
        if (ncl::launch_ipm_point(a, q, ncl::IPM_SIGMA, nullptr, 0.0, sg, nullptr, nullptr, nullptr, st) != hipSuccess)
            return NCL_ERR_HIP;
        ncl_kkt_point pt{s.z, sg, rho, NCL_NO_SHIFT};
        int rc = ncl_kkt_assemble(k, &pt, st);
        if (rc) return rc;
        if (ncl::launch_ipm_point(a, q, ncl::IPM_MASK, nullptr, 0.0, e0, nullptr, nullptr, nullptr, st) != hipSuccess)
            return NCL_ERR_HIP;
        if ((rc = residual_column(h, a, e0, e0, nullptr, st))) return rc;
        return hip_rc(ncl::launch_ipm_cons(a, q, cg, st));
    }
    // hs[0] = max |G| at p.mu, hs[1] = at 0, hs[2] = max |rt| (dual rows)
    int errors(const ncl_ipm_problem &p, const ncl_ipm_state &s, bool all) {
        const ncl::IpmArgs q = ipm_args(p, s);
        if (ncl::launch_ipm_point(a, q, ncl::IPM_ERROR, cg, 0.0, e0, e1, e2, nullptr, st) != hipSuccess)
            return NCL_ERR_HIP;
        int rc = reduce_max(e0, 0);
        if (!rc && all) rc = reduce_max(e1, 1);
        if (!rc && all) rc = reduce_max(e2, 2);
        return rc ? rc : read(all ? 3 : 1);
    }
};

// ncl_kkt_ipm_step after NclRun::prepare at the same point: sigma, K(z,
// sigma) without the shift, J'y and c(w) are in place.  wk: 2 N doubles.
int ipm_step_prepared(Handle &h, ncl_kkt *k, const ncl_ipm_problem &p, const ncl_ipm_state &s,
                      const ncl_ipm_direction &d, ncl_inertia_opts &o, const double *sg, const double *cg, double *wk,
                      hipStream_t st) {
    const ncl::DevArgs a = dev_args(h);
    const ncl::IpmArgs q = ipm_args(p, s);
    const int64_t N = h.N;
    int nfac = 0;
    int rc = inertia_loop(h, k, s.z, sg, p.rho, o.dw_last, nfac, wk, st, true);
    o.nfactor = nfac;
    if (rc) return rc;
    double *r = wk + N;
    if (ncl::launch_ipm_point(a, q, ncl::IPM_RHS, cg, 0.0, r, nullptr, nullptr, nullptr, st) != hipSuccess)
        return NCL_ERR_HIP;
    if ((rc = ncl_kkt_solve(k, r, d.dz, 1, N, st))) return rc;
    return hip_rc(ncl::launch_ipm_point(a, q, ncl::IPM_RECOVER, d.dz, 0.0, d.drt, d.ds, d.dzl, d.dzu, st));
}

int solve_opts_ok(const ncl_solve_opts *o, double rho) {
    return o->tol > 0 && o->mu_min > 0 && o->mu0 >= o->mu_min && o->mu_warm >= o->mu_min && o->kappa_eps > 0 &&
           o->kappa_mu > 0 && o->kappa_mu < 1 && o->theta_mu > 1 && o->tau_min > 0 && o->tau_min < 1 &&
           o->eta0 > 0 && o->eta_shrink > 1 && o->rho_grow > 1 && o->rho_max >= rho && o->max_inner >= 1 &&
           o->max_outer >= 1;
}

}  // namespace

int ncl_kkt_ncl_solve(ncl_kkt *k, const ncl_ipm_problem *p, const ncl_solve_state *s, const ncl_solve_opts *o,
                      ncl_solve_report *rep, double *dwork, void *stream) {
    if (!k || !p || !s || !o || !rep || !dwork || !s->z || !s->rt || !s->s || !s->zl || !s->zu || !s->y_n)
        return NCL_ERR_ARG;
    if (!solve_opts_ok(o, p->rho)) return NCL_ERR_ARG;
    Handle &h = k->h;
    ncl_ipm_problem pr = *p;
    pr.y_n = s->y_n;
    pr.mu = o->mu0;
    const ncl_ipm_state cs{s->z, s->rt, s->s, s->zl, s->zu};
    int rc = ipm_check(h, &pr, &cs);
    if (rc) return rc;
    const int64_t N = h.N;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // dwork: the direction (5 N), ncl_kkt_ipm_step's work (3 N), c and grad
    // phi, three error vectors, sigma, reduction partials, scalars
    double *dz = dwork, *drt = dz + N, *ds = drt + N, *dzl = ds + N, *dzu = dzl + N, *wk = dzu + N;
    NclRun R{h, k, st, dev_args(h), N};
    R.cg = wk + 3 * N;
    R.e0 = R.cg + N;
    R.e1 = R.e0 + N;
    R.e2 = R.e1 + N;
    R.sg = R.e2 + N;
    R.part = R.sg + N;
    R.sc = R.part + ncl::vec_reduce_partials(N);
    if (R.sc + 8 > dwork + 17 * N + 64) return NCL_ERR_ARG;
    // the start must be strictly interior (and finite)
    if (ncl::launch_ipm_point(R.a, ipm_args(pr, cs), ncl::IPM_INTERIOR, nullptr, 0.0, R.e0, nullptr, nullptr, nullptr,
                              st) != hipSuccess)
        return NCL_ERR_HIP;
    if ((rc = R.reduce_max(R.e0, 0)) || (rc = R.read(1))) return rc;
    if (R.hs[0] != 0.0) return NCL_ERR_ARG;
    *rep = ncl_solve_report{};
    rep->status = 1;
    double eta = o->eta0, mu = o->mu0;
    const ncl_ipm_direction dir{dz, drt, ds, dzl, dzu};
    const ncl::IpmMove mv{s->z, s->rt, s->s, s->zl, s->zu, dz, drt, ds, dzl, dzu};
    for (int outer = 0; outer < o->max_outer; outer++) {
        // the subproblem at (y_n, rho), from the current point
        double dw_last = 0.0;
        pr.mu = mu;
        if ((rc = R.prepare(pr, cs, pr.rho)) || (rc = R.errors(pr, cs, true))) return rc;
        double emu = R.hs[0], e0 = R.hs[1], r_inf = R.hs[2];
        int its = 0;
        bool ok = true;
        for (;;) {
            rep->kkt_err = e0;
            if (e0 <= o->tol) break;
            while (emu <= o->kappa_eps * mu && mu > o->mu_min) {
                mu = std::max(o->mu_min, std::min(o->kappa_mu * mu, std::pow(mu, o->theta_mu)));
                pr.mu = mu;
                if ((rc = R.errors(pr, cs, false))) return rc;
                emu = R.hs[0];
            }
            if (its == o->max_inner) {
                ok = false;
                break;
            }
            ncl_inertia_opts io{dw_last, 0, 0};
            rc = ipm_step_prepared(h, k, pr, cs, dir, io, R.sg, R.cg, wk, st);
            rep->factorizations += io.nfactor;
            if (rc) {
                rep->inner += its;
                rep->status = 3;
                return rc;
            }
            dw_last = io.dw_last;
            const ncl::IpmArgs q = ipm_args(pr, cs);
            const double tau = std::max(o->tau_min, 1.0 - mu);
            if (ncl::launch_ipm_line(R.a, q, mv, ncl::IPM_FTB, tau, 0.0, R.e0, R.e1, st) != hipSuccess)
                return NCL_ERR_HIP;
            if ((rc = R.reduce_max(R.e0, 0)) || (rc = R.reduce_max(R.e1, 1)) || (rc = R.read(2))) return rc;
            const double ap = 1.0 / R.hs[0], ad = 1.0 / R.hs[1];
            const int t = rep->inner + its;
            if (o->trace && t < o->trace_len) {
                double *rec = o->trace + size_t(t) * NCL_TRACE_W;
                const double v[NCL_TRACE_W] = {double(outer), mu, e0, emu, dw_last, double(io.nfactor), ap, ad,
                                               pr.rho};
                std::memcpy(rec, v, sizeof(v));
            }
            if (ncl::launch_ipm_line(R.a, q, mv, ncl::IPM_UPDATE, ap, ad, nullptr, nullptr, st) != hipSuccess)
                return NCL_ERR_HIP;
            its++;
            if ((rc = R.prepare(pr, cs, pr.rho)) || (rc = R.errors(pr, cs, true))) return rc;
            emu = R.hs[0];
            e0 = R.hs[1];
            r_inf = R.hs[2];
        }
        rep->inner += its;
        rep->outer = outer + 1;
        rep->mu = mu;
        rep->rho = pr.rho;
        rep->r_inf = r_inf;
        if (!ok) {
            rep->status = 2;
            return NCL_OK;
        }
        if (r_inf <= o->tol) {
            rep->status = 0;
            return NCL_OK;
        }
        if (r_inf <= eta) {
            const ncl::IpmArgs q = ipm_args(pr, cs);
            if (ncl::launch_ipm_point(R.a, q, ncl::IPM_YN, nullptr, 0.0, s->y_n, nullptr, nullptr, nullptr, st) !=
                hipSuccess)
                return NCL_ERR_HIP;
            eta = std::max(eta / o->eta_shrink, o->tol);
        } else {
            pr.rho = std::min(o->rho_grow * pr.rho, o->rho_max);
        }
        mu = o->mu_warm;
    }
    return NCL_OK;
}

const char *ncl_kernel_name(int kind) {
    static const char *names[NCL_K_COUNT] = {
        "k_assemble", "k_values", "k_fac_gather", "k_fac_diag", "k_fac_rows", "k_border_schur", "k_border_sum",
        "k_border_factor", "k_status_init", "k_status", "k_sol_load", "k_sol_fwd_gather", "k_sol_fwd_diag",
        "k_sol_bpart", "k_sol_border", "k_sol_bwd_border", "k_sol_bwd", "k_sol_store",
        "k_residual", "k_max_step", "k_interleave", "k_berr_rows",
        "k_berr_border", "k_berr_final"};
    return kind >= 0 && kind < NCL_K_COUNT ? names[kind] : nullptr;
}

int ncl_kkt_kernel_model(const ncl_kkt *k, int32_t kind, int64_t *launches, int64_t *bytes) {
    if (!k || kind < 0 || kind >= NCL_K_COUNT) return NCL_ERR_ARG;
    if (launches) *launches = k->h.km_launch[kind];
    if (bytes) *bytes = k->h.km_bytes[kind];
    return NCL_OK;
}

int ncl_stream_copy(const double *dsrc, double *ddst, int64_t n, void *stream) {
    if (!dsrc || !ddst || n < 0 || (n & 1) || (reinterpret_cast<uintptr_t>(dsrc) & 15) ||
        (reinterpret_cast<uintptr_t>(ddst) & 15))
        return NCL_ERR_ARG;
    return ncl::launch_copy(dsrc, ddst, n, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? NCL_OK : NCL_ERR_HIP;
}

int ncl_kkt_profile(ncl_kkt *k, int32_t kind) {
    if (!k || kind < -1 || kind >= NCL_K_COUNT) return NCL_ERR_ARG;
    k->h.prof_kind = kind;
    k->h.ev_used = 0;
    k->h.prof_stride = 1;
    k->h.prof_seen = 0;
    return NCL_OK;
}

int ncl_kkt_profile_stride(ncl_kkt *k, int32_t stride) {
    if (!k || stride < 1) return NCL_ERR_ARG;
    k->h.prof_stride = stride;
    k->h.prof_seen = 0;
    return NCL_OK;
}

int ncl_kkt_profile_read(ncl_kkt *k, int64_t *launches, double *total_ms) {
    if (!k) return NCL_ERR_ARG;
    Handle &h = k->h;
    double ms = 0.0;
    if (h.ev_used) {
        if (hipEventSynchronize(static_cast<hipEvent_t>(h.ev[2 * h.ev_used - 1])) != hipSuccess) return NCL_ERR_HIP;
        for (size_t i = 0; i < h.ev_used; i++) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, static_cast<hipEvent_t>(h.ev[2 * i]), static_cast<hipEvent_t>(h.ev[2 * i + 1])) !=
                hipSuccess)
                return NCL_ERR_HIP;
            ms += double(t);
        }
    }
    if (launches) *launches = int64_t(h.ev_used);
    if (total_ms) *total_ms = ms;
    return NCL_OK;
}

int ncl_kkt_solve(ncl_kkt *k, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream) {
    return do_solve(k, db, dx, nrhs, ld, stream);
}

int ncl_kkt_factor_solve(ncl_kkt *k, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream) {
    if (!k || !db || !dx || nrhs < 1) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.values_set) return NCL_ERR_STATE;
    if (nrhs > h.nrhs_max || ld < h.N) return NCL_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ncl::DevArgs a = dev_args(h);
    h.blocks_done = false;
    h.factored = false;
    h.factor_failed = false;
    // a border of fewer than kForkMinBorder rows is factored in line: its
    // work is too short to hide, and the fork and join would cost more than
    // they save
    constexpr int kForkMinBorder = 128;
    const bool fork = h.max_nbd >= kForkMinBorder;
    const ncl::LaunchArgs v = solve_args(h, db, dx, nrhs, ld, false);
    const ncl::LaunchArgs none;
    int rc = NCL_OK;
    if (!fork) {
        if ((rc = factor_levels(h, a, st))) return rc;
        if (h.nbd_tot && (rc = border_launches(h, a, true, st))) return rc;
        for (int kind : {NCL_K_STATUS_INIT, NCL_K_STATUS})
            if (run(h, kind, a, none, st) != hipSuccess) return NCL_ERR_HIP;
        if ((rc = solve_first_half(h, a, v, false, st))) return rc;
    } else if (big_border(h)) {
        // a border over the register kernel's size is the long chain (the
        // blocked factor): it runs on the side stream beside the whole
        // forward substitution, which it outlasts
        if ((rc = factor_levels(h, a, st)) || (rc = side_stream(h))) return rc;
        hipStream_t side = static_cast<hipStream_t>(h.side);
        hipEvent_t ef = static_cast<hipEvent_t>(h.ev_fork);
        if (hipEventRecord(ef, st) != hipSuccess || hipStreamWaitEvent(side, ef, 0) != hipSuccess) return NCL_ERR_HIP;
        if ((rc = border_launches(h, a, true, side))) return rc;
        for (int kind : {NCL_K_STATUS_INIT, NCL_K_STATUS})
            if (run(h, kind, a, none, side) != hipSuccess) return NCL_ERR_HIP;
        if (hipEventRecord(static_cast<hipEvent_t>(h.ev_join), side) != hipSuccess) return NCL_ERR_HIP;
        if ((rc = solve_first_half(h, a, v, false, st))) return rc;
        if (hipStreamWaitEvent(st, static_cast<hipEvent_t>(h.ev_join), 0) != hipSuccess) return NCL_ERR_HIP;
    } else {
        // a border in registers: the forward substitution of level l needs
        // the factor of levels <= l only, so it runs on the side stream a
        // level behind the factor, in the compute units the factor's upper
        // levels leave idle, and the border's Schur products, sum and dense
        // factor then have the GPU to themselves after the last level
        if ((rc = side_stream(h)) || (rc = level_events(h))) return rc;
        hipStream_t side = static_cast<hipStream_t>(h.side);
        hipEvent_t ef = static_cast<hipEvent_t>(h.ev_fork);
        if (hipEventRecord(ef, st) != hipSuccess || hipStreamWaitEvent(side, ef, 0) != hipSuccess) return NCL_ERR_HIP;
        if ((rc = solve_load(h, a, v, side))) return rc;
        const ncl::Schedule &S = h.sched;
        for (int l = 0; l < S.nlev; l++) {
            if ((rc = factor_level(h, a, l, st))) return rc;
            hipEvent_t el = static_cast<hipEvent_t>(h.ev_lev[l]);
            if (hipEventRecord(el, st) != hipSuccess || hipStreamWaitEvent(side, el, 0) != hipSuccess)
                return NCL_ERR_HIP;
            if ((rc = solve_forward_level(h, a, v, l, side))) return rc;
        }
        if ((rc = solve_border_partials(h, a, v, side))) return rc;
        if (hipEventRecord(static_cast<hipEvent_t>(h.ev_join), side) != hipSuccess) return NCL_ERR_HIP;
        if ((rc = border_launches(h, a, true, st))) return rc;
        for (int kind : {NCL_K_STATUS_INIT, NCL_K_STATUS})
            if (run(h, kind, a, none, st) != hipSuccess) return NCL_ERR_HIP;
        if (hipStreamWaitEvent(st, static_cast<hipEvent_t>(h.ev_join), 0) != hipSuccess) return NCL_ERR_HIP;
    }
    h.blocks_done = true;
    h.factored = true;
    return solve_second_half(h, a, v, st);
}

int ncl_kkt_solve_adjoint(ncl_kkt *k, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream) {
    // K = K^T: the transposed system uses the same factors and the same kernels
    return do_solve(k, db, dx, nrhs, ld, stream);
}

int ncl_kkt_backward_error(ncl_kkt *k, const double *db, const double *dx, int32_t nrhs, int64_t ld, double *derr,
                           void *stream) {
    if (!k || !db || !dx || !derr || nrhs < 1) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.values_set) return NCL_ERR_STATE;
    if (ld < h.N) return NCL_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ncl::DevArgs a = dev_args(h);
    for (int rhs = 0; rhs < nrhs; rhs++) {
        const int rc = residual_column(h, a, db + int64_t(rhs) * ld, dx + int64_t(rhs) * ld, derr + 2 * rhs, st);
        if (rc) return rc;
    }
    return NCL_OK;
}

// Doubles of residual staging one backward-error call needs: x, b and r in
// the interleaved order, r in layout order and the partial maxima, each
// rounded up to 256 bytes.
static int64_t berr_staging(const Handle &h) {
    auto up = [](int64_t n) { return (n + 31) / 32 * 32; };
    const int64_t v = up(h.dint + h.nbd_tot);
    return 3 * v + up(h.N) + up(8 * berr_partials(h));
}

int ncl_kkt_backward_error_noalloc(ncl_kkt *k, const double *db, const double *dx, int32_t nrhs, int64_t ld,
                                   double *derr, void *stream) {
    if (!k || !db || !dx || !derr || nrhs < 1) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (ld < h.N || berr_staging(h) > ncl::kScratchDoubles) return NCL_ERR_ARG;
    if (!h.bound || !h.values_set) return NCL_ERR_STATE;
    double *sc = nullptr;
    if (ncl::scratch_address(&sc) != hipSuccess) return NCL_ERR_HIP;
    auto up = [](int64_t n) { return (n + 31) / 32 * 32; };
    const int64_t v = up(h.dint + h.nbd_tot);
    ncl::DevArgs a = dev_args(h);
    a.xint = sc;
    a.bint = sc + v;
    a.rint = sc + 2 * v;
    a.rbuf = sc + 3 * v;
    a.epart = sc + 3 * v + up(h.N);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int rhs = 0; rhs < nrhs; rhs++) {
        const int rc = residual_column(h, a, db + int64_t(rhs) * ld, dx + int64_t(rhs) * ld, derr + 2 * rhs, st);
        if (rc) return rc;
    }
    return NCL_OK;
}

int ncl_kkt_refine(ncl_kkt *k, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream) {
    if (!k || !db || !dx || nrhs < 1) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.factored || h.factor_failed || !h.values_set) return NCL_ERR_STATE;
    if (nrhs > h.nrhs_max || ld < h.N) return NCL_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ncl::DevArgs a = dev_args(h);
    for (int rhs = 0; rhs < nrhs; rhs++) {
        double *x = dx + int64_t(rhs) * ld;
        int rc = residual_column(h, a, db + int64_t(rhs) * ld, x, nullptr, st);
        if (!rc) rc = solve_columns(h, a, nullptr, x, 1, ld, true, st);
        if (rc) return rc;
    }
    return NCL_OK;
}

}  // extern "C"

ncl_kkt::~ncl_kkt() {
    for (void *e : h.ev) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    for (void *e : h.ev_lev) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    if (h.ev_fork) (void)hipEventDestroy(static_cast<hipEvent_t>(h.ev_fork));
    if (h.ev_join) (void)hipEventDestroy(static_cast<hipEvent_t>(h.ev_join));
    if (h.side) (void)hipStreamDestroy(static_cast<hipStream_t>(h.side));
}
