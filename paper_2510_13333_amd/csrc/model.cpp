// Network model: the layout of each block template, the union sparsity
// pattern of K (lower triangle), and the tables the assembly kernel uses to
// find where each value goes.  Structure of K follows the Newton system of
// Section IV-B (blocks A, B, C) for the corrective SCOPF of Section II-B
// with the PV/PQ complementarity rows of eq. (pvpq) and the AGC droop rows
// of eq. (droopmpec).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "ncl_internal.h"

namespace ncl {

namespace {

struct Net {
    int nb, nl, ng, K;
    const int32_t *f, *t, *gb, *out;
    bool pvpq, screen, agc;
};

// template kinds; the screening ones are contingency blocks whose first-stage
// variables (pg, and vm0 with PV/PQ rows) are fixed, so they have no border.
// Any contingency kind may also carry the AGC droop rows (TemplKind::agc).
enum { T_SINGLE, T_PLAIN, T_PVPQ_BASE, T_PVPQ_CONT, T_SCREEN_PLAIN, T_SCREEN_PVPQ };

struct TemplKind {
    int kind;
    bool agc;
};

struct Local {
    std::vector<int32_t> vm, va, qg, pg, nup, num, sup, slo, vm0, rP, rQ, rFf, rFt, rLin, rDup, rDlo, rCup, rClo;
    // AGC rows: pg holds the block's own pgk and pg0 the first-stage pg
    std::vector<int32_t> pg0, pip, pim, spu, spl, rAlin, rAdup, rAdlo, rAcup, rAclo;
    int32_t delta = -1;
};

using PairList = std::vector<std::pair<int32_t, int32_t>>;   // (row, col), row >= col

void add_pair(PairList &tp, PairList &bp, int n, int32_t a, int32_t b) {
    if (a < 0 || b < 0) return;        // a fixed (screening) first-stage variable
    int32_t r = std::max(a, b), c = std::min(a, b);
    if (c >= n) bp.emplace_back(r - n, c - n);
    else tp.emplace_back(r, c);
}

void layout(const Net &net, TemplKind tk, Local &L, int &n, int &nprim, std::vector<uint8_t> &isprim) {
    const int nb = net.nb, nl = net.nl, ng = net.ng;
    const int kind = tk.kind;
    const bool agc = tk.agc;
    std::vector<int> genat(nb, -1);
    for (int g = 0; g < ng; g++) genat[net.gb[g]] = g;
    const bool base_pvpq = kind == T_PVPQ_BASE, cont_pvpq = kind == T_PVPQ_CONT || kind == T_SCREEN_PVPQ;
    const bool screen = kind == T_SCREEN_PLAIN || kind == T_SCREEN_PVPQ;
    nprim = (base_pvpq ? nb - ng : nb) + nb + ng + (kind == T_SINGLE ? ng : 0) + (cont_pvpq ? 4 * ng : 0) +
            (agc ? 5 * ng + 1 : 0);
    int ndual = 2 * nb + 2 * nl + (cont_pvpq ? 5 * ng : 0) + (agc ? 5 * ng : 0);
    n = nprim + ndual;
    const int bpg = n, bvm0 = n + ng;   // border local indices
    int k = 0;
    L.vm.assign(nb, -1);
    for (int i = 0; i < nb; i++) {
        if (base_pvpq && genat[i] >= 0) L.vm[i] = bvm0 + genat[i];
        else L.vm[i] = k++;
    }
    auto seq = [&](std::vector<int32_t> &v, int cnt) {
        v.resize(cnt);
        for (int i = 0; i < cnt; i++) v[i] = k++;
    };
    seq(L.va, nb);
    seq(L.qg, ng);
    if (kind == T_SINGLE) seq(L.pg, ng);
    else {
        L.pg.resize(ng);
        for (int g = 0; g < ng; g++) L.pg[g] = screen ? -1 : bpg + g;
    }
    if (cont_pvpq) { seq(L.nup, ng); seq(L.num, ng); seq(L.sup, ng); seq(L.slo, ng); }
    if (agc) {
        L.pg0 = L.pg;
        seq(L.pg, ng);
        seq(L.pip, ng); seq(L.pim, ng); seq(L.spu, ng); seq(L.spl, ng);
        L.delta = k++;
    }
    L.vm0.resize(ng);
    for (int g = 0; g < ng; g++) L.vm0[g] = net.pvpq && !screen ? bvm0 + g : -1;
    seq(L.rP, nb); seq(L.rQ, nb); seq(L.rFf, nl); seq(L.rFt, nl);
    if (cont_pvpq) { seq(L.rLin, ng); seq(L.rDup, ng); seq(L.rDlo, ng); seq(L.rCup, ng); seq(L.rClo, ng); }
    if (agc) { seq(L.rAlin, ng); seq(L.rAdup, ng); seq(L.rAdlo, ng); seq(L.rAcup, ng); seq(L.rAclo, ng); }
    isprim.assign(n, 0);
    for (int i = 0; i < nprim; i++) isprim[i] = 1;
}

void enumerate(const Net &net, TemplKind tk, const Local &L, int n, PairList &tp, PairList &bp) {
    const int nb = net.nb, nl = net.nl, ng = net.ng;
    const int kind = tk.kind;
    for (int l = 0; l < nl; l++) {
        int f = net.f[l], t = net.t[l];
        int32_t V[4] = {L.vm[f], L.vm[t], L.va[f], L.va[t]};
        for (int a = 0; a < 4; a++)
            for (int b = a; b < 4; b++) add_pair(tp, bp, n, V[a], V[b]);
        int32_t R[6] = {L.rP[f], L.rQ[f], L.rP[t], L.rQ[t], L.rFf[l], L.rFt[l]};
        for (int r = 0; r < 6; r++)
            for (int a = 0; a < 4; a++) add_pair(tp, bp, n, R[r], V[a]);
        add_pair(tp, bp, n, L.rFf[l], L.rFf[l]);
        add_pair(tp, bp, n, L.rFt[l], L.rFt[l]);
    }
    for (int i = 0; i < nb; i++) {
        add_pair(tp, bp, n, L.vm[i], L.vm[i]);
        add_pair(tp, bp, n, L.va[i], L.va[i]);
        add_pair(tp, bp, n, L.rP[i], L.rP[i]);
        add_pair(tp, bp, n, L.rQ[i], L.rQ[i]);
    }
    for (int g = 0; g < ng; g++) {
        int i = net.gb[g];
        add_pair(tp, bp, n, L.rP[i], L.pg[g]);
        add_pair(tp, bp, n, L.rQ[i], L.qg[g]);
        add_pair(tp, bp, n, L.qg[g], L.qg[g]);
        if (kind == T_SINGLE) add_pair(tp, bp, n, L.pg[g], L.pg[g]);
        if (kind == T_PVPQ_CONT || kind == T_SCREEN_PVPQ) {
            add_pair(tp, bp, n, L.rLin[g], L.nup[g]);
            add_pair(tp, bp, n, L.rLin[g], L.num[g]);
            add_pair(tp, bp, n, L.rLin[g], L.vm[i]);
            add_pair(tp, bp, n, L.rLin[g], L.vm0[g]);
            add_pair(tp, bp, n, L.rDup[g], L.sup[g]);
            add_pair(tp, bp, n, L.rDup[g], L.qg[g]);
            add_pair(tp, bp, n, L.rDlo[g], L.slo[g]);
            add_pair(tp, bp, n, L.rDlo[g], L.qg[g]);
            add_pair(tp, bp, n, L.rCup[g], L.num[g]);
            add_pair(tp, bp, n, L.rCup[g], L.sup[g]);
            add_pair(tp, bp, n, L.rClo[g], L.nup[g]);
            add_pair(tp, bp, n, L.rClo[g], L.slo[g]);
            add_pair(tp, bp, n, L.num[g], L.sup[g]);
            add_pair(tp, bp, n, L.nup[g], L.slo[g]);
            for (auto v : {L.nup[g], L.num[g], L.sup[g], L.slo[g], L.rLin[g], L.rDup[g], L.rDlo[g], L.rCup[g], L.rClo[g]})
                add_pair(tp, bp, n, v, v);
        }
        if (tk.agc) {
            add_pair(tp, bp, n, L.rAlin[g], L.pip[g]);
            add_pair(tp, bp, n, L.rAlin[g], L.pim[g]);
            add_pair(tp, bp, n, L.rAlin[g], L.pg[g]);
            add_pair(tp, bp, n, L.rAlin[g], L.pg0[g]);
            add_pair(tp, bp, n, L.rAlin[g], L.delta);
            add_pair(tp, bp, n, L.rAdup[g], L.spu[g]);
            add_pair(tp, bp, n, L.rAdup[g], L.pg[g]);
            add_pair(tp, bp, n, L.rAdlo[g], L.spl[g]);
            add_pair(tp, bp, n, L.rAdlo[g], L.pg[g]);
            add_pair(tp, bp, n, L.rAcup[g], L.pim[g]);
            add_pair(tp, bp, n, L.rAcup[g], L.spu[g]);
            add_pair(tp, bp, n, L.rAclo[g], L.pip[g]);
            add_pair(tp, bp, n, L.rAclo[g], L.spl[g]);
            add_pair(tp, bp, n, L.pim[g], L.spu[g]);
            add_pair(tp, bp, n, L.pip[g], L.spl[g]);
            for (auto v : {L.pg[g], L.pip[g], L.pim[g], L.spu[g], L.spl[g], L.rAlin[g], L.rAdup[g], L.rAdlo[g],
                           L.rAcup[g], L.rAclo[g]})
                add_pair(tp, bp, n, v, v);
        }
    }
    if (tk.agc) add_pair(tp, bp, n, L.delta, L.delta);
}

void to_csc(PairList &p, int ncol, std::vector<int64_t> &colptr, std::vector<int32_t> &rowind) {
    std::sort(p.begin(), p.end(), [](const auto &a, const auto &b) {
        return a.second != b.second ? a.second < b.second : a.first < b.first;
    });
    p.erase(std::unique(p.begin(), p.end()), p.end());
    colptr.assign(ncol + 1, 0);
    rowind.resize(p.size());
    for (size_t e = 0; e < p.size(); e++) {
        colptr[p[e].second + 1]++;
        rowind[e] = p[e].first;
    }
    for (int c = 0; c < ncol; c++) colptr[c + 1] += colptr[c];
}

int32_t find_pos(const std::vector<int64_t> &cp, const std::vector<int32_t> &ri, int32_t r, int32_t c) {
    auto b = ri.begin() + cp[c], e = ri.begin() + cp[c + 1];
    auto it = std::lower_bound(b, e, r);
    if (it == e || *it != r) return -1;
    return int32_t(it - ri.begin());
}

}  // namespace

int build_network_model(const ncl_network *nw, Handle &h, std::string &err) {
    if (!nw || nw->nbus < 1 || nw->nbranch < 0 || nw->ngen < 0 || nw->ncont < 0) { err = "bad sizes"; return NCL_ERR_ARG; }
    if (!nw->br_from || !nw->br_to || !nw->br_r || !nw->br_x || (nw->ngen && (!nw->gen_bus || !nw->gen_c2)) ||
        (nw->ncont && !nw->outage)) { err = "null array"; return NCL_ERR_ARG; }
    Net net{nw->nbus, nw->nbranch, nw->ngen, nw->ncont, nw->br_from, nw->br_to, nw->gen_bus, nw->outage,
            (nw->flags & NCL_PVPQ) != 0, (nw->flags & NCL_SCREEN) != 0, (nw->flags & NCL_AGC) != 0};
    if (net.pvpq && net.K == 0) { err = "PV/PQ rows need contingencies"; return NCL_ERR_ARG; }
    if (net.agc && net.K == 0) { err = "AGC rows need contingencies"; return NCL_ERR_ARG; }
    if (net.agc && net.ng && !nw->gen_alpha) { err = "AGC rows need participation factors"; return NCL_ERR_ARG; }
    if (net.agc)
        for (int g = 0; g < net.ng; g++)
            if (!std::isfinite(nw->gen_alpha[g])) { err = "participation factor not finite"; return NCL_ERR_ARG; }
    if (net.screen && net.K == 0) { err = "screening needs contingencies"; return NCL_ERR_ARG; }
    for (int l = 0; l < net.nl; l++) {
        if (net.f[l] < 0 || net.t[l] >= net.nb || net.f[l] >= net.t[l]) { err = "branch endpoints"; return NCL_ERR_ARG; }
        if (l && (net.f[l] < net.f[l - 1] || (net.f[l] == net.f[l - 1] && net.t[l] <= net.t[l - 1]))) {
            err = "branches not sorted or duplicated";
            return NCL_ERR_ARG;
        }
        if (!(nw->br_r[l] * nw->br_r[l] + nw->br_x[l] * nw->br_x[l] > 0)) { err = "zero impedance"; return NCL_ERR_ARG; }
    }
    {
        std::vector<char> used(net.nb, 0);
        for (int g = 0; g < net.ng; g++) {
            if (net.gb[g] < 0 || net.gb[g] >= net.nb || used[net.gb[g]]) { err = "generator buses"; return NCL_ERR_ARG; }
            used[net.gb[g]] = 1;
        }
    }
    {
        std::vector<char> used(net.nl, 0);
        for (int k = 0; k < net.K; k++) {
            if (net.out[k] < 0 || net.out[k] >= net.nl || used[net.out[k]]) { err = "outage index"; return NCL_ERR_ARG; }
            used[net.out[k]] = 1;
        }
    }
    // append one instance: its templates, blocks and border
    h.from_network = true;
    h.inst.emplace_back();
    Inst &I = h.inst.back();
    I.nb = net.nb; I.nl = net.nl; I.ng = net.ng; I.flags = nw->flags;
    I.blk0 = h.nblk;
    I.nblk = net.screen ? net.K : net.K + 1;
    I.nbd = net.K == 0 || net.screen ? 0 : net.ng * (net.pvpq ? 2 : 1);
    I.gen_c2.assign(nw->gen_c2, nw->gen_c2 + net.ng);
    if (net.agc) I.gen_alpha.assign(nw->gen_alpha, nw->gen_alpha + net.ng);
    else I.gen_alpha.assign(net.ng, 0.0);
    I.br_r.assign(nw->br_r, nw->br_r + net.nl);
    I.br_x.assign(nw->br_x, nw->br_x + net.nl);
    std::vector<TemplKind> kinds;
    if (net.screen) kinds = {{net.pvpq ? T_SCREEN_PVPQ : T_SCREEN_PLAIN, net.agc}};
    else if (net.K == 0) kinds = {{T_SINGLE, false}};
    else if (!net.pvpq) {
        // the base and contingency blocks share one template unless the
        // contingencies carry AGC rows
        if (net.agc) kinds = {{T_PLAIN, false}, {T_PLAIN, true}};
        else kinds = {{T_PLAIN, false}};
    } else kinds = {{T_PVPQ_BASE, false}, {T_PVPQ_CONT, net.agc}};
    const int t0 = int(h.tmpl.size());
    I.t0 = t0;
    I.nt = int(kinds.size());
    h.tmpl.resize(t0 + kinds.size());
    for (int k = 0; k < I.nblk; k++) {
        // screening: block k is contingency k; otherwise block 0 is the base case
        h.block_tmpl.push_back(t0 + (k > 0 && kinds.size() > 1 ? 1 : 0));
        h.block_outage.push_back(net.screen ? net.out[k] : k > 0 ? net.out[k - 1] : -1);
        h.block_inst.push_back(int32_t(h.inst.size() - 1));
    }
    h.nblk += I.nblk;
    PairList border_pairs;
    std::vector<Local> locs(kinds.size());
    for (size_t q = 0; q < kinds.size(); q++) {
        Template &t = h.tmpl[t0 + q];
        int n, nprim;
        layout(net, kinds[q], locs[q], n, nprim, t.is_primal);
        t.inst = int(h.inst.size()) - 1;
        t.n = n;
        t.nprim = nprim;
        t.pvpq_rows = kinds[q].kind == T_PVPQ_CONT || kinds[q].kind == T_SCREEN_PVPQ;
        t.pg_local = kinds[q].kind == T_SINGLE;
        t.agc_rows = kinds[q].agc;
        PairList tp;
        enumerate(net, kinds[q], locs[q], n, tp, border_pairs);
        to_csc(tp, n, t.colptr, t.rowind);
    }
    for (int b = 0; b < I.nbd; b++) border_pairs.emplace_back(b, b);
    to_csc(border_pairs, I.nbd, I.bcolptr, I.browind);
    I.border_primal.assign(I.nbd, 1);
    I.border_pg.assign(net.ng, -1);
    if (I.nbd)
        for (int g = 0; g < net.ng; g++) I.border_pg[g] = g;
    // global columns and public CSC positions (layout order: the blocks, then the border)
    I.col0 = h.N;
    int64_t col = h.N;
    for (int k = I.blk0; k < h.nblk; k++) {
        const Template &t = h.tmpl[h.block_tmpl[k]];
        h.block_col0.push_back(col);
        h.kbase.push_back(h.nnzK);
        col += t.n;
        h.nnzK += t.colptr[t.n];
        I.nprimal += t.nprim;
    }
    I.bstart = col;
    I.kcsc_border = h.nnzK;
    I.N = col + I.nbd - I.col0;
    I.nprimal += I.nbd;
    h.N += I.N;
    h.nnzK += I.nbb();
    h.nprimal += I.nprimal;
    I.kbb_pos.assign(size_t(I.nbd) * I.nbd, -1);
    for (int c = 0; c < I.nbd; c++)
        for (int64_t p = I.bcolptr[c]; p < I.bcolptr[c + 1]; p++) I.kbb_pos[size_t(I.browind[p]) * I.nbd + c] = int32_t(p);

    // assembly tables
    for (size_t q = 0; q < kinds.size(); q++) {
        Template &t = h.tmpl[t0 + q];
        const Local &L = locs[q];
        const int n = t.n;
        auto slot = [&](int32_t a, int32_t b) -> int32_t {
            if (a < 0 || b < 0) return -1;
            int32_t r = std::max(a, b), c = std::min(a, b);
            if (c >= n) {
                int32_t p = find_pos(I.bcolptr, I.browind, r - n, c - n);
                return p < 0 ? -1 : (kBorderFlag | p);
            }
            return find_pos(t.colptr, t.rowind, r, c);
        };
        const int nb = net.nb, nl = net.nl, ng = net.ng;
        t.bus_idx.assign(size_t(nb) * BI_N, -1);
        t.bus_slot.assign(size_t(nb) * BS_N, -1);
        for (int i = 0; i < nb; i++) {
            int32_t *bi = &t.bus_idx[size_t(i) * BI_N];
            bi[BI_VM] = L.vm[i]; bi[BI_VA] = L.va[i]; bi[BI_P] = L.rP[i]; bi[BI_Q] = L.rQ[i];
            int32_t *bs = &t.bus_slot[size_t(i) * BS_N];
            bs[BS_VMVM] = slot(L.vm[i], L.vm[i]);
            bs[BS_VAVA] = slot(L.va[i], L.va[i]);
            bs[BS_VMVA] = slot(L.vm[i], L.va[i]);
            bs[BS_PVM] = slot(L.rP[i], L.vm[i]);
            bs[BS_PVA] = slot(L.rP[i], L.va[i]);
            bs[BS_QVM] = slot(L.rQ[i], L.vm[i]);
            bs[BS_QVA] = slot(L.rQ[i], L.va[i]);
            bs[BS_PP] = slot(L.rP[i], L.rP[i]);
            bs[BS_QQ] = slot(L.rQ[i], L.rQ[i]);
        }
        t.bus_adj_ptr.assign(nb + 1, 0);
        for (int l = 0; l < nl; l++) { t.bus_adj_ptr[net.f[l] + 1]++; t.bus_adj_ptr[net.t[l] + 1]++; }
        for (int i = 0; i < nb; i++) t.bus_adj_ptr[i + 1] += t.bus_adj_ptr[i];
        t.bus_adj.assign(t.bus_adj_ptr[nb], 0);
        {
            std::vector<int32_t> fill(t.bus_adj_ptr.begin(), t.bus_adj_ptr.end() - 1);
            for (int l = 0; l < nl; l++) {
                t.bus_adj[fill[net.f[l]]++] = l;
                t.bus_adj[fill[net.t[l]]++] = ~l;
            }
        }
        t.br_slot.assign(size_t(nl) * LS_N, -1);
        t.br_idx.assign(size_t(nl) * 4, -1);
        for (int l = 0; l < nl; l++) {
            int f = net.f[l], tt = net.t[l];
            int32_t *s = &t.br_slot[size_t(l) * LS_N];
            s[LS_VMVM] = slot(L.vm[f], L.vm[tt]);
            s[LS_VMVA] = slot(L.vm[f], L.va[tt]);
            s[LS_VAVM] = slot(L.va[f], L.vm[tt]);
            s[LS_VAVA] = slot(L.va[f], L.va[tt]);
            s[LS_PF_VMT] = slot(L.rP[f], L.vm[tt]);
            s[LS_PF_VAT] = slot(L.rP[f], L.va[tt]);
            s[LS_QF_VMT] = slot(L.rQ[f], L.vm[tt]);
            s[LS_QF_VAT] = slot(L.rQ[f], L.va[tt]);
            s[LS_PT_VMF] = slot(L.rP[tt], L.vm[f]);
            s[LS_PT_VAF] = slot(L.rP[tt], L.va[f]);
            s[LS_QT_VMF] = slot(L.rQ[tt], L.vm[f]);
            s[LS_QT_VAF] = slot(L.rQ[tt], L.va[f]);
            s[LS_FF_VMF] = slot(L.rFf[l], L.vm[f]);
            s[LS_FF_VMT] = slot(L.rFf[l], L.vm[tt]);
            s[LS_FF_VAF] = slot(L.rFf[l], L.va[f]);
            s[LS_FF_VAT] = slot(L.rFf[l], L.va[tt]);
            s[LS_FT_VMF] = slot(L.rFt[l], L.vm[f]);
            s[LS_FT_VMT] = slot(L.rFt[l], L.vm[tt]);
            s[LS_FT_VAF] = slot(L.rFt[l], L.va[f]);
            s[LS_FT_VAT] = slot(L.rFt[l], L.va[tt]);
            s[LS_FFFF] = slot(L.rFf[l], L.rFf[l]);
            s[LS_FTFT] = slot(L.rFt[l], L.rFt[l]);
            int32_t *bi = &t.br_idx[size_t(l) * 4];
            bi[0] = L.rFf[l]; bi[1] = L.rFt[l]; bi[2] = f; bi[3] = tt;
        }
        t.bus_gen.assign(nb, -1);
        for (int g = 0; g < ng; g++) t.bus_gen[net.gb[g]] = g;
        t.lkind.assign(n, LK_OTHER);
        auto kind = [&](const std::vector<int32_t> &v, LocalKind k) {
            for (int32_t x : v)
                if (x >= 0 && x < n) t.lkind[x] = k;
        };
        kind(L.vm, LK_VM);
        kind(L.va, LK_VA);
        kind(L.qg, LK_QG);
        kind(L.pg, LK_PG);
        kind(L.rP, LK_ROWP);
        kind(L.rQ, LK_ROWQ);
        kind(L.rFf, LK_FLOW);
        kind(L.rFt, LK_FLOW);
        kind(L.nup, LK_NUP);
        kind(L.num, LK_NUM);
        kind(L.sup, LK_SUP);
        kind(L.slo, LK_SLO);
        kind(L.rLin, LK_LIN);
        kind(L.rDup, LK_DUP);
        kind(L.rDlo, LK_DLO);
        kind(L.rCup, LK_CUP);
        kind(L.rClo, LK_CLO);
        if (t.agc_rows) {
            kind(L.pg, LK_PGK);
            kind(L.pip, LK_PIP);
            kind(L.pim, LK_PIM);
            kind(L.spu, LK_SPU);
            kind(L.spl, LK_SPL);
            kind({L.delta}, LK_DELTA);
            kind(L.rAlin, LK_ALIN);
            kind(L.rAdup, LK_ADUP);
            kind(L.rAdlo, LK_ADLO);
            kind(L.rAcup, LK_ACUP);
            kind(L.rAclo, LK_ACLO);
        }
        t.gen_idx.assign(size_t(ng) * GI_N, -1);
        t.gen_slot.assign(size_t(ng) * GS_N, -1);
        for (int g = 0; g < ng; g++) {
            int i = net.gb[g];
            int32_t *gi = &t.gen_idx[size_t(g) * GI_N];
            gi[GI_BUS] = i;
            gi[GI_QG] = L.qg[g];
            gi[GI_PG] = L.pg[g];
            gi[GI_VM0] = L.vm0[g];
            int32_t *gs = &t.gen_slot[size_t(g) * GS_N];
            gs[GS_PPG] = slot(L.rP[i], L.pg[g]);
            gs[GS_QQG] = slot(L.rQ[i], L.qg[g]);
            gs[GS_QGQG] = slot(L.qg[g], L.qg[g]);
            gs[GS_PGPG] = t.pg_local ? slot(L.pg[g], L.pg[g]) : -1;
            if (t.pvpq_rows) {
                gi[GI_NUP] = L.nup[g]; gi[GI_NUM] = L.num[g]; gi[GI_SUP] = L.sup[g]; gi[GI_SLO] = L.slo[g];
                gi[GI_LIN] = L.rLin[g]; gi[GI_DUP] = L.rDup[g]; gi[GI_DLO] = L.rDlo[g];
                gi[GI_CUP] = L.rCup[g]; gi[GI_CLO] = L.rClo[g];
                gs[GS_LIN_NUP] = slot(L.rLin[g], L.nup[g]);
                gs[GS_LIN_NUM] = slot(L.rLin[g], L.num[g]);
                gs[GS_LIN_VM] = slot(L.rLin[g], L.vm[i]);
                gs[GS_LIN_VM0] = slot(L.rLin[g], L.vm0[g]);
                gs[GS_DUP_SUP] = slot(L.rDup[g], L.sup[g]);
                gs[GS_DUP_QG] = slot(L.rDup[g], L.qg[g]);
                gs[GS_DLO_SLO] = slot(L.rDlo[g], L.slo[g]);
                gs[GS_DLO_QG] = slot(L.rDlo[g], L.qg[g]);
                gs[GS_CUP_NUM] = slot(L.rCup[g], L.num[g]);
                gs[GS_CUP_SUP] = slot(L.rCup[g], L.sup[g]);
                gs[GS_CLO_NUP] = slot(L.rClo[g], L.nup[g]);
                gs[GS_CLO_SLO] = slot(L.rClo[g], L.slo[g]);
                gs[GS_H_NUM_SUP] = slot(L.num[g], L.sup[g]);
                gs[GS_H_NUP_SLO] = slot(L.nup[g], L.slo[g]);
                gs[GS_NUPNUP] = slot(L.nup[g], L.nup[g]);
                gs[GS_NUMNUM] = slot(L.num[g], L.num[g]);
                gs[GS_SUPSUP] = slot(L.sup[g], L.sup[g]);
                gs[GS_SLOSLO] = slot(L.slo[g], L.slo[g]);
                gs[GS_LL] = slot(L.rLin[g], L.rLin[g]);
                gs[GS_UU] = slot(L.rDup[g], L.rDup[g]);
                gs[GS_DD] = slot(L.rDlo[g], L.rDlo[g]);
                gs[GS_CUCU] = slot(L.rCup[g], L.rCup[g]);
                gs[GS_CLCL] = slot(L.rClo[g], L.rClo[g]);
            }
            if (t.agc_rows) {
                gi[GI_PIP] = L.pip[g]; gi[GI_PIM] = L.pim[g]; gi[GI_SPU] = L.spu[g]; gi[GI_SPL] = L.spl[g];
                gi[GI_ALIN] = L.rAlin[g]; gi[GI_ADUP] = L.rAdup[g]; gi[GI_ADLO] = L.rAdlo[g];
                gi[GI_ACUP] = L.rAcup[g]; gi[GI_ACLO] = L.rAclo[g]; gi[GI_DELTA] = L.delta;
                gi[GI_PG0] = L.pg0[g];
                gs[GS_ALIN_PIP] = slot(L.rAlin[g], L.pip[g]);
                gs[GS_ALIN_PIM] = slot(L.rAlin[g], L.pim[g]);
                gs[GS_ALIN_PGK] = slot(L.rAlin[g], L.pg[g]);
                gs[GS_ALIN_PG0] = slot(L.rAlin[g], L.pg0[g]);
                gs[GS_ALIN_DEL] = slot(L.rAlin[g], L.delta);
                gs[GS_ADUP_SPU] = slot(L.rAdup[g], L.spu[g]);
                gs[GS_ADUP_PGK] = slot(L.rAdup[g], L.pg[g]);
                gs[GS_ADLO_SPL] = slot(L.rAdlo[g], L.spl[g]);
                gs[GS_ADLO_PGK] = slot(L.rAdlo[g], L.pg[g]);
                gs[GS_ACUP_PIM] = slot(L.rAcup[g], L.pim[g]);
                gs[GS_ACUP_SPU] = slot(L.rAcup[g], L.spu[g]);
                gs[GS_ACLO_PIP] = slot(L.rAclo[g], L.pip[g]);
                gs[GS_ACLO_SPL] = slot(L.rAclo[g], L.spl[g]);
                gs[GS_H_PIM_SPU] = slot(L.pim[g], L.spu[g]);
                gs[GS_H_PIP_SPL] = slot(L.pip[g], L.spl[g]);
                gs[GS_PIPPIP] = slot(L.pip[g], L.pip[g]);
                gs[GS_PIMPIM] = slot(L.pim[g], L.pim[g]);
                gs[GS_SPUSPU] = slot(L.spu[g], L.spu[g]);
                gs[GS_SPLSPL] = slot(L.spl[g], L.spl[g]);
                gs[GS_PGKPGK] = slot(L.pg[g], L.pg[g]);
                gs[GS_AL] = slot(L.rAlin[g], L.rAlin[g]);
                gs[GS_AU] = slot(L.rAdup[g], L.rAdup[g]);
                gs[GS_AD] = slot(L.rAdlo[g], L.rAdlo[g]);
                gs[GS_ACUACU] = slot(L.rAcup[g], L.rAcup[g]);
                gs[GS_ACLACL] = slot(L.rAclo[g], L.rAclo[g]);
                gs[GS_DELDEL] = g == 0 ? slot(L.delta, L.delta) : -1;
            }
        }
    }
    return NCL_OK;
}

int build_pattern_model(int64_t N, int nblk, const int64_t *block_off, const int64_t *colptr, const int32_t *rowind,
                        const uint8_t *is_primal, Handle &h, std::string &err) {
    if (N <= 0 || nblk <= 0 || !block_off || !colptr || !rowind || !is_primal) { err = "bad arguments"; return NCL_ERR_ARG; }
    if (block_off[0] != 0 || block_off[nblk] > N) { err = "block offsets"; return NCL_ERR_ARG; }
    for (int b = 0; b < nblk; b++)
        if (block_off[b + 1] <= block_off[b]) { err = "empty block"; return NCL_ERR_ARG; }
    const int64_t bstart = block_off[nblk];
    if (N - bstart > NCL_MAX_BORDER) { err = "border too large"; return NCL_ERR_ARG; }
    h.from_network = false;
    h.inst.assign(1, Inst());
    Inst &I = h.inst[0];
    I.blk0 = 0;
    I.nblk = nblk;
    I.nbd = int(N - bstart);
    I.col0 = 0;
    I.N = N;
    I.bstart = bstart;
    h.nblk = nblk;
    h.block_col0.assign(block_off, block_off + nblk);
    h.block_outage.assign(nblk, -1);
    h.block_tmpl.assign(nblk, -1);
    h.block_inst.assign(nblk, 0);
    h.kbase.assign(nblk, 0);
    h.N = N;
    // validate the pattern: lower, sorted, diagonal present, no block coupling
    for (int64_t j = 0; j < N; j++) {
        if (colptr[j + 1] < colptr[j]) { err = "colptr"; return NCL_ERR_ARG; }
        bool diag = false;
        int bj = -1;
        for (int b = 0; b < nblk; b++)
            if (j >= block_off[b] && j < block_off[b + 1]) bj = b;
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int64_t i = rowind[p];
            if (i < j || i >= N || (p > colptr[j] && rowind[p - 1] >= i)) { err = "pattern not lower/sorted"; return NCL_ERR_ARG; }
            if (i == j) diag = true;
            if (bj >= 0 && i < bstart && (i < block_off[bj] || i >= block_off[bj + 1])) { err = "entry couples two blocks"; return NCL_ERR_ARG; }
        }
        if (!diag) { err = "missing diagonal"; return NCL_ERR_ARG; }
    }
    // templates: blocks with identical local patterns and signs share one
    for (int b = 0; b < nblk; b++) {
        int64_t o = block_off[b];
        int n = int(block_off[b + 1] - o);
        Template cand;
        cand.n = n;
        cand.colptr.assign(n + 1, 0);
        for (int c = 0; c < n; c++) cand.colptr[c + 1] = cand.colptr[c] + (colptr[o + c + 1] - colptr[o + c]);
        cand.rowind.resize(cand.colptr[n]);
        for (int c = 0; c < n; c++)
            for (int64_t p = colptr[o + c]; p < colptr[o + c + 1]; p++) {
                int64_t i = rowind[p];
                cand.rowind[cand.colptr[c] + (p - colptr[o + c])] = int32_t(i >= bstart ? n + (i - bstart) : i - o);
            }
        cand.is_primal.assign(is_primal + o, is_primal + o + n);
        int found = -1;
        for (size_t ti = 0; ti < h.tmpl.size() && found < 0; ti++) {
            const Template &t = h.tmpl[ti];
            if (t.n == n && t.colptr == cand.colptr && t.rowind == cand.rowind && t.is_primal == cand.is_primal) found = int(ti);
        }
        if (found < 0) {
            cand.nprim = 0;
            for (int c = 0; c < n; c++) cand.nprim += cand.is_primal[c];
            h.tmpl.push_back(std::move(cand));
            found = int(h.tmpl.size()) - 1;
        }
        h.block_tmpl[b] = found;
        h.kbase[b] = colptr[o];
    }
    I.t0 = 0;
    I.nt = int(h.tmpl.size());
    I.bcolptr.assign(I.nbd + 1, 0);
    for (int c = 0; c < I.nbd; c++) I.bcolptr[c + 1] = I.bcolptr[c] + (colptr[bstart + c + 1] - colptr[bstart + c]);
    I.browind.resize(I.bcolptr[I.nbd]);
    for (int c = 0; c < I.nbd; c++)
        for (int64_t p = colptr[bstart + c]; p < colptr[bstart + c + 1]; p++)
            I.browind[I.bcolptr[c] + (p - colptr[bstart + c])] = int32_t(rowind[p] - bstart);
    I.border_primal.assign(is_primal + bstart, is_primal + N);
    I.kcsc_border = colptr[bstart];
    h.nnzK = colptr[N];
    h.nprimal = 0;
    for (int64_t j = 0; j < N; j++) h.nprimal += is_primal[j] ? 1 : 0;
    I.nprimal = h.nprimal;
    I.kbb_pos.assign(size_t(I.nbd) * I.nbd, -1);
    for (int c = 0; c < I.nbd; c++)
        for (int64_t p = I.bcolptr[c]; p < I.bcolptr[c + 1]; p++) I.kbb_pos[size_t(I.browind[p]) * I.nbd + c] = int32_t(p);
    return NCL_OK;
}

}  // namespace ncl
