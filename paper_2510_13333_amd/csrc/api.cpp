// C ABI of libnclkkt: handle life cycle, workspace binding, launches and the
// host-side views of the symbolic result.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <new>

#include "kernels.h"

using ncl::Handle;
using ncl::Template;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int finish_analyze(Handle &h, const ncl_analyze_opts *opts) {
    int maxw = 16, znum = 1, zden = 4;
    if (opts) {
        if (opts->relax_maxw) maxw = opts->relax_maxw;
        if (opts->relax_zden) { znum = opts->relax_znum; zden = opts->relax_zden; }
        if (maxw < 1 || zden <= 0 || znum < 0) return NCL_ERR_ARG;
    }
    for (auto &t : h.tmpl) {
        int rc = ncl::analyze_template(t, h.nbd, maxw, znum, zden);
        if (rc) return rc;
        rc = ncl::build_schedule(t, h.nbd);
        if (rc) return rc;
    }
    int rc = ncl::analyze_border(h, maxw, znum, zden);
    if (rc) return rc;
    h.nnzL = 0;
    h.nsuper = 0;
    h.npanel = 0;
    h.lbase.assign(h.nblk + 1, 0);
    for (int b = 0; b < h.nblk; b++) {
        const Template &t = h.tmpl[h.block_tmpl[b]];
        h.nnzL += t.lp[t.n];
        h.nsuper += int64_t(t.sup.size()) - 1;
        h.npanel += int64_t(t.sri.size());
        h.lbase[b + 1] = h.lbase[b] + t.panel_off.back();
    }
    if (h.nbd) {
        h.nnzL += h.blp[h.nbd];
        h.nsuper += int64_t(h.bsup.size()) - 1;
        std::vector<int32_t> mk(h.nbd, -1);
        for (size_t s = 0; s + 1 < h.bsup.size(); s++) {
            int f = h.bsup[s], l = h.bsup[s + 1] - 1;
            h.npanel += l - f + 1;
            for (int j = f; j <= l; j++)
                for (int p = h.blp[j]; p < h.blp[j + 1]; p++)
                    if (h.bli[p] > l && mk[h.bli[p]] != int(s)) { mk[h.bli[p]] = int(s); h.npanel++; }
        }
    }
    return NCL_OK;
}

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    }
};

template <class T>
size_t vbytes(const std::vector<T> &v) { return v.size() * sizeof(T); }

// All device memory the handle uses, carved from one buffer.
struct Plan {
    size_t tables_end = 0, total = 0;
    size_t kval, lpan, dval, spart, sbb, ybuf, cpart, stat, dmm;
    size_t tdev, bdev, kbb, bpg, c2, brr, brx, bprim;
    std::vector<std::vector<size_t>> toff;   // per template, per array
};

template <class T>
void stage(std::vector<uint8_t> &buf, size_t off, const std::vector<T> &v) {
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), vbytes(v));
}

Plan plan_ws(const Handle &h, int64_t nrhs) {
    Plan p;
    Layout L;
    p.toff.resize(h.tmpl.size());
    for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
        const Template &t = h.tmpl[ti];
        std::vector<size_t> &o = p.toff[ti];
        o.push_back(L.take(vbytes(t.sup)));
        o.push_back(L.take(vbytes(t.srp)));
        o.push_back(L.take(vbytes(t.sri)));
        o.push_back(L.take(vbytes(t.panel_off)));
        o.push_back(L.take(vbytes(t.lev_sup_ptr)));
        o.push_back(L.take(vbytes(t.lev_sup)));
        o.push_back(L.take(vbytes(t.lev_task_ptr)));
        o.push_back(L.take(vbytes(t.task_s)));
        o.push_back(L.take(vbytes(t.task_p)));
        o.push_back(L.take(vbytes(t.task_gptr)));
        o.push_back(L.take(vbytes(t.gitems)));
        o.push_back(L.take(vbytes(t.crel)));
        o.push_back(L.take(vbytes(t.task_aptr)));
        o.push_back(L.take(vbytes(t.aents)));
        o.push_back(L.take(vbytes(t.lev_dtask_ptr)));
        o.push_back(L.take(vbytes(t.dtask)));
        o.push_back(L.take(vbytes(t.bpath_ptr)));
        o.push_back(L.take(vbytes(t.bpath_s)));
        o.push_back(L.take(vbytes(t.bpath_pos)));
        o.push_back(L.take(vbytes(t.bus_idx)));
        o.push_back(L.take(vbytes(t.bus_slot)));
        o.push_back(L.take(vbytes(t.bus_adj_ptr)));
        o.push_back(L.take(vbytes(t.bus_adj)));
        o.push_back(L.take(vbytes(t.br_slot)));
        o.push_back(L.take(vbytes(t.br_idx)));
        o.push_back(L.take(vbytes(t.gen_idx)));
        o.push_back(L.take(vbytes(t.gen_slot)));
        o.push_back(L.take(vbytes(t.perm)));
        o.push_back(L.take(size_t(t.n)));      // col_primal
    }
    p.tdev = L.take(sizeof(ncl::TemplDev) * h.tmpl.size());
    p.bdev = L.take(sizeof(ncl::BlockDev) * size_t(h.nblk));
    p.kbb = L.take(vbytes(h.kbb_pos));
    p.bpg = L.take(vbytes(h.border_pg));
    p.c2 = L.take(vbytes(h.gen_c2));
    p.brr = L.take(vbytes(h.br_r));
    p.brx = L.take(vbytes(h.br_x));
    p.bprim = L.take(vbytes(h.border_primal));
    p.tables_end = L.off;
    const int64_t npk = int64_t(h.nbd) * (h.nbd + 1) / 2;
    p.kval = L.take(sizeof(double) * size_t(h.nnzK));
    p.lpan = L.take(sizeof(double) * size_t(h.lbase[h.nblk]));
    p.dval = L.take(sizeof(double) * size_t(h.N));
    p.spart = L.take(sizeof(double) * size_t(h.nblk) * size_t(npk));
    p.sbb = L.take(sizeof(double) * size_t(npk));
    p.ybuf = L.take(sizeof(double) * size_t(h.N) * size_t(nrhs));
    p.cpart = L.take(sizeof(double) * size_t(nrhs) * size_t(h.nblk) * size_t(h.nbd));
    p.stat = L.take(sizeof(int64_t) * 4 * size_t(h.nblk + 1));
    p.dmm = L.take(sizeof(double) * 2 * size_t(h.nblk + 1));
    p.total = L.off;
    return p;
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
        if (!rc) rc = finish_analyze(k->h, opts);
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
        if (!rc) rc = finish_analyze(k->h, opts);
        if (rc) { delete k; return rc; }
    } catch (const std::bad_alloc &) {
        delete k;
        return NCL_ERR_ALLOC;
    }
    *out = k;
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
    const int64_t bstart = h.block_off[h.nblk];
    int64_t lq = 0, sq = 0, pq = 0;
    if (lcolptr) lcolptr[0] = 0;
    if (srowptr) srowptr[0] = 0;
    for (int b = 0; b < h.nblk; b++) {
        const Template &t = h.tmpl[h.block_tmpl[b]];
        const int64_t o = h.block_off[b];
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
    std::vector<int32_t> mk(h.nbd, -1), buf;
    for (int j = 0; j < h.nbd; j++) {
        const int64_t g = bstart + j;
        if (perm) perm[g] = int32_t(g);
        if (colcount) colcount[g] = h.bcolcount[j];
        if (etree) etree[g] = h.bparent[j] >= 0 ? int32_t(bstart + h.bparent[j]) : -1;
        for (int p = h.blp[j]; p < h.blp[j + 1]; p++) {
            if (lrowind) lrowind[lq] = int32_t(bstart + h.bli[p]);
            lq++;
        }
        if (lcolptr) lcolptr[g + 1] = lq;
    }
    for (size_t s = 0; s + 1 < h.bsup.size(); s++) {
        const int f = h.bsup[s], l = h.bsup[s + 1] - 1;
        if (super_ptr) super_ptr[sq] = bstart + f;
        buf.clear();
        for (int j = f; j <= l; j++) buf.push_back(j);
        size_t c0 = buf.size();
        for (int j = f; j <= l; j++)
            for (int p = h.blp[j]; p < h.blp[j + 1]; p++)
                if (h.bli[p] > l && mk[h.bli[p]] != int(s)) { mk[h.bli[p]] = int(s); buf.push_back(h.bli[p]); }
        std::sort(buf.begin() + c0, buf.end());
        for (int32_t r : buf) {
            if (srowind) srowind[pq] = int32_t(bstart + r);
            pq++;
        }
        sq++;
        if (srowptr) srowptr[sq] = pq;
    }
    if (super_ptr) super_ptr[sq] = h.N;
    return NCL_OK;
}

int ncl_kkt_pattern(const ncl_kkt *k, int64_t *colptr, int32_t *rowind) {
    if (!k || !colptr || !rowind) return NCL_ERR_ARG;
    const Handle &h = k->h;
    const int64_t bstart = h.block_off[h.nblk];
    colptr[0] = 0;
    for (int b = 0; b < h.nblk; b++) {
        const Template &t = h.tmpl[h.block_tmpl[b]];
        const int64_t o = h.block_off[b];
        for (int c = 0; c < t.n; c++) {
            colptr[o + c + 1] = h.kbase[b] + t.colptr[c + 1];
            for (int64_t p = t.colptr[c]; p < t.colptr[c + 1]; p++) {
                int32_t r = t.rowind[p];
                rowind[h.kbase[b] + p] = int32_t(r < t.n ? o + r : bstart + (r - t.n));
            }
        }
    }
    for (int c = 0; c < h.nbd; c++) {
        colptr[bstart + c + 1] = h.kbase[h.nblk] + h.bcolptr[c + 1];
        for (int64_t p = h.bcolptr[c]; p < h.bcolptr[c + 1]; p++)
            rowind[h.kbase[h.nblk] + p] = int32_t(bstart + h.browind[p]);
    }
    return NCL_OK;
}

int ncl_kkt_workspace_bytes(const ncl_kkt *k, int32_t nrhs_max, size_t *bytes) {
    if (!k || !bytes || nrhs_max < 1) return NCL_ERR_ARG;
    *bytes = plan_ws(k->h, nrhs_max).total;
    return NCL_OK;
}

int ncl_kkt_bind_workspace(ncl_kkt *k, void *dptr, size_t bytes, int32_t nrhs_max, void *stream) {
    if (!k || !dptr || nrhs_max < 1 || (reinterpret_cast<uintptr_t>(dptr) & (kAlign - 1))) return NCL_ERR_ARG;
    Handle &h = k->h;
    Plan p = plan_ws(h, nrhs_max);
    if (bytes < p.total) return NCL_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *base = static_cast<uint8_t *>(dptr);
    std::vector<uint8_t> buf(p.tables_end, 0);
    std::vector<ncl::TemplDev> tdev(h.tmpl.size());
    for (size_t ti = 0; ti < h.tmpl.size(); ti++) {
        const Template &t = h.tmpl[ti];
        const std::vector<size_t> &o = p.toff[ti];
        int q = 0;
        auto put = [&](const auto &v) {
            stage(buf, o[q], v);
            return base + o[q++];
        };
        ncl::TemplDev &d = tdev[ti];
        d.n = t.n;
        d.nsup = int32_t(t.sup.size()) - 1;
        d.nlev = t.nlev;
        d.ntask = int32_t(t.task_s.size());
        d.nbd = h.nbd;
        d.nb = h.nb;
        d.nl = h.nl;
        d.ng = h.ng;
        d.panel_size = t.panel_off.back();
        d.pvpq_rows = t.pvpq_rows;
        d.has_pg_local = t.pg_local;
        d.sup_first = reinterpret_cast<const int32_t *>(put(t.sup));
        d.sup_rowptr = reinterpret_cast<const int32_t *>(put(t.srp));
        d.sup_rows = reinterpret_cast<const int32_t *>(put(t.sri));
        d.panel_off = reinterpret_cast<const int32_t *>(put(t.panel_off));
        d.lev_sup_ptr = reinterpret_cast<const int32_t *>(put(t.lev_sup_ptr));
        d.lev_sup = reinterpret_cast<const int32_t *>(put(t.lev_sup));
        d.lev_task_ptr = reinterpret_cast<const int32_t *>(put(t.lev_task_ptr));
        d.task_s = reinterpret_cast<const int32_t *>(put(t.task_s));
        d.task_p = reinterpret_cast<const int32_t *>(put(t.task_p));
        d.task_gptr = reinterpret_cast<const int32_t *>(put(t.task_gptr));
        d.gitems = reinterpret_cast<const ncl::GItem *>(put(t.gitems));
        d.crel = reinterpret_cast<const uint8_t *>(put(t.crel));
        d.task_aptr = reinterpret_cast<const int32_t *>(put(t.task_aptr));
        d.aents = reinterpret_cast<const ncl::AEnt *>(put(t.aents));
        d.lev_dtask_ptr = reinterpret_cast<const int32_t *>(put(t.lev_dtask_ptr));
        d.dtask = reinterpret_cast<const int32_t *>(put(t.dtask));
        d.bpath_ptr = reinterpret_cast<const int32_t *>(put(t.bpath_ptr));
        d.bpath_s = reinterpret_cast<const int32_t *>(put(t.bpath_s));
        d.bpath_pos = reinterpret_cast<const int32_t *>(put(t.bpath_pos));
        d.bus_idx = reinterpret_cast<const int32_t *>(put(t.bus_idx));
        d.bus_slot = reinterpret_cast<const int32_t *>(put(t.bus_slot));
        d.bus_adj_ptr = reinterpret_cast<const int32_t *>(put(t.bus_adj_ptr));
        d.bus_adj = reinterpret_cast<const int32_t *>(put(t.bus_adj));
        d.br_slot = reinterpret_cast<const int32_t *>(put(t.br_slot));
        d.br_idx = reinterpret_cast<const int32_t *>(put(t.br_idx));
        d.gen_idx = reinterpret_cast<const int32_t *>(put(t.gen_idx));
        d.gen_slot = reinterpret_cast<const int32_t *>(put(t.gen_slot));
        d.perm = reinterpret_cast<const int32_t *>(put(t.perm));
        std::vector<uint8_t> cp(t.n);
        for (int j = 0; j < t.n; j++) cp[j] = t.is_primal[t.perm[j]];
        d.col_primal = reinterpret_cast<const uint8_t *>(put(cp));
    }
    std::memcpy(buf.data() + p.tdev, tdev.data(), sizeof(ncl::TemplDev) * tdev.size());
    std::vector<ncl::BlockDev> bdev(h.nblk);
    for (int b = 0; b < h.nblk; b++) {
        bdev[b].tmpl = h.block_tmpl[b];
        bdev[b].outage = h.block_outage[b];
        bdev[b].col0 = h.block_off[b];
        bdev[b].kbase = h.kbase[b];
        bdev[b].lbase = h.lbase[b];
    }
    std::memcpy(buf.data() + p.bdev, bdev.data(), sizeof(ncl::BlockDev) * bdev.size());
    stage(buf, p.kbb, h.kbb_pos);
    stage(buf, p.bpg, h.border_pg);
    stage(buf, p.c2, h.gen_c2);
    stage(buf, p.brr, h.br_r);
    stage(buf, p.brx, h.br_x);
    stage(buf, p.bprim, h.border_primal);
    if (hipMemcpyAsync(base, buf.data(), buf.size(), hipMemcpyHostToDevice, st) != hipSuccess) return NCL_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return NCL_ERR_HIP;
    h.ws = dptr;
    h.ws_bytes = bytes;
    h.nrhs_max = nrhs_max;
    h.d.tmpl = reinterpret_cast<ncl::TemplDev *>(base + p.tdev);
    h.d.blk = reinterpret_cast<ncl::BlockDev *>(base + p.bdev);
    h.d.kbb_pos = reinterpret_cast<int32_t *>(base + p.kbb);
    h.d.border_pg = reinterpret_cast<int32_t *>(base + p.bpg);
    h.d.gen_c2 = reinterpret_cast<double *>(base + p.c2);
    h.d.br_g = reinterpret_cast<double *>(base + p.brr);
    h.d.br_b = reinterpret_cast<double *>(base + p.brx);
    h.d.kval = reinterpret_cast<double *>(base + p.kval);
    h.d.lpan = reinterpret_cast<double *>(base + p.lpan);
    h.d.dval = reinterpret_cast<double *>(base + p.dval);
    h.d.spart = reinterpret_cast<double *>(base + p.spart);
    h.d.sbb = reinterpret_cast<double *>(base + p.sbb);
    h.d.ybuf = reinterpret_cast<double *>(base + p.ybuf);
    h.d.cpart = reinterpret_cast<double *>(base + p.cpart);
    h.d.stat = reinterpret_cast<int64_t *>(base + p.stat);
    h.d.dmm = reinterpret_cast<double *>(base + p.dmm);
    h.bprim_dev = base + p.bprim;
    h.bound = true;
    h.factored = false;
    h.blocks_done = false;
    return NCL_OK;
}

int ncl_kkt_assemble(ncl_kkt *k, const ncl_kkt_point *pt, void *stream) {
    if (!k || !pt || !pt->z || !pt->sigma || !(pt->rho > 0)) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.from_network) return NCL_ERR_STATE;
    ncl::AsmArgs a{};
    a.tmpls = h.d.tmpl;
    a.blks = h.d.blk;
    a.nblk = h.nblk;
    a.nb = h.nb;
    a.ng = h.ng;
    a.nbd = h.nbd;
    a.z = pt->z;
    a.sig = pt->sigma;
    a.rho = pt->rho;
    a.kval = h.d.kval;
    a.kbase_border = h.kbase[h.nblk];
    a.bstart = h.block_off[h.nblk];
    a.br_r = h.d.br_g;
    a.br_x = h.d.br_b;
    a.gen_c2 = h.d.gen_c2;
    a.border_pg = h.d.border_pg;
    a.kbb_pos = h.d.kbb_pos;
    return hip_rc(ncl::launch_assemble(a, reinterpret_cast<hipStream_t>(stream)));
}

int ncl_kkt_set_values(ncl_kkt *k, const double *dvals, void *stream) {
    if (!k || !dvals) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound) return NCL_ERR_STATE;
    return hip_rc(hipMemcpyAsync(h.d.kval, dvals, sizeof(double) * size_t(h.nnzK), hipMemcpyDeviceToDevice,
                                 reinterpret_cast<hipStream_t>(stream)));
}

int ncl_kkt_get_values(ncl_kkt *k, double *dvals, void *stream) {
    if (!k || !dvals) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound) return NCL_ERR_STATE;
    return hip_rc(hipMemcpyAsync(dvals, h.d.kval, sizeof(double) * size_t(h.nnzK), hipMemcpyDeviceToDevice,
                                 reinterpret_cast<hipStream_t>(stream)));
}

static ncl::FactorArgs factor_args(Handle &h) {
    ncl::FactorArgs fa{};
    fa.tmpls = h.d.tmpl;
    fa.blks = h.d.blk;
    fa.kval = h.d.kval;
    fa.lpan = h.d.lpan;
    fa.dval = h.d.dval;
    fa.spart = h.d.spart;
    fa.stat = h.d.stat;
    fa.dminmax = h.d.dmm;
    fa.nbd = h.nbd;
    return fa;
}

static ncl::BorderArgs border_args(Handle &h) {
    ncl::BorderArgs ba{};
    ba.nblk = h.nblk;
    ba.nbd = h.nbd;
    ba.kval = h.d.kval;
    ba.kbase_border = h.kbase[h.nblk];
    ba.kbb_pos = h.d.kbb_pos;
    ba.spart = h.d.spart;
    ba.sbb = h.d.sbb;
    ba.dval = h.d.dval;
    ba.bcol0 = h.block_off[h.nblk];
    ba.bprimal = h.bprim_dev;
    ba.stat = h.d.stat;
    ba.dminmax = h.d.dmm;
    return ba;
}

int ncl_kkt_factor_blocks(ncl_kkt *k, void *stream) {
    if (!k) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound) return NCL_ERR_STATE;
    h.blocks_done = false;
    int rc = hip_rc(ncl::launch_factor_blocks(factor_args(h), h.nblk, reinterpret_cast<hipStream_t>(stream)));
    if (rc == NCL_OK) h.blocks_done = true;
    return rc;
}

int ncl_kkt_factor_border(ncl_kkt *k, void *stream) {
    if (!k) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.blocks_done) return NCL_ERR_STATE;
    int rc = hip_rc(ncl::launch_factor_border(border_args(h), reinterpret_cast<hipStream_t>(stream)));
    if (rc == NCL_OK) h.factored = true;
    return rc;
}

int ncl_kkt_factor(ncl_kkt *k, void *stream) {
    int rc = ncl_kkt_factor_blocks(k, stream);
    return rc ? rc : ncl_kkt_factor_border(k, stream);
}

int ncl_kkt_info(ncl_kkt *k, ncl_kkt_report *rep, void *stream) {
    if (!k || !rep) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.factored) return NCL_ERR_STATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nrow = h.nblk + (h.nbd ? 1 : 0);
    std::vector<int64_t> s(4 * size_t(nrow));
    std::vector<double> m(2 * size_t(nrow));
    if (hipStreamSynchronize(st) != hipSuccess) return NCL_ERR_HIP;
    if (hipMemcpy(s.data(), h.d.stat, sizeof(int64_t) * s.size(), hipMemcpyDeviceToHost) != hipSuccess) return NCL_ERR_HIP;
    if (hipMemcpy(m.data(), h.d.dmm, sizeof(double) * m.size(), hipMemcpyDeviceToHost) != hipSuccess) return NCL_ERR_HIP;
    int64_t bad = INT64_MAX;
    rep->npos = rep->nneg = rep->nzero = 0;
    rep->min_absd = INFINITY;
    rep->max_absd = 0.0;
    for (int r = 0; r < nrow; r++) {
        rep->npos += s[4 * r];
        rep->nneg += s[4 * r + 1];
        rep->nzero += s[4 * r + 2];
        bad = std::min(bad, s[4 * r + 3]);
        rep->min_absd = std::min(rep->min_absd, m[2 * r]);
        rep->max_absd = std::max(rep->max_absd, m[2 * r + 1]);
    }
    if (bad == INT64_MAX) {
        rep->first_bad = -1;
        rep->status = NCL_OK;
    } else {
        rep->first_bad = bad / 8;
        const int code = int(bad % 8);
        rep->status = code == 1 ? NCL_ERR_INERTIA : code == 2 ? NCL_ERR_ZERO_PIVOT : NCL_ERR_NONFINITE;
    }
    return NCL_OK;
}

int ncl_kkt_get_factors(ncl_kkt *k, double *lx, double *dd, void *stream) {
    if (!k) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.factored) return NCL_ERR_STATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(st) != hipSuccess) return NCL_ERR_HIP;
    if (dd && hipMemcpy(dd, h.d.dval, sizeof(double) * size_t(h.N), hipMemcpyDeviceToHost) != hipSuccess)
        return NCL_ERR_HIP;
    if (!lx) return NCL_OK;
    std::vector<double> pan(size_t(h.lbase[h.nblk]));
    const int64_t npk = int64_t(h.nbd) * (h.nbd + 1) / 2;
    std::vector<double> sbb(static_cast<size_t>(npk));
    if (!pan.empty() && hipMemcpy(pan.data(), h.d.lpan, sizeof(double) * pan.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return NCL_ERR_HIP;
    if (npk && hipMemcpy(sbb.data(), h.d.sbb, sizeof(double) * sbb.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return NCL_ERR_HIP;
    int64_t q = 0;
    for (int b = 0; b < h.nblk; b++) {
        const Template &t = h.tmpl[h.block_tmpl[b]];
        const double *P = pan.data() + h.lbase[b];
        const int ns = int(t.sup.size()) - 1;
        for (int s = 0; s < ns; s++) {
            const int f = t.sup[s], w = t.sup[s + 1] - f, r = t.srp[s + 1] - t.srp[s];
            const int32_t *R = &t.sri[t.srp[s]];
            for (int c = 0; c < w; c++) {
                const int j = f + c;
                for (int p = t.lp[j]; p < t.lp[j + 1]; p++) {
                    const int32_t row = t.li[p];
                    const int pos = int(std::lower_bound(R, R + r, row) - R);
                    lx[q++] = P[t.panel_off[s] + int64_t(c) * r + pos];
                }
            }
        }
    }
    for (int j = 0; j < h.nbd; j++)
        for (int p = h.blp[j]; p < h.blp[j + 1]; p++) {
            const int i = h.bli[p];
            lx[q++] = sbb[size_t(i) * (i + 1) / 2 + j];
        }
    return NCL_OK;
}

static int do_solve(ncl_kkt *k, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream) {
    if (!k || !db || !dx || nrhs < 1) return NCL_ERR_ARG;
    Handle &h = k->h;
    if (!h.bound || !h.factored) return NCL_ERR_STATE;
    if (nrhs > h.nrhs_max || ld < h.N) return NCL_ERR_ARG;
    ncl::SolveArgs a{};
    a.tmpls = h.d.tmpl;
    a.blks = h.d.blk;
    a.lpan = h.d.lpan;
    a.dval = h.d.dval;
    a.sbb = h.d.sbb;
    a.ybuf = h.d.ybuf;
    a.cpart = h.d.cpart;
    a.b = db;
    a.x = dx;
    a.ld = ld;
    a.N = h.N;
    a.bstart = h.block_off[h.nblk];
    a.nblk = h.nblk;
    a.nbd = h.nbd;
    a.nrhs = nrhs;
    return hip_rc(ncl::launch_solve(a, reinterpret_cast<hipStream_t>(stream)));
}

int ncl_kkt_solve(ncl_kkt *k, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream) {
    return do_solve(k, db, dx, nrhs, ld, stream);
}

int ncl_kkt_solve_adjoint(ncl_kkt *k, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream) {
    // K = K^T: the transposed system uses the same factors and the same kernels
    return do_solve(k, db, dx, nrhs, ld, stream);
}

}  // extern "C"
