// Device kernels of libnclkkt (gfx950, FP64, wave64).
//
// Blocks that share a template run the same schedule, one block per lane:
// every address a wavefront computes is uniform (scalar loads of the
// schedule) plus the lane's block offset, and the numeric arrays are stored
// interleaved across the template's blocks, so that each vector load moves
// 64 consecutive doubles.  Each launch processes one work list (one
// wavefront per item); the dependency levels of the supernodal tree are
// separated by kernel boundaries.
//
//   assemble            K from the state (Section IV-B blocks A, B, C)
//   fac_gather  (A)     panel entries = K - sum of descendant updates
//   fac_diag    (B)     LDL^T of the diagonal blocks of wide supernodes
//   fac_rows    (C)     pivots of width-1 supernodes and off-diagonal rows
//   border_schur        S_k = L_bk D_k L_bk^T per block
//   border_sum/factor   S = K_bb - sum_k S_k (fixed order), dense LDL^T
//   sol_*               forward, border, backward substitutions
// No floating-point atomics: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace ncl {

constexpr int kWG = 256;                 // threads per workgroup of the list kernels (4 wavefronts)
constexpr int kBorderThreads = 1024;

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(int((blockIdx.x * kWG + threadIdx.x) >> 6)); }
__device__ inline int lane_id() { return int(threadIdx.x & 63); }

// sum_k a[k*st] d[k*sd] c[k*st] with four independent partial sums
// (a, c: two rows of a panel, stride st; d: the panel's pivots, stride sd)
__device__ inline double wdot(const double *__restrict__ a, const double *__restrict__ c,
                              const double *__restrict__ d, int w, int64_t st, int64_t sd) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = 0;
    for (; k + 4 <= w; k += 4) {
        s0 += a[k * st] * d[k * sd] * c[k * st];
        s1 += a[(k + 1) * st] * d[(k + 1) * sd] * c[(k + 1) * st];
        s2 += a[(k + 2) * st] * d[(k + 2) * sd] * c[(k + 2) * st];
        s3 += a[(k + 3) * st] * d[(k + 3) * sd] * c[(k + 3) * st];
    }
    for (; k < w; k++) s0 += a[k * st] * d[k * sd] * c[k * st];
    return (s0 + s1) + (s2 + s3);
}

// sum_k a[k*sa] y[k*sy]
__device__ inline double rdot(const double *__restrict__ a, int64_t sa, const double *__restrict__ y, int64_t sy,
                              int w) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = 0;
    for (; k + 4 <= w; k += 4) {
        s0 += a[k * sa] * y[k * sy];
        s1 += a[(k + 1) * sa] * y[(k + 1) * sy];
        s2 += a[(k + 2) * sa] * y[(k + 2) * sy];
        s3 += a[(k + 3) * sa] * y[(k + 3) * sy];
    }
    for (; k < w; k++) s0 += a[k * sa] * y[k * sy];
    return (s0 + s1) + (s2 + s3);
}

// template owning a flat interleaved index (binary search over the bases)
__device__ inline int find_tmpl(const DevArgs &a, int64_t idx, int64_t TemplDev::*base) {
    int lo = 0, hi = a.ntmpl - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.tmpls[mid].*base <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ assembly

struct EndDeriv {
    double P, Q;
    double gP[4], gQ[4];   // (v_s, v_o, th_s, th_o)
};

// Flow leaving end s of a branch with series admittance g + jb:
//   P = g vs^2 - vs vo (g cos th + b sin th),  Q = -b vs^2 - vs vo (g sin th - b cos th)
// with th = th_s - th_o.  Adds wP * Hess P + wQ * Hess Q + wF * Hess(P^2 + Q^2)
// into W (4x4 over v_s, v_o, th_s, th_o, mapped through idx into the branch order).
__device__ inline void branch_end(double g, double b, double vs, double vo, double ts, double to, double wP,
                                  double wQ, double wF, const int idx[4], double W[4][4], EndDeriv &e) {
    double sn, cs;
    sincos(ts - to, &sn, &cs);
    const double A = g * cs + b * sn;
    const double Bq = g * sn - b * cs;
    const double vv = vs * vo;
    e.P = g * vs * vs - vv * A;
    e.Q = -b * vs * vs - vv * Bq;
    e.gP[0] = 2.0 * g * vs - vo * A;
    e.gP[1] = -vs * A;
    e.gP[2] = vv * Bq;
    e.gP[3] = -vv * Bq;
    e.gQ[0] = -2.0 * b * vs - vo * Bq;
    e.gQ[1] = -vs * Bq;
    e.gQ[2] = -vv * A;
    e.gQ[3] = vv * A;
    // Hess(P^2+Q^2) = 2 (gP gP^T + P HP + gQ gQ^T + Q HQ)
    const double al = wP + 2.0 * wF * e.P;
    const double be = wQ + 2.0 * wF * e.Q;
    double HP[4][4], HQ[4][4];
    HP[0][0] = 2.0 * g;   HP[0][1] = -A;        HP[0][2] = vo * Bq;  HP[0][3] = -vo * Bq;
    HP[1][1] = 0.0;       HP[1][2] = vs * Bq;   HP[1][3] = -vs * Bq;
    HP[2][2] = vv * A;    HP[2][3] = -vv * A;   HP[3][3] = vv * A;
    HQ[0][0] = -2.0 * b;  HQ[0][1] = -Bq;       HQ[0][2] = -vo * A;  HQ[0][3] = vo * A;
    HQ[1][1] = 0.0;       HQ[1][2] = -vs * A;   HQ[1][3] = vs * A;
    HQ[2][2] = vv * Bq;   HQ[2][3] = -vv * Bq;  HQ[3][3] = vv * Bq;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = a; c < 4; c++) {
            double h = al * HP[a][c] + be * HQ[a][c] + 2.0 * wF * (e.gP[a] * e.gP[c] + e.gQ[a] * e.gQ[c]);
            int ia = idx[a], ic = idx[c];
            W[ia][ic] += h;
            if (ia != ic) W[ic][ia] += h;
        }
}

struct AsmCtx {
    const DevArgs *a;
    int64_t kb;      // template K base + the lane's block
    int64_t nb;      // blocks of the template (stride)
};

__device__ inline void put(const AsmCtx &c, int32_t slot, double v) {
    if (slot < 0) return;
    if (slot & kBorderFlag) c.a->kval[c.a->kint + (slot & ~kBorderFlag)] = v;
    else c.a->kval[c.kb + int64_t(slot) * c.nb] = v;
}

__device__ inline int64_t zi(const DevArgs &a, const BlockDev &B, int n, int32_t x) {
    return x < n ? B.col0 + x : a.bstart + (x - n);
}

// Threads: (bus, block) pairs, then (generator, block) pairs, then border pg;
// the block index runs fastest so that neighbouring threads write
// neighbouring interleaved values.
__global__ __launch_bounds__(256) void k_assemble(DevArgs a, const double *__restrict__ z,
                                                  const double *__restrict__ sig, double rho) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nbus_t = int64_t(a.nblk) * a.nb;
    const int64_t ngen_t = int64_t(a.nblk) * a.ng;
    const double irho = 1.0 / rho;
    if (tid < nbus_t) {
        const int blk = int(tid % a.nblk), i = int(tid / a.nblk);
        const BlockDev B = a.blks[blk];
        const TemplDev &T = a.tmpls[B.tmpl];
        const int n = T.n;
        const AsmCtx cx{&a, T.kbase + B.bl, T.nblk};
        const int32_t *bi = T.bus_idx + size_t(i) * BI_N;
        double Hvv = 0, Haa = 0, Hva = 0, dPv = 0, dPa = 0, dQv = 0, dQa = 0, absv = 0, absa = 0;
        for (int q = T.bus_adj_ptr[i]; q < T.bus_adj_ptr[i + 1]; q++) {
            const int32_t e = T.bus_adj[q];
            const bool self_from = e >= 0;
            const int l = self_from ? e : ~e;
            const int32_t *br = T.br_idx + size_t(l) * 4;
            const int f = br[2], t = br[3];
            const int32_t *bf = T.bus_idx + size_t(f) * BI_N, *bt = T.bus_idx + size_t(t) * BI_N;
            const double vf = z[zi(a, B, n, bf[BI_VM])], vt = z[zi(a, B, n, bt[BI_VM])];
            const double tf = z[zi(a, B, n, bf[BI_VA])], tt = z[zi(a, B, n, bt[BI_VA])];
            const double yPf = z[zi(a, B, n, bf[BI_P])], yQf = z[zi(a, B, n, bf[BI_Q])];
            const double yPt = z[zi(a, B, n, bt[BI_P])], yQt = z[zi(a, B, n, bt[BI_Q])];
            const double yFf = z[zi(a, B, n, br[0])], yFt = z[zi(a, B, n, br[1])];
            const double st = (l == B.outage) ? 0.0 : 1.0;
            const double r = a.br_r[l], x = a.br_x[l];
            const double den = r * r + x * x;
            const double g = st * (r / den), b = st * (-x / den);
            double W[4][4] = {};
            EndDeriv ef, et;
            const int idf[4] = {0, 1, 2, 3}, idt[4] = {1, 0, 3, 2};
            branch_end(g, b, vf, vt, tf, tt, yPf, yQf, yFf, idf, W, ef);
            branch_end(g, b, vt, vf, tt, tf, yPt, yQt, yFt, idt, W, et);
            const int sv = self_from ? 0 : 1, sa = self_from ? 2 : 3, ov = self_from ? 1 : 0, oa = self_from ? 3 : 2;
            Hvv += W[sv][sv];
            Haa += W[sa][sa];
            Hva += W[sv][sa];
            absv += fabs(W[sv][ov]) + fabs(W[sv][oa]);
            absa += fabs(W[sa][ov]) + fabs(W[sa][oa]);
            const EndDeriv &es = self_from ? ef : et;
            dPv += es.gP[0];
            dPa += es.gP[2];
            dQv += es.gQ[0];
            dQa += es.gQ[2];
            if (self_from) {
                const int32_t *s = T.br_slot + size_t(l) * LS_N;
                put(cx, s[LS_VMVM], W[0][1]);
                put(cx, s[LS_VMVA], W[0][3]);
                put(cx, s[LS_VAVM], W[2][1]);
                put(cx, s[LS_VAVA], W[2][3]);
                put(cx, s[LS_PF_VMT], ef.gP[1]);
                put(cx, s[LS_PF_VAT], ef.gP[3]);
                put(cx, s[LS_QF_VMT], ef.gQ[1]);
                put(cx, s[LS_QF_VAT], ef.gQ[3]);
                put(cx, s[LS_PT_VMF], et.gP[1]);
                put(cx, s[LS_PT_VAF], et.gP[3]);
                put(cx, s[LS_QT_VMF], et.gQ[1]);
                put(cx, s[LS_QT_VAF], et.gQ[3]);
                // flow rows: grad (P^2 + Q^2) = 2 P gP + 2 Q gQ
                double hf[4], ht[4];
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    hf[c] = 2.0 * ef.P * ef.gP[c] + 2.0 * ef.Q * ef.gQ[c];
                    ht[c] = 2.0 * et.P * et.gP[c] + 2.0 * et.Q * et.gQ[c];
                }
                put(cx, s[LS_FF_VMF], hf[0]);
                put(cx, s[LS_FF_VMT], hf[1]);
                put(cx, s[LS_FF_VAF], hf[2]);
                put(cx, s[LS_FF_VAT], hf[3]);
                put(cx, s[LS_FT_VMF], ht[1]);
                put(cx, s[LS_FT_VMT], ht[0]);
                put(cx, s[LS_FT_VAF], ht[3]);
                put(cx, s[LS_FT_VAT], ht[2]);
                put(cx, s[LS_FFFF], -irho);
                put(cx, s[LS_FTFT], -irho);
            }
        }
        const double dv = fmax(0.0, absv + fabs(Hva) - Hvv);
        const double da = fmax(0.0, absa + fabs(Hva) - Haa);
        const int32_t *bs = T.bus_slot + size_t(i) * BS_N;
        put(cx, bs[BS_VMVM], Hvv + dv + sig[zi(a, B, n, bi[BI_VM])]);
        put(cx, bs[BS_VAVA], Haa + da + sig[zi(a, B, n, bi[BI_VA])]);
        put(cx, bs[BS_VMVA], Hva);
        put(cx, bs[BS_PVM], dPv);
        put(cx, bs[BS_PVA], dPa);
        put(cx, bs[BS_QVM], dQv);
        put(cx, bs[BS_QVA], dQa);
        put(cx, bs[BS_PP], -irho);
        put(cx, bs[BS_QQ], -irho);
        return;
    }
    if (tid < nbus_t + ngen_t) {
        const int64_t u = tid - nbus_t;
        const int blk = int(u % a.nblk), g = int(u / a.nblk);
        const BlockDev B = a.blks[blk];
        const TemplDev &T = a.tmpls[B.tmpl];
        const int n = T.n;
        const AsmCtx cx{&a, T.kbase + B.bl, T.nblk};
        const int32_t *gi = T.gen_idx + size_t(g) * GI_N;
        const int32_t *gs = T.gen_slot + size_t(g) * GS_N;
        put(cx, gs[GS_PPG], -1.0);
        put(cx, gs[GS_QQG], -1.0);
        put(cx, gs[GS_QGQG], sig[zi(a, B, n, gi[GI_QG])]);
        if (T.has_pg_local) {
            const double h = 2.0 * a.gen_c2[g];
            put(cx, gs[GS_PGPG], h + fmax(0.0, -h) + sig[zi(a, B, n, gi[GI_PG])]);
        }
        if (T.pvpq_rows) {
            const double nup = z[zi(a, B, n, gi[GI_NUP])], num = z[zi(a, B, n, gi[GI_NUM])];
            const double sup = z[zi(a, B, n, gi[GI_SUP])], slo = z[zi(a, B, n, gi[GI_SLO])];
            const int64_t cu = zi(a, B, n, gi[GI_CUP]), cl = zi(a, B, n, gi[GI_CLO]);
            const double n0u = z[cu], n0l = z[cl];
            put(cx, gs[GS_LIN_NUP], 1.0);
            put(cx, gs[GS_LIN_NUM], -1.0);
            put(cx, gs[GS_LIN_VM], -1.0);
            put(cx, gs[GS_LIN_VM0], 1.0);
            put(cx, gs[GS_DUP_SUP], 1.0);
            put(cx, gs[GS_DUP_QG], 1.0);
            put(cx, gs[GS_DLO_SLO], 1.0);
            put(cx, gs[GS_DLO_QG], -1.0);
            put(cx, gs[GS_CUP_NUM], sup);
            put(cx, gs[GS_CUP_SUP], num);
            put(cx, gs[GS_CLO_NUP], slo);
            put(cx, gs[GS_CLO_SLO], nup);
            put(cx, gs[GS_H_NUM_SUP], n0u);
            put(cx, gs[GS_H_NUP_SLO], n0l);
            put(cx, gs[GS_NUPNUP], fabs(n0l) + sig[zi(a, B, n, gi[GI_NUP])]);
            put(cx, gs[GS_NUMNUM], fabs(n0u) + sig[zi(a, B, n, gi[GI_NUM])]);
            put(cx, gs[GS_SUPSUP], fabs(n0u) + sig[zi(a, B, n, gi[GI_SUP])]);
            put(cx, gs[GS_SLOSLO], fabs(n0l) + sig[zi(a, B, n, gi[GI_SLO])]);
            put(cx, gs[GS_LL], -irho);
            put(cx, gs[GS_UU], -irho);
            put(cx, gs[GS_DD], -irho);
            put(cx, gs[GS_CUCU], -(irho + sig[cu] / n0u));
            put(cx, gs[GS_CLCL], -(irho + sig[cl] / n0l));
        }
        return;
    }
    const int64_t g = tid - nbus_t - ngen_t;
    if (g < a.ng && a.nbd > 0) {
        const int bidx = a.border_pg[g];
        const int32_t p = a.kbb_pos[size_t(bidx) * a.nbd + bidx];
        const double h = 2.0 * a.gen_c2[g];
        if (p >= 0) a.kval[a.kint + p] = h + fmax(0.0, -h) + sig[a.bstart + bidx];
    }
}

// Public lower-CSC values <-> internal (interleaved blocks, then K_bb).
__global__ __launch_bounds__(256) void k_values(DevArgs a, const double *__restrict__ src, double *__restrict__ dst,
                                                int to_internal, int64_t nnz_border, int64_t kcsc_border) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < a.kint) {
        const int ti = find_tmpl(a, idx, &TemplDev::kbase);
        const TemplDev &T = a.tmpls[ti];
        const int64_t off = idx - T.kbase;
        const int64_t e = off / T.nblk;
        const int bl = int(off % T.nblk);
        const int64_t c = a.blks[T.blocks[bl]].kcsc + e;
        if (to_internal) dst[idx] = src[c];
        else dst[c] = src[idx];
    } else if (idx < a.kint + nnz_border) {
        const int64_t p = idx - a.kint;
        if (to_internal) dst[idx] = src[kcsc_border + p];
        else dst[kcsc_border + p] = src[idx];
    }
}

// ------------------------------------------------------------------ factor

struct Lane {
    const TemplDev *T;
    int k, bl, nb;
    bool on;
};

__device__ inline Lane lane_work(const DevArgs &a, const Work *wl, int wid) {
    const Work wk = wl[wid];
    Lane L;
    L.T = a.tmpls + (wk.tg >> 16);
    L.k = wk.k;
    L.nb = L.T->nblk;
    const int b = (wk.tg & 0xffff) * 64 + lane_id();
    L.on = b < L.nb;
    L.bl = L.on ? b : 0;
    return L;
}

// A: one lower panel entry = its K value minus the updates of all descendant
// supernodes that hold the entry's row and column, in increasing order of
// the descendant; two descendants are in flight at a time.
__global__ __launch_bounds__(kWG) void k_fac_gather(DevArgs a, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const double *__restrict__ Lp = a.lpan + T.lbase + W.bl;
    const double *__restrict__ Dv = a.dval + T.dbase + W.bl;
    const int e = W.k;
    const int kp = T.ent_kpos[e];
    const int i1 = T.ent_iptr[e + 1];
    int it = T.ent_iptr[e];
    double v = kp >= 0 ? a.kval[T.kbase + W.bl + int64_t(kp) * nb] : 0.0;
    for (; it + 2 <= i1; it += 2) {
        const CItem c0 = T.citems[it], c1 = T.citems[it + 1];
        const double u0 = wdot(Lp + int64_t(c0.ioff) * nb, Lp + int64_t(c0.coff) * nb, Dv + int64_t(c0.dcol) * nb,
                               c0.meta >> 16, int64_t(c0.meta & 0xffff) * nb, nb);
        const double u1 = wdot(Lp + int64_t(c1.ioff) * nb, Lp + int64_t(c1.coff) * nb, Dv + int64_t(c1.dcol) * nb,
                               c1.meta >> 16, int64_t(c1.meta & 0xffff) * nb, nb);
        v -= u0;
        v -= u1;
    }
    if (it < i1) {
        const CItem c0 = T.citems[it];
        v -= wdot(Lp + int64_t(c0.ioff) * nb, Lp + int64_t(c0.coff) * nb, Dv + int64_t(c0.dcol) * nb, c0.meta >> 16,
                  int64_t(c0.meta & 0xffff) * nb, nb);
    }
    if (W.on) a.lpan[T.lbase + W.bl + int64_t(T.ent_out[e]) * nb] = v;
}

// B: LDL^T of the diagonal block of a wide supernode.  Two blocks per
// wavefront; lane i of each half holds row i of its block's diagonal block
// in registers, and the right-looking elimination exchanges columns by
// cross-lane shuffles.  Row i ends with l_ik (k < i) and d_i.
__global__ __launch_bounds__(kWG) void k_fac_diag(DevArgs a, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const int lane = lane_id();
    const int half = lane >> 5, i = lane & 31;
    const Work wk = wl[wid];
    const TemplDev &T = a.tmpls[wk.tg >> 16];
    const int nb = T.nblk;
    const int b = (wk.tg & 0xffff) * 2 + half;
    const int bl = b < nb ? b : 0;
    const int s = wk.k;
    const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
    const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
    const bool on = b < nb && i < w;
    double *P = a.lpan + T.lbase + bl + int64_t(T.panel_off[s]) * nb;   // P(row, col) = P[(col * r + row) * nb]
    double row[kMaxW];
#pragma unroll
    for (int k = 0; k < kMaxW; k++) row[k] = (k < w && k <= i && i < w) ? P[(int64_t(k) * r + i) * nb] : 0.0;
    const int base = half << 5;
#pragma unroll
    for (int j = 0; j < kMaxW; j++) {
        if (j < w) {
            const double dj = __shfl(row[j], base + j);
            const double lij = i > j ? row[j] / dj : 0.0;
#pragma unroll
            for (int k = j + 1; k < kMaxW; k++) {
                if (k < w) {
                    const double lkj = __shfl(lij, base + k);
                    if (i >= k) row[k] -= lij * dj * lkj;
                }
            }
            if (i > j) row[j] = lij;
        }
    }
    if (on) {
        double di = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxW; k++) {
            if (k < i) P[(int64_t(k) * r + i) * nb] = row[k];
            if (k == i) di = row[k];
        }
        a.dval[T.dbase + bl + int64_t(f + i) * nb] = di;
    }
}

// C: pivot and off-diagonal rows.  Width-1 supernodes: d = P(0,0) and
// L(p,0) = P(p,0) / d.  Wide supernodes: row p >= w solves
// x_j = (P(p,j) - sum_{k<j} x_k d_k L(j,k)) / d_j.
__global__ __launch_bounds__(kWG) void k_fac_rows(DevArgs a, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const int s = T.task_s[W.k], p = T.task_p[W.k];
    const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
    const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
    double *P = a.lpan + T.lbase + W.bl + int64_t(T.panel_off[s]) * nb;
    double *Dv = a.dval + T.dbase + W.bl + int64_t(f) * nb;
    if (w == 1) {
        if (!W.on) return;
        if (p == 0) Dv[0] = P[0];
        else P[int64_t(p) * nb] = P[int64_t(p) * nb] / P[0];
        return;
    }
    double x[kMaxW];
#pragma unroll
    for (int j = 0; j < kMaxW; j++) {
        if (j < w) {
            double v = P[(int64_t(j) * r + p) * nb];
#pragma unroll
            for (int k = 0; k < kMaxW; k++)
                if (k < j) v -= x[k] * Dv[int64_t(k) * nb] * P[(int64_t(k) * r + j) * nb];
            x[j] = v / Dv[int64_t(j) * nb];
        }
    }
    if (W.on) {
#pragma unroll
        for (int j = 0; j < kMaxW; j++)
            if (j < w) P[(int64_t(j) * r + p) * nb] = x[j];
    }
}

// Border Schur contribution S_k[e] = sum over common panels of L[i,:] D L[j,:]^T
// for packed border entry e = (i, j); written entry-major, block fastest.
__global__ __launch_bounds__(kWG) void k_border_schur(DevArgs a, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const double *__restrict__ Lp = a.lpan + T.lbase + W.bl;
    const double *__restrict__ Dv = a.dval + T.dbase + W.bl;
    const int e = W.k;
    double sum = 0.0;
    for (int it = T.sitem_ptr[e]; it < T.sitem_ptr[e + 1]; it++) {
        const SItem si = T.sitems[it];
        const int f = T.sup_first[si.s], w = T.sup_first[si.s + 1] - f;
        const int r = T.sup_rowptr[si.s + 1] - T.sup_rowptr[si.s];
        const int64_t po = T.panel_off[si.s];
        sum += wdot(Lp + (po + si.pi) * nb, Lp + (po + si.pj) * nb, Dv + int64_t(f) * nb, w, int64_t(r) * nb, nb);
    }
    if (W.on) a.spart[int64_t(e) * a.nblk + T.blocks[W.bl]] = sum;
}

// ------------------------------------------------------------------ border

__device__ inline void unpack(int64_t e, int &i, int &j) {
    int ii = int((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
    while (int64_t(ii) * (ii + 1) / 2 > e) ii--;
    while (int64_t(ii + 1) * (ii + 2) / 2 <= e) ii++;
    i = ii;
    j = int(e - int64_t(ii) * (ii + 1) / 2);
}

__device__ inline int pk(int i, int j) { return i * (i + 1) / 2 + j; }

// S[e] = K_bb[e] - sum_k S_k[e]: one wavefront per entry, blocks summed in a
// fixed order (lane-strided partial sums, then a fixed shuffle tree).
__global__ __launch_bounds__(kWG) void k_border_sum(DevArgs a) {
    const int64_t npk = int64_t(a.nbd) * (a.nbd + 1) / 2;
    const int64_t e = wave_id();
    if (e >= npk) return;
    const int lane = lane_id();
    double s = 0.0;
    for (int b = lane; b < a.nblk; b += 64) s += a.spart[e * a.nblk + b];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) {
        int i, j;
        unpack(e, i, j);
        const int32_t p = a.kbb_pos[size_t(i) * a.nbd + j];
        a.sbb[e] = (p >= 0 ? a.kval[a.kint + p] : 0.0) - s;
    }
}

// Dense LDL^T of the packed border matrix.  The matrix is held in 4x4
// register tiles spread over the workgroup (lower-triangular tiles, tile q
// in thread q mod 1024); each pivot step broadcasts the current column
// through a double-buffered LDS vector and every thread updates the tiles
// right of the pivot.  Used when the tiles fit (border <= kTileMaxB);
// otherwise the column-by-column version below runs in place.
constexpr int kTileMaxB = 252;                 // 2 tiles per thread cover 63 tile rows

template <int kTPT>
__global__ __launch_bounds__(kBorderThreads) void k_border_factor_tiles(DevArgs a) {
    __shared__ double col[2][kTileMaxB + 4];
    const int nbd = a.nbd;
    const int nt = (nbd + 3) / 4;                  // tile rows
    const int ntiles = nt * (nt + 1) / 2;
    const int tid = threadIdx.x;
    double S[kTPT][4][4];
    int TI[kTPT], TK[kTPT];
#pragma unroll
    for (int q = 0; q < kTPT; q++) {
        const int t = tid + q * kBorderThreads;
        int I = 0, K = 0;
        if (t < ntiles) {
            int ii, jj;
            unpack(t, ii, jj);
            I = ii;
            K = jj;
        }
        TI[q] = t < ntiles ? I : -1;
        TK[q] = K;
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = 4 * I + u, k = 4 * K + v;
                S[q][u][v] = (t < ntiles && i < nbd && k <= i) ? a.sbb[pk(i, k)] : 0.0;
            }
    }
    for (int j = 0; j < nbd; j++) {
        double *cj = col[j & 1];
        const int J = j >> 2, jv = j & 3;
        // owners of tile column J publish column j (rows >= j)
#pragma unroll
        for (int q = 0; q < kTPT; q++)
            if (TI[q] >= 0 && TK[q] == J)
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int i = 4 * TI[q] + u;
                    if (i >= j && i < nbd) {
                        double v = 0.0;
#pragma unroll
                        for (int w = 0; w < 4; w++)
                            if (w == jv) v = S[q][u][w];
                        cj[i] = v;
                    }
                }
        __syncthreads();
        const double inv = 1.0 / cj[j];
#pragma unroll
        for (int q = 0; q < kTPT; q++) {
            if (TI[q] < 0 || 4 * TI[q] + 3 <= j || 4 * TK[q] + 3 <= j) continue;
            double ci[4], ck[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int i = 4 * TI[q] + u, k = 4 * TK[q] + u;
                ci[u] = (i > j && i < nbd) ? cj[i] * inv : 0.0;
                ck[u] = (k > j && k < nbd) ? cj[k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) S[q][u][v] -= ci[u] * ck[v];
        }
        // next step writes the other buffer; a barrier every step keeps a
        // buffer from being overwritten while a slow thread still reads it
    }
    __syncthreads();
    // pivots: diagonal of the diagonal tiles
    double *Db = a.dval + a.dint;
#pragma unroll
    for (int q = 0; q < kTPT; q++)
        if (TI[q] >= 0 && TI[q] == TK[q])
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int i = 4 * TI[q] + u;
                if (i < nbd) Db[i] = S[q][u][u];
            }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTPT; q++) {
        if (TI[q] < 0) continue;
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = 4 * TI[q] + u, k = 4 * TK[q] + v;
                if (i < nbd && k <= i) a.sbb[pk(i, k)] = (i == k) ? 1.0 : S[q][u][v] / Db[k];
            }
    }
}

// Column-by-column dense LDL^T of the packed border matrix in LDS, or in
// place in global memory when it does not fit.
__global__ __launch_bounds__(kBorderThreads) void k_border_factor(DevArgs a, int use_lds) {
    extern __shared__ double lds[];
    const int nbd = a.nbd;
    const int npk = nbd * (nbd + 1) / 2;
    const int tid = threadIdx.x;
    double *S = use_lds ? lds : a.sbb;
    if (use_lds)
        for (int e = tid; e < npk; e += kBorderThreads) S[e] = a.sbb[e];
    __syncthreads();
    const int tx = tid & 31, ty = tid >> 5;
    for (int j = 0; j < nbd; j++) {
        const double inv = 1.0 / S[pk(j, j)];
        for (int i = j + 1 + ty; i < nbd; i += 32) {
            const double ci = S[pk(i, j)] * inv;
            for (int k = j + 1 + tx; k <= i; k += 32) S[pk(i, k)] -= ci * S[pk(k, j)];
        }
        __syncthreads();
    }
    double *Db = a.dval + a.dint;
    for (int j = tid; j < nbd; j += kBorderThreads) Db[j] = S[pk(j, j)];
    __syncthreads();
    for (int e = tid; e < npk; e += kBorderThreads) {
        int i, j;
        unpack(e, i, j);
        a.sbb[e] = (i == j) ? 1.0 : S[e] / Db[j];
    }
}

// Pivot signs and magnitudes of the whole factorisation (integer atomics only).
__global__ __launch_bounds__(64) void k_status_init(DevArgs a) {
    if (threadIdx.x == 0) {
        a.stat[0] = 0;
        a.stat[1] = 0;
        a.stat[2] = 0;
        a.stat[3] = INT64_MAX;
        a.stat[4] = INT64_MAX;
        a.stat[5] = 0;
    }
}

__device__ inline int pivot_code(double d, bool primal) {
    if (!isfinite(d)) return 3;                 // non-finite
    if (d == 0.0) return 2;                     // zero
    if ((d > 0.0) != primal) return 1;          // wrong sign
    return 0;
}

__global__ __launch_bounds__(256) void k_status(DevArgs a) {
    int64_t np = 0, nn = 0, nz = 0, bad = INT64_MAX, mn = INT64_MAX, mx = 0;
    const int64_t total = a.dint + a.nbd;
    for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * blockDim.x) {
        double d;
        bool primal;
        int64_t col;
        if (idx < a.dint) {
            const int ti = find_tmpl(a, idx, &TemplDev::dbase);
            const TemplDev &T = a.tmpls[ti];
            const int64_t off = idx - T.dbase;
            const int j = int(off / T.nblk), bl = int(off % T.nblk);
            d = a.dval[idx];
            primal = T.col_primal[j] != 0;
            col = a.blks[T.blocks[bl]].col0 + j;
        } else {
            const int j = int(idx - a.dint);
            d = a.dval[idx];
            primal = a.bprim[j] != 0;
            col = a.bstart + j;
        }
        const int code = pivot_code(d, primal);
        if (code == 0 || code == 1) {
            if (d > 0) np++;
            else nn++;
        } else if (code == 2) nz++;
        if (code && col * 8 + code < bad) bad = col * 8 + code;
        const double ad = fabs(d);
        if (isfinite(ad)) {
            const int64_t bits = __double_as_longlong(ad);
            mn = bits < mn ? bits : mn;
            mx = bits > mx ? bits : mx;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        np += __shfl_xor(np, o);
        nn += __shfl_xor(nn, o);
        nz += __shfl_xor(nz, o);
        const int64_t ob = __shfl_xor(bad, o), om = __shfl_xor(mn, o), ox = __shfl_xor(mx, o);
        bad = ob < bad ? ob : bad;
        mn = om < mn ? om : mn;
        mx = ox > mx ? ox : mx;
    }
    __shared__ int64_t red[6][4];
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) {
        red[0][wv] = np; red[1][wv] = nn; red[2][wv] = nz; red[3][wv] = bad; red[4][wv] = mn; red[5][wv] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; q++) {
            red[0][0] += red[0][q];
            red[1][0] += red[1][q];
            red[2][0] += red[2][q];
            red[3][0] = red[3][q] < red[3][0] ? red[3][q] : red[3][0];
            red[4][0] = red[4][q] < red[4][0] ? red[4][q] : red[4][0];
            red[5][0] = red[5][q] > red[5][0] ? red[5][q] : red[5][0];
        }
        unsigned long long *u = reinterpret_cast<unsigned long long *>(a.stat);
        if (red[0][0]) atomicAdd(u + 0, (unsigned long long)red[0][0]);
        if (red[1][0]) atomicAdd(u + 1, (unsigned long long)red[1][0]);
        if (red[2][0]) atomicAdd(u + 2, (unsigned long long)red[2][0]);
        if (red[3][0] != INT64_MAX) atomicMin(reinterpret_cast<long long *>(a.stat + 3), (long long)red[3][0]);
        if (red[4][0] != INT64_MAX) atomicMin(reinterpret_cast<long long *>(a.stat + 4), (long long)red[4][0]);
        if (red[5][0]) atomicMax(reinterpret_cast<long long *>(a.stat + 5), (long long)red[5][0]);
    }
}

// ------------------------------------------------------------------ solve

// y (interleaved, factor order) = b (layout order, one column)
__global__ __launch_bounds__(256) void k_sol_load(DevArgs a, const double *__restrict__ b, double *__restrict__ y) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= a.dint) return;
    const int ti = find_tmpl(a, idx, &TemplDev::dbase);
    const TemplDev &T = a.tmpls[ti];
    const int64_t off = idx - T.dbase;
    const int j = int(off / T.nblk), bl = int(off % T.nblk);
    y[idx] = b[a.blks[T.blocks[bl]].col0 + T.perm[j]];
}

__global__ __launch_bounds__(256) void k_sol_store(DevArgs a, const double *__restrict__ y, double *__restrict__ x) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= a.dint) return;
    const int ti = find_tmpl(a, idx, &TemplDev::dbase);
    const TemplDev &T = a.tmpls[ti];
    const int64_t off = idx - T.dbase;
    const int j = int(off / T.nblk), bl = int(off % T.nblk);
    x[a.blks[T.blocks[bl]].col0 + T.perm[j]] = y[idx];
}

__global__ __launch_bounds__(256) void k_sol_scale(DevArgs a, double *__restrict__ y) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < a.dint) y[idx] = y[idx] / a.dval[idx];
}

// forward gather of a diagonal row: y_row -= sum over descendants L_d[row,:] y_d
__global__ __launch_bounds__(kWG) void k_sol_fwd_gather(DevArgs a, double *y, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const double *__restrict__ Lp = a.lpan + T.lbase + W.bl;
    double *yb = y + T.dbase + W.bl;
    const int s = T.task_s[W.k], p = T.task_p[W.k];
    const int col = T.sup_first[s] + p;
    const int e = T.task_cbase[W.k] + p;
    double v = 0.0;
    for (int it = T.ent_iptr[e]; it < T.ent_iptr[e + 1]; it++) {
        const CItem ci = T.citems[it];
        const int ld = ci.meta & 0xffff, wd = ci.meta >> 16;
        v += rdot(Lp + int64_t(ci.ioff) * nb, int64_t(ld) * nb, yb + int64_t(ci.dcol) * nb, nb, wd);
    }
    if (W.on) yb[int64_t(col) * nb] -= v;
}

// unit lower triangular solve with a wide supernode's diagonal block
__global__ __launch_bounds__(kWG) void k_sol_fwd_diag(DevArgs a, double *y, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const int s = W.k;
    const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
    const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
    const double *P = a.lpan + T.lbase + W.bl + int64_t(T.panel_off[s]) * nb;
    double *yb = y + T.dbase + W.bl + int64_t(f) * nb;
    double x[kMaxW];
#pragma unroll
    for (int j = 0; j < kMaxW; j++) {
        if (j < w) {
            double v = yb[int64_t(j) * nb];
#pragma unroll
            for (int k = 0; k < kMaxW; k++)
                if (k < j) v -= P[(int64_t(k) * r + j) * nb] * x[k];
            x[j] = v;
        }
    }
    if (W.on) {
#pragma unroll
        for (int j = 1; j < kMaxW; j++)
            if (j < w) yb[int64_t(j) * nb] = x[j];
    }
}

// this block's part of the border right-hand side: cpart[b][block] = L_bk y_k
__global__ __launch_bounds__(kWG) void k_sol_bpart(DevArgs a, const double *y, double *cpart,
                                                   const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const double *__restrict__ Lp = a.lpan + T.lbase + W.bl;
    const double *yb = y + T.dbase + W.bl;
    const int bi = W.k;
    double v = 0.0;
    for (int it = T.bpath_ptr[bi]; it < T.bpath_ptr[bi + 1]; it++) {
        const int s = T.bpath_s[it];
        const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
        const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
        v += rdot(Lp + int64_t(T.panel_off[s] + T.bpath_pos[it]) * nb, int64_t(r) * nb, yb + int64_t(f) * nb, nb, w);
    }
    if (W.on) cpart[int64_t(bi) * a.nblk + T.blocks[W.bl]] = v;
}

// border: c = b_b - sum_k cpart; forward with L_bb, D_b^{-1}, backward with
// L_bb^T.  Blocked by 32 rows: wavefront 0 solves a diagonal block with
// cross-lane shuffles (lane = row), then the workgroup updates the other rows.
__global__ __launch_bounds__(kBorderThreads) void k_sol_border(DevArgs a, const double *__restrict__ b, double *x,
                                                               double *y, const double *__restrict__ cpart) {
    extern __shared__ double c[];
    const int nbd = a.nbd, tid = threadIdx.x, lane = lane_id();
    const double *Db = a.dval + a.dint;
    const double *Lb = a.sbb;
    for (int i = tid; i < nbd; i += kBorderThreads) {
        double v = 0.0;
        for (int k = 0; k < a.nblk; k++) v += cpart[int64_t(i) * a.nblk + k];
        c[i] = b[a.bstart + i] - v;
    }
    __syncthreads();
    // forward: L y = c
    for (int b0 = 0; b0 < nbd; b0 += 32) {
        const int bs = nbd - b0 < 32 ? nbd - b0 : 32;
        if (tid < 64) {
            const int i = b0 + lane;
            double ci = lane < bs ? c[i] : 0.0;
            for (int k = 0; k < bs - 1; k++) {
                const double xk = __shfl(ci, k);
                if (lane > k && lane < bs) ci -= Lb[pk(i, b0 + k)] * xk;
            }
            if (lane < bs) c[i] = ci;
        }
        __syncthreads();
        for (int i = b0 + bs + tid; i < nbd; i += kBorderThreads) {
            const double *li = Lb + pk(i, b0);
            double s0 = 0.0, s1 = 0.0;
            int k = 0;
            for (; k + 2 <= bs; k += 2) {
                s0 += li[k] * c[b0 + k];
                s1 += li[k + 1] * c[b0 + k + 1];
            }
            if (k < bs) s0 += li[k] * c[b0 + k];
            c[i] -= s0 + s1;
        }
        __syncthreads();
    }
    for (int i = tid; i < nbd; i += kBorderThreads) c[i] /= Db[i];
    __syncthreads();
    // backward: L^T x = y, last block first
    for (int b0 = ((nbd - 1) / 32) * 32; b0 >= 0; b0 -= 32) {
        const int bs = nbd - b0 < 32 ? nbd - b0 : 32;
        if (tid < 64) {
            double cj = lane < bs ? c[b0 + lane] : 0.0;
            for (int i = bs - 1; i > 0; i--) {
                const double xi = __shfl(cj, i);
                if (lane < i) cj -= Lb[pk(b0 + i, b0 + lane)] * xi;
            }
            if (lane < bs) c[b0 + lane] = cj;
        }
        __syncthreads();
        for (int j = tid; j < b0; j += kBorderThreads) {
            double s0 = 0.0, s1 = 0.0;
            int k = 0;
            for (; k + 2 <= bs; k += 2) {
                s0 += Lb[pk(b0 + k, j)] * c[b0 + k];
                s1 += Lb[pk(b0 + k + 1, j)] * c[b0 + k + 1];
            }
            if (k < bs) s0 += Lb[pk(b0 + k, j)] * c[b0 + k];
            c[j] -= s0 + s1;
        }
        __syncthreads();
    }
    for (int i = tid; i < nbd; i += kBorderThreads) {
        y[a.dint + i] = c[i];
        x[a.bstart + i] = c[i];
    }
}

// backward gather of column p of a supernode: y_col -= sum_{i >= w} L(i, p) x_{row i}
__global__ __launch_bounds__(kWG) void k_sol_bwd_gather(DevArgs a, double *y, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const int n = T.n;
    const int s = T.task_s[W.k], p = T.task_p[W.k];
    const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
    const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
    const int32_t *R = T.sup_rows + T.sup_rowptr[s];
    const double *Pc = a.lpan + T.lbase + W.bl + (int64_t(T.panel_off[s]) + int64_t(p) * r) * nb;
    double *yb = y + T.dbase + W.bl;
    const double *xb = y + a.dint;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = w;
    for (; i + 4 <= r; i += 4) {
        const int r0 = R[i], r1 = R[i + 1], r2 = R[i + 2], r3 = R[i + 3];
        s0 += Pc[int64_t(i) * nb] * (r0 < n ? yb[int64_t(r0) * nb] : xb[r0 - n]);
        s1 += Pc[int64_t(i + 1) * nb] * (r1 < n ? yb[int64_t(r1) * nb] : xb[r1 - n]);
        s2 += Pc[int64_t(i + 2) * nb] * (r2 < n ? yb[int64_t(r2) * nb] : xb[r2 - n]);
        s3 += Pc[int64_t(i + 3) * nb] * (r3 < n ? yb[int64_t(r3) * nb] : xb[r3 - n]);
    }
    for (; i < r; i++) {
        const int ri = R[i];
        s0 += Pc[int64_t(i) * nb] * (ri < n ? yb[int64_t(ri) * nb] : xb[ri - n]);
    }
    if (W.on) yb[int64_t(f + p) * nb] -= (s0 + s1) + (s2 + s3);
}

// unit upper triangular solve with the transposed diagonal block
__global__ __launch_bounds__(kWG) void k_sol_bwd_diag(DevArgs a, double *y, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const int s = W.k;
    const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
    const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
    const double *P = a.lpan + T.lbase + W.bl + int64_t(T.panel_off[s]) * nb;
    double *yb = y + T.dbase + W.bl + int64_t(f) * nb;
    double x[kMaxW];
#pragma unroll
    for (int j = kMaxW - 1; j >= 0; j--) {
        if (j < w) {
            double v = yb[int64_t(j) * nb];
#pragma unroll
            for (int k = 0; k < kMaxW; k++)
                if (k > j && k < w) v -= P[(int64_t(j) * r + k) * nb] * x[k];
            x[j] = v;
        }
    }
    if (W.on) {
#pragma unroll
        for (int j = 0; j < kMaxW - 1; j++)
            if (j < w - 1) yb[int64_t(j) * nb] = x[j];
    }
}

// ------------------------------------------------------------------ launchers

static inline unsigned waves_grid(int nw) { return unsigned((nw + (kWG / 64) - 1) / (kWG / 64)); }
static inline unsigned elems_grid(int64_t n) { return unsigned((n + 255) / 256); }

hipError_t launch_assemble(const DevArgs &a, const double *z, const double *sig, double rho, hipStream_t st) {
    const int64_t total = int64_t(a.nblk) * (a.nb + a.ng) + a.ng;
    hipLaunchKernelGGL(k_assemble, dim3(elems_grid(total)), dim3(256), 0, st, a, z, sig, rho);
    return hipGetLastError();
}

hipError_t launch_values(const DevArgs &a, const double *src, double *dst, bool to_internal, int64_t nnz_border,
                         int64_t kcsc_border, hipStream_t st) {
    const int64_t total = a.kint + nnz_border;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_values, dim3(elems_grid(total)), dim3(256), 0, st, a, src, dst, to_internal ? 1 : 0,
                       nnz_border, kcsc_border);
    return hipGetLastError();
}

hipError_t launch_factor_level(const DevArgs &a, const Work *wa, int na, const Work *wb, int nb, const Work *wc,
                               int nc, hipStream_t st) {
    if (na) hipLaunchKernelGGL(k_fac_gather, dim3(waves_grid(na)), dim3(kWG), 0, st, a, wa, na);
    if (nb) hipLaunchKernelGGL(k_fac_diag, dim3(waves_grid(nb)), dim3(kWG), 0, st, a, wb, nb);
    if (nc) hipLaunchKernelGGL(k_fac_rows, dim3(waves_grid(nc)), dim3(kWG), 0, st, a, wc, nc);
    return hipGetLastError();
}

hipError_t launch_schur(const DevArgs &a, const Work *ws, int nw, hipStream_t st) {
    if (nw) hipLaunchKernelGGL(k_border_schur, dim3(waves_grid(nw)), dim3(kWG), 0, st, a, ws, nw);
    return hipGetLastError();
}

hipError_t launch_factor_border(const DevArgs &a, hipStream_t st) {
    if (a.nbd > 0) {
        const int64_t npk = int64_t(a.nbd) * (a.nbd + 1) / 2;
        hipLaunchKernelGGL(k_border_sum, dim3(waves_grid(int(npk))), dim3(kWG), 0, st, a);
        const int nt = (a.nbd + 3) / 4;
        if (a.nbd <= kTileMaxB && nt * (nt + 1) / 2 <= 2 * kBorderThreads) {
            hipLaunchKernelGGL(k_border_factor_tiles<2>, dim3(1), dim3(kBorderThreads), 0, st, a);
        } else {
            const size_t lbytes = size_t(npk) * sizeof(double);
            const int use_lds = lbytes <= 150 * 1024 ? 1 : 0;
            hipLaunchKernelGGL(k_border_factor, dim3(1), dim3(kBorderThreads), use_lds ? lbytes : 0, st, a, use_lds);
        }
    }
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, st, a);
    const int64_t ne = a.dint + a.nbd;
    const unsigned sg = unsigned(ne / 256 / 16 + 1 < 1024 ? ne / 256 / 16 + 1 : 1024);
    hipLaunchKernelGGL(k_status, dim3(sg), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_solve_load(const DevArgs &a, const double *b, double *y, hipStream_t st) {
    if (a.dint) hipLaunchKernelGGL(k_sol_load, dim3(elems_grid(a.dint)), dim3(256), 0, st, a, b, y);
    return hipGetLastError();
}

hipError_t launch_solve_fwd_level(const DevArgs &a, double *y, const Work *wf, int nf, const Work *wd, int nd,
                                  hipStream_t st) {
    if (nf) hipLaunchKernelGGL(k_sol_fwd_gather, dim3(waves_grid(nf)), dim3(kWG), 0, st, a, y, wf, nf);
    if (nd) hipLaunchKernelGGL(k_sol_fwd_diag, dim3(waves_grid(nd)), dim3(kWG), 0, st, a, y, wd, nd);
    return hipGetLastError();
}

hipError_t launch_solve_bpart(const DevArgs &a, const double *y, double *cpart, const Work *wp, int np,
                              hipStream_t st) {
    if (np) hipLaunchKernelGGL(k_sol_bpart, dim3(waves_grid(np)), dim3(kWG), 0, st, a, y, cpart, wp, np);
    return hipGetLastError();
}

hipError_t launch_solve_border(const DevArgs &a, const double *b, double *x, double *y, const double *cpart,
                               hipStream_t st) {
    if (a.nbd > 0)
        hipLaunchKernelGGL(k_sol_border, dim3(1), dim3(kBorderThreads), size_t(a.nbd) * sizeof(double), st, a, b, x,
                           y, cpart);
    return hipGetLastError();
}

hipError_t launch_solve_scale(const DevArgs &a, double *y, hipStream_t st) {
    if (a.dint) hipLaunchKernelGGL(k_sol_scale, dim3(elems_grid(a.dint)), dim3(256), 0, st, a, y);
    return hipGetLastError();
}

hipError_t launch_solve_bwd_level(const DevArgs &a, double *y, const Work *wg, int ng, const Work *wd, int nd,
                                  hipStream_t st) {
    if (ng) hipLaunchKernelGGL(k_sol_bwd_gather, dim3(waves_grid(ng)), dim3(kWG), 0, st, a, y, wg, ng);
    if (nd) hipLaunchKernelGGL(k_sol_bwd_diag, dim3(waves_grid(nd)), dim3(kWG), 0, st, a, y, wd, nd);
    return hipGetLastError();
}

hipError_t launch_solve_store(const DevArgs &a, const double *y, double *x, hipStream_t st) {
    if (a.dint) hipLaunchKernelGGL(k_sol_store, dim3(elems_grid(a.dint)), dim3(256), 0, st, a, y, x);
    return hipGetLastError();
}

}  // namespace ncl
