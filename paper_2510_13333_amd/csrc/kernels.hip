// Device kernels of libnclkkt (gfx950, FP64, wave64).
//
// assemble      one thread per (block, bus), (block, generator), border pg:
//               polar power-flow Jacobian and Lagrangian Hessian plus Sigma,
//               the diagonal-dominance shift and -C (Section IV-B), written
//               straight into the lower-CSC values of K.
// factor_blocks one workgroup per block: level-scheduled left-looking
//               supernodal LDL^T without pivoting, panels in HBM, then the
//               block's border Schur contribution L_b D L_b^T.
// border_sum    S = K_bb - sum_k S_k, blocks summed in a fixed order.
// border_factor dense LDL^T of S in LDS (one workgroup).
// solve_fwd / solve_border / solve_bwd  the triangular solves in the same
//               structure (forward per block, border, backward per block).
// No floating-point atomics anywhere: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace ncl {

constexpr int kFactorThreads = 256;
constexpr int kSolveThreads = 256;
constexpr int kBorderThreads = 1024;

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

__device__ inline void put(const AsmArgs &a, int64_t kbase, int32_t slot, double v) {
    if (slot < 0) return;
    if (slot & kBorderFlag) a.kval[a.kbase_border + (slot & ~kBorderFlag)] = v;
    else a.kval[kbase + slot] = v;
}

__device__ inline int64_t zi(const AsmArgs &a, const BlockDev &B, int n, int32_t x) {
    return x < n ? B.col0 + x : a.bstart + (x - n);
}

__global__ __launch_bounds__(256) void k_assemble(AsmArgs a) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nbus_t = int64_t(a.nblk) * a.nb;
    const int64_t ngen_t = int64_t(a.nblk) * a.ng;
    const double irho = 1.0 / a.rho;
    if (tid < nbus_t) {
        const int blk = int(tid / a.nb), i = int(tid % a.nb);
        const BlockDev B = a.blks[blk];
        const TemplDev &T = a.tmpls[B.tmpl];
        const int n = T.n;
        const int32_t *bi = T.bus_idx + size_t(i) * BI_N;
        const double vi = a.z[zi(a, B, n, bi[BI_VM])];
        const double ti = a.z[zi(a, B, n, bi[BI_VA])];
        double Hvv = 0, Haa = 0, Hva = 0, dPv = 0, dPa = 0, dQv = 0, dQa = 0, absv = 0, absa = 0;
        for (int q = T.bus_adj_ptr[i]; q < T.bus_adj_ptr[i + 1]; q++) {
            const int32_t e = T.bus_adj[q];
            const bool self_from = e >= 0;
            const int l = self_from ? e : ~e;
            const int32_t *br = T.br_idx + size_t(l) * 4;
            const int f = br[2], t = br[3];
            const int32_t *bf = T.bus_idx + size_t(f) * BI_N, *bt = T.bus_idx + size_t(t) * BI_N;
            const double vf = a.z[zi(a, B, n, bf[BI_VM])], vt = a.z[zi(a, B, n, bt[BI_VM])];
            const double tf = a.z[zi(a, B, n, bf[BI_VA])], tt = a.z[zi(a, B, n, bt[BI_VA])];
            const double yPf = a.z[zi(a, B, n, bf[BI_P])], yQf = a.z[zi(a, B, n, bf[BI_Q])];
            const double yPt = a.z[zi(a, B, n, bt[BI_P])], yQt = a.z[zi(a, B, n, bt[BI_Q])];
            const double yFf = a.z[zi(a, B, n, br[0])], yFt = a.z[zi(a, B, n, br[1])];
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
                put(a, B.kbase, s[LS_VMVM], W[0][1]);
                put(a, B.kbase, s[LS_VMVA], W[0][3]);
                put(a, B.kbase, s[LS_VAVM], W[2][1]);
                put(a, B.kbase, s[LS_VAVA], W[2][3]);
                put(a, B.kbase, s[LS_PF_VMT], ef.gP[1]);
                put(a, B.kbase, s[LS_PF_VAT], ef.gP[3]);
                put(a, B.kbase, s[LS_QF_VMT], ef.gQ[1]);
                put(a, B.kbase, s[LS_QF_VAT], ef.gQ[3]);
                put(a, B.kbase, s[LS_PT_VMF], et.gP[1]);
                put(a, B.kbase, s[LS_PT_VAF], et.gP[3]);
                put(a, B.kbase, s[LS_QT_VMF], et.gQ[1]);
                put(a, B.kbase, s[LS_QT_VAF], et.gQ[3]);
                // flow rows: grad (P^2 + Q^2) = 2 P gP + 2 Q gQ
                double hf[4], ht[4];
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    hf[c] = 2.0 * ef.P * ef.gP[c] + 2.0 * ef.Q * ef.gQ[c];
                    ht[c] = 2.0 * et.P * et.gP[c] + 2.0 * et.Q * et.gQ[c];
                }
                put(a, B.kbase, s[LS_FF_VMF], hf[0]);
                put(a, B.kbase, s[LS_FF_VMT], hf[1]);
                put(a, B.kbase, s[LS_FF_VAF], hf[2]);
                put(a, B.kbase, s[LS_FF_VAT], hf[3]);
                put(a, B.kbase, s[LS_FT_VMF], ht[1]);
                put(a, B.kbase, s[LS_FT_VMT], ht[0]);
                put(a, B.kbase, s[LS_FT_VAF], ht[3]);
                put(a, B.kbase, s[LS_FT_VAT], ht[2]);
                put(a, B.kbase, s[LS_FFFF], -irho);
                put(a, B.kbase, s[LS_FTFT], -irho);
            }
        }
        (void)vi;
        (void)ti;
        const double dv = fmax(0.0, absv + fabs(Hva) - Hvv);
        const double da = fmax(0.0, absa + fabs(Hva) - Haa);
        const int32_t *bs = T.bus_slot + size_t(i) * BS_N;
        put(a, B.kbase, bs[BS_VMVM], Hvv + dv + a.sig[zi(a, B, n, bi[BI_VM])]);
        put(a, B.kbase, bs[BS_VAVA], Haa + da + a.sig[zi(a, B, n, bi[BI_VA])]);
        put(a, B.kbase, bs[BS_VMVA], Hva);
        put(a, B.kbase, bs[BS_PVM], dPv);
        put(a, B.kbase, bs[BS_PVA], dPa);
        put(a, B.kbase, bs[BS_QVM], dQv);
        put(a, B.kbase, bs[BS_QVA], dQa);
        put(a, B.kbase, bs[BS_PP], -irho);
        put(a, B.kbase, bs[BS_QQ], -irho);
        return;
    }
    if (tid < nbus_t + ngen_t) {
        const int64_t u = tid - nbus_t;
        const int blk = int(u / a.ng), g = int(u % a.ng);
        const BlockDev B = a.blks[blk];
        const TemplDev &T = a.tmpls[B.tmpl];
        const int n = T.n;
        const int32_t *gi = T.gen_idx + size_t(g) * GI_N;
        const int32_t *gs = T.gen_slot + size_t(g) * GS_N;
        put(a, B.kbase, gs[GS_PPG], -1.0);
        put(a, B.kbase, gs[GS_QQG], -1.0);
        put(a, B.kbase, gs[GS_QGQG], a.sig[zi(a, B, n, gi[GI_QG])]);
        if (T.has_pg_local) {
            const double h = 2.0 * a.gen_c2[g];
            put(a, B.kbase, gs[GS_PGPG], h + fmax(0.0, -h) + a.sig[zi(a, B, n, gi[GI_PG])]);
        }
        if (T.pvpq_rows) {
            const double nup = a.z[zi(a, B, n, gi[GI_NUP])], num = a.z[zi(a, B, n, gi[GI_NUM])];
            const double sup = a.z[zi(a, B, n, gi[GI_SUP])], slo = a.z[zi(a, B, n, gi[GI_SLO])];
            const int64_t cu = zi(a, B, n, gi[GI_CUP]), cl = zi(a, B, n, gi[GI_CLO]);
            const double n0u = a.z[cu], n0l = a.z[cl];
            put(a, B.kbase, gs[GS_LIN_NUP], 1.0);
            put(a, B.kbase, gs[GS_LIN_NUM], -1.0);
            put(a, B.kbase, gs[GS_LIN_VM], -1.0);
            put(a, B.kbase, gs[GS_LIN_VM0], 1.0);
            put(a, B.kbase, gs[GS_DUP_SUP], 1.0);
            put(a, B.kbase, gs[GS_DUP_QG], 1.0);
            put(a, B.kbase, gs[GS_DLO_SLO], 1.0);
            put(a, B.kbase, gs[GS_DLO_QG], -1.0);
            put(a, B.kbase, gs[GS_CUP_NUM], sup);
            put(a, B.kbase, gs[GS_CUP_SUP], num);
            put(a, B.kbase, gs[GS_CLO_NUP], slo);
            put(a, B.kbase, gs[GS_CLO_SLO], nup);
            put(a, B.kbase, gs[GS_H_NUM_SUP], n0u);
            put(a, B.kbase, gs[GS_H_NUP_SLO], n0l);
            put(a, B.kbase, gs[GS_NUPNUP], fabs(n0l) + a.sig[zi(a, B, n, gi[GI_NUP])]);
            put(a, B.kbase, gs[GS_NUMNUM], fabs(n0u) + a.sig[zi(a, B, n, gi[GI_NUM])]);
            put(a, B.kbase, gs[GS_SUPSUP], fabs(n0u) + a.sig[zi(a, B, n, gi[GI_SUP])]);
            put(a, B.kbase, gs[GS_SLOSLO], fabs(n0l) + a.sig[zi(a, B, n, gi[GI_SLO])]);
            put(a, B.kbase, gs[GS_LL], -irho);
            put(a, B.kbase, gs[GS_UU], -irho);
            put(a, B.kbase, gs[GS_DD], -irho);
            put(a, B.kbase, gs[GS_CUCU], -(irho + a.sig[cu] / n0u));
            put(a, B.kbase, gs[GS_CLCL], -(irho + a.sig[cl] / n0l));
        }
        return;
    }
    const int64_t g = tid - nbus_t - ngen_t;
    if (g < a.ng && a.nbd > 0) {
        const int bidx = a.border_pg[g];
        const int32_t p = a.kbb_pos[size_t(bidx) * a.nbd + bidx];
        const double h = 2.0 * a.gen_c2[g];
        if (p >= 0) a.kval[a.kbase_border + p] = h + fmax(0.0, -h) + a.sig[a.bstart + bidx];
    }
}

// ------------------------------------------------------------------ factor



__device__ inline int pivot_code(double d, bool primal) {
    if (!isfinite(d)) return 3;                 // non-finite
    if (d == 0.0) return 2;                     // zero
    if ((d > 0.0) != primal) return 1;          // wrong sign
    return 0;
}

__global__ __launch_bounds__(kFactorThreads) void k_factor_blocks(FactorArgs fa) {
    const int blk = blockIdx.x;
    const int tid = threadIdx.x;
    const BlockDev B = fa.blks[blk];
    const TemplDev &T = fa.tmpls[B.tmpl];
    double *__restrict__ L = fa.lpan + B.lbase;
    double *__restrict__ D = fa.dval + B.col0;
    const double *__restrict__ Kv = fa.kval + B.kbase;
    __shared__ double acc[kMaxW * kFactorThreads];
    __shared__ int64_t red_i[4][kFactorThreads / 64];
    __shared__ double red_d[2][kFactorThreads / 64];
    double *my = acc + tid;
    int64_t npos = 0, nneg = 0, nzero = 0, bad = INT64_MAX;
    double dmin = INFINITY, dmax = 0.0;

    for (int lev = 0; lev < T.nlev; lev++) {
        const int t0 = T.lev_task_ptr[lev], t1 = T.lev_task_ptr[lev + 1];
        // A: gather the K entries and every descendant's update into each panel row
        for (int k = t0 + tid; k < t1; k += kFactorThreads) {
            const int s = T.task_s[k], p = T.task_p[k];
            const int w = T.sup_first[s + 1] - T.sup_first[s];
            const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
            for (int c = 0; c < w; c++) my[c * kFactorThreads] = 0.0;
            for (int e = T.task_aptr[k]; e < T.task_aptr[k + 1]; e++) {
                const AEnt ae = T.aents[e];
                my[ae.crel * kFactorThreads] = Kv[ae.kpos];
            }
            for (int e = T.task_gptr[k]; e < T.task_gptr[k + 1]; e++) {
                const GItem gi = T.gitems[e];
                const int ld = gi.meta & 0xffff, wd = (gi.meta >> 16) & 0xff, nc = (gi.meta >> 24) & 0xff;
                const double *Li = L + gi.ioff;
                const double *Lc = L + gi.coff;
                const double *Dd = D + gi.dcol;
                const uint8_t *cr = T.crel + gi.crel;
                for (int kk = 0; kk < wd; kk++) {
                    const double tv = Li[kk * ld] * Dd[kk];
                    for (int q = 0; q < nc; q++) my[cr[q] * kFactorThreads] -= tv * Lc[q + kk * ld];
                }
            }
            double *P = L + T.panel_off[s] + p;
            for (int c = 0; c < w; c++) P[c * r] = my[c * kFactorThreads];
        }
        __syncthreads();
        // B: dense LDL^T of each supernode's diagonal block (one thread per supernode)
        for (int q = T.lev_sup_ptr[lev] + tid; q < T.lev_sup_ptr[lev + 1]; q += kFactorThreads) {
            const int s = T.lev_sup[q];
            const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
            const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
            double *P = L + T.panel_off[s];
            for (int j = 0; j < w; j++) {
                double dj = P[j * r + j];
                for (int kk = 0; kk < j; kk++) {
                    const double l = P[kk * r + j];
                    dj -= l * D[f + kk] * l;
                }
                D[f + j] = dj;
                const int code = pivot_code(dj, T.col_primal[f + j] != 0);
                if (code == 0 || code == 1) {
                    if (dj > 0) npos++;
                    else nneg++;
                } else if (code == 2) nzero++;
                if (code && bad == INT64_MAX) bad = (B.col0 + f + j) * 8 + code;
                const double ad = fabs(dj);
                dmin = fmin(dmin, ad);
                dmax = fmax(dmax, ad);
                for (int i = j + 1; i < w; i++) {
                    double v = P[j * r + i];
                    for (int kk = 0; kk < j; kk++) v -= P[kk * r + i] * D[f + kk] * P[kk * r + j];
                    P[j * r + i] = v / dj;
                }
                P[j * r + j] = 1.0;
            }
        }
        __syncthreads();
        // C: off-diagonal rows, L[i, :] = P[i, :] L_ss^{-T} D^{-1}
        for (int k = t0 + tid; k < t1; k += kFactorThreads) {
            const int s = T.task_s[k], p = T.task_p[k];
            const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
            if (p < w) continue;
            const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
            double *P = L + T.panel_off[s];
            for (int j = 0; j < w; j++) {
                double v = P[j * r + p];
                for (int kk = 0; kk < j; kk++) v -= my[kk * kFactorThreads] * D[f + kk] * P[kk * r + j];
                v /= D[f + j];
                my[j * kFactorThreads] = v;
                P[j * r + p] = v;
            }
        }
        __syncthreads();
    }
    // border Schur contribution S_k[i][j] = sum over common panels L[i,:] D L[j,:]^T
    if (fa.nbd > 0) {
        const int nbd = fa.nbd;
        const int64_t npk = int64_t(nbd) * (nbd + 1) / 2;
        double *Sk = fa.spart + int64_t(blk) * npk;
        for (int64_t e = tid; e < npk; e += kFactorThreads) {
            int i = int((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
            while (int64_t(i) * (i + 1) / 2 > e) i--;
            while (int64_t(i + 1) * (i + 2) / 2 <= e) i++;
            const int j = int(e - int64_t(i) * (i + 1) / 2);
            double sum = 0.0;
            int ai = T.bpath_ptr[i + 1] - 1, aj = T.bpath_ptr[j + 1] - 1;
            const int ai0 = T.bpath_ptr[i], aj0 = T.bpath_ptr[j];
            while (ai >= ai0 && aj >= aj0) {
                const int si = T.bpath_s[ai], sj = T.bpath_s[aj];
                if (si == sj) {
                    const int f = T.sup_first[si], w = T.sup_first[si + 1] - f;
                    const int r = T.sup_rowptr[si + 1] - T.sup_rowptr[si];
                    const double *P = L + T.panel_off[si];
                    const int pi = T.bpath_pos[ai], pj = T.bpath_pos[aj];
                    for (int kk = 0; kk < w; kk++) sum += P[kk * r + pi] * D[f + kk] * P[kk * r + pj];
                    ai--;
                    aj--;
                } else if (si > sj) ai--;
                else aj--;
            }
            Sk[e] = sum;
        }
    }
    // block status, reduced in a fixed order
    {
        const int lane = tid & 63, wv = tid >> 6;
        for (int o = 32; o > 0; o >>= 1) {
            npos += __shfl_xor(npos, o);
            nneg += __shfl_xor(nneg, o);
            nzero += __shfl_xor(nzero, o);
            const int64_t ob = __shfl_xor(bad, o);
            bad = ob < bad ? ob : bad;
            dmin = fmin(dmin, __shfl_xor(dmin, o));
            dmax = fmax(dmax, __shfl_xor(dmax, o));
        }
        if (lane == 0) {
            red_i[0][wv] = npos;
            red_i[1][wv] = nneg;
            red_i[2][wv] = nzero;
            red_i[3][wv] = bad;
            red_d[0][wv] = dmin;
            red_d[1][wv] = dmax;
        }
        __syncthreads();
        if (tid == 0) {
            int64_t a0 = 0, a1 = 0, a2 = 0, a3 = INT64_MAX;
            double m0 = INFINITY, m1 = 0.0;
            for (int q = 0; q < kFactorThreads / 64; q++) {
                a0 += red_i[0][q];
                a1 += red_i[1][q];
                a2 += red_i[2][q];
                a3 = red_i[3][q] < a3 ? red_i[3][q] : a3;
                m0 = fmin(m0, red_d[0][q]);
                m1 = fmax(m1, red_d[1][q]);
            }
            int64_t *st = fa.stat + int64_t(blk) * 4;
            st[0] = a0;
            st[1] = a1;
            st[2] = a2;
            st[3] = a3;
            fa.dminmax[2 * blk] = m0;
            fa.dminmax[2 * blk + 1] = m1;
        }
    }
}

// ------------------------------------------------------------------ border



__global__ __launch_bounds__(256) void k_border_sum(BorderArgs a) {
    const int64_t npk = int64_t(a.nbd) * (a.nbd + 1) / 2;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= npk) return;
    int i = int((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
    while (int64_t(i) * (i + 1) / 2 > e) i--;
    while (int64_t(i + 1) * (i + 2) / 2 <= e) i++;
    const int j = int(e - int64_t(i) * (i + 1) / 2);
    const int32_t p = a.kbb_pos[size_t(i) * a.nbd + j];
    double s = p >= 0 ? a.kval[a.kbase_border + p] : 0.0;
    for (int b = 0; b < a.nblk; b++) s -= a.spart[int64_t(b) * npk + e];
    a.sbb[e] = s;
}

__device__ inline int pk(int i, int j) { return i * (i + 1) / 2 + j; }

__global__ __launch_bounds__(kBorderThreads) void k_border_factor(BorderArgs a, int use_lds) {
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
        const double dj = S[pk(j, j)];
        const double inv = 1.0 / dj;
        for (int i = j + 1 + ty; i < nbd; i += 32) {
            const double ci = S[pk(i, j)] * inv;
            for (int k = j + 1 + tx; k <= i; k += 32) S[pk(i, k)] -= ci * S[pk(k, j)];
        }
        __syncthreads();
    }
    // pivots, then scale the columns into L (strict part)
    int64_t npos = 0, nneg = 0, nzero = 0, bad = INT64_MAX;
    double dmin = INFINITY, dmax = 0.0;
    for (int j = tid; j < nbd; j += kBorderThreads) {
        const double dj = S[pk(j, j)];
        a.dval[a.bcol0 + j] = dj;
        const int code = pivot_code(dj, a.bprimal[j] != 0);
        if (code == 0 || code == 1) {
            if (dj > 0) npos++;
            else nneg++;
        } else if (code == 2) nzero++;
        if (code && bad == INT64_MAX) bad = (a.bcol0 + j) * 8 + code;
        dmin = fmin(dmin, fabs(dj));
        dmax = fmax(dmax, fabs(dj));
    }
    __syncthreads();
    for (int e = tid; e < npk; e += kBorderThreads) {
        int i = int((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
        while (i * (i + 1) / 2 > e) i--;
        while ((i + 1) * (i + 2) / 2 <= e) i++;
        const int j = e - i * (i + 1) / 2;
        a.sbb[e] = (i == j) ? 1.0 : S[e] / a.dval[a.bcol0 + j];
    }
    __shared__ int64_t ri[4][kBorderThreads / 64];
    __shared__ double rd[2][kBorderThreads / 64];
    const int lane = tid & 63, wv = tid >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        npos += __shfl_xor(npos, o);
        nneg += __shfl_xor(nneg, o);
        nzero += __shfl_xor(nzero, o);
        const int64_t ob = __shfl_xor(bad, o);
        bad = ob < bad ? ob : bad;
        dmin = fmin(dmin, __shfl_xor(dmin, o));
        dmax = fmax(dmax, __shfl_xor(dmax, o));
    }
    if (lane == 0) {
        ri[0][wv] = npos; ri[1][wv] = nneg; ri[2][wv] = nzero; ri[3][wv] = bad;
        rd[0][wv] = dmin; rd[1][wv] = dmax;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t a0 = 0, a1 = 0, a2 = 0, a3 = INT64_MAX;
        double m0 = INFINITY, m1 = 0.0;
        for (int q = 0; q < kBorderThreads / 64; q++) {
            a0 += ri[0][q]; a1 += ri[1][q]; a2 += ri[2][q];
            a3 = ri[3][q] < a3 ? ri[3][q] : a3;
            m0 = fmin(m0, rd[0][q]); m1 = fmax(m1, rd[1][q]);
        }
        int64_t *st = a.stat + int64_t(a.nblk) * 4;
        st[0] = a0; st[1] = a1; st[2] = a2; st[3] = a3;
        a.dminmax[2 * a.nblk] = m0;
        a.dminmax[2 * a.nblk + 1] = m1;
    }
}

// ------------------------------------------------------------------ solve



__global__ __launch_bounds__(kSolveThreads) void k_solve_fwd(SolveArgs a) {
    const int blk = blockIdx.x, tid = threadIdx.x;
    const BlockDev B = a.blks[blk];
    const TemplDev &T = a.tmpls[B.tmpl];
    const double *__restrict__ L = a.lpan + B.lbase;
    for (int rhs = 0; rhs < a.nrhs; rhs++) {
        double *y = a.ybuf + int64_t(rhs) * a.N + B.col0;
        const double *bb = a.b + int64_t(rhs) * a.ld + B.col0;
        for (int j = tid; j < T.n; j += kSolveThreads) y[j] = bb[T.perm[j]];
        __syncthreads();
        for (int lev = 0; lev < T.nlev; lev++) {
            for (int q = T.lev_dtask_ptr[lev] + tid; q < T.lev_dtask_ptr[lev + 1]; q += kSolveThreads) {
                const int k = T.dtask[q];
                const int s = T.task_s[k], p = T.task_p[k];
                const int col = T.sup_first[s] + p;
                double v = y[col];
                for (int e = T.task_gptr[k]; e < T.task_gptr[k + 1]; e++) {
                    const GItem gi = T.gitems[e];
                    const int ldd = gi.meta & 0xffff, wd = (gi.meta >> 16) & 0xff;
                    const double *Li = L + gi.ioff;
                    for (int kk = 0; kk < wd; kk++) v -= Li[kk * ldd] * y[gi.dcol + kk];
                }
                y[col] = v;
            }
            __syncthreads();
            for (int q = T.lev_sup_ptr[lev] + tid; q < T.lev_sup_ptr[lev + 1]; q += kSolveThreads) {
                const int s = T.lev_sup[q];
                const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
                const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
                const double *P = L + T.panel_off[s];
                for (int j = 1; j < w; j++) {
                    double v = y[f + j];
                    for (int kk = 0; kk < j; kk++) v -= P[kk * r + j] * y[f + kk];
                    y[f + j] = v;
                }
            }
            __syncthreads();
        }
        // this block's contribution to the border rows
        for (int bi = tid; bi < a.nbd; bi += kSolveThreads) {
            double v = 0.0;
            for (int e = T.bpath_ptr[bi]; e < T.bpath_ptr[bi + 1]; e++) {
                const int s = T.bpath_s[e], pos = T.bpath_pos[e];
                const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
                const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
                const double *P = L + T.panel_off[s];
                for (int kk = 0; kk < w; kk++) v += P[kk * r + pos] * y[f + kk];
            }
            a.cpart[(int64_t(rhs) * a.nblk + blk) * a.nbd + bi] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBorderThreads) void k_solve_border(SolveArgs a) {
    extern __shared__ double c[];
    const int nbd = a.nbd, tid = threadIdx.x;
    const double *Db = a.dval + a.bstart;
    for (int rhs = 0; rhs < a.nrhs; rhs++) {
        for (int i = tid; i < nbd; i += kBorderThreads) {
            double v = a.b[int64_t(rhs) * a.ld + a.bstart + i];
            for (int k = 0; k < a.nblk; k++) v -= a.cpart[(int64_t(rhs) * a.nblk + k) * nbd + i];
            c[i] = v;
        }
        __syncthreads();
        for (int j = 0; j < nbd; j++) {
            const double cj = c[j];
            for (int i = j + 1 + tid; i < nbd; i += kBorderThreads) c[i] -= a.sbb[pk(i, j)] * cj;
            __syncthreads();
        }
        for (int i = tid; i < nbd; i += kBorderThreads) c[i] /= Db[i];
        __syncthreads();
        for (int j = nbd - 1; j >= 0; j--) {
            // c[j] is final; remove its contribution from the rows above
            const double cj = c[j];
            for (int i = tid; i < j; i += kBorderThreads) c[i] -= a.sbb[pk(j, i)] * cj;
            __syncthreads();
        }
        for (int i = tid; i < nbd; i += kBorderThreads) {
            a.ybuf[int64_t(rhs) * a.N + a.bstart + i] = c[i];
            a.x[int64_t(rhs) * a.ld + a.bstart + i] = c[i];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSolveThreads) void k_solve_bwd(SolveArgs a) {
    const int blk = blockIdx.x, tid = threadIdx.x;
    const BlockDev B = a.blks[blk];
    const TemplDev &T = a.tmpls[B.tmpl];
    const double *__restrict__ L = a.lpan + B.lbase;
    const double *D = a.dval + B.col0;
    for (int rhs = 0; rhs < a.nrhs; rhs++) {
        double *y = a.ybuf + int64_t(rhs) * a.N + B.col0;
        const double *xb = a.ybuf + int64_t(rhs) * a.N + a.bstart;
        for (int j = tid; j < T.n; j += kSolveThreads) y[j] /= D[j];
        __syncthreads();
        for (int lev = T.nlev - 1; lev >= 0; lev--) {
            for (int q = T.lev_dtask_ptr[lev] + tid; q < T.lev_dtask_ptr[lev + 1]; q += kSolveThreads) {
                const int k = T.dtask[q];
                const int s = T.task_s[k], p = T.task_p[k];
                const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
                const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
                const int32_t *R = T.sup_rows + T.sup_rowptr[s];
                const double *Pc = L + T.panel_off[s] + int64_t(p) * r;
                double v = y[f + p];
                for (int i = w; i < r; i++) {
                    const int row = R[i];
                    v -= Pc[i] * (row < T.n ? y[row] : xb[row - T.n]);
                }
                y[f + p] = v;
            }
            __syncthreads();
            for (int q = T.lev_sup_ptr[lev] + tid; q < T.lev_sup_ptr[lev + 1]; q += kSolveThreads) {
                const int s = T.lev_sup[q];
                const int f = T.sup_first[s], w = T.sup_first[s + 1] - f;
                const int r = T.sup_rowptr[s + 1] - T.sup_rowptr[s];
                const double *P = L + T.panel_off[s];
                for (int j = w - 2; j >= 0; j--) {
                    double v = y[f + j];
                    for (int kk = j + 1; kk < w; kk++) v -= P[j * r + kk] * y[f + kk];
                    y[f + j] = v;
                }
            }
            __syncthreads();
        }
        double *xo = a.x + int64_t(rhs) * a.ld + B.col0;
        for (int j = tid; j < T.n; j += kSolveThreads) xo[T.perm[j]] = y[j];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_assemble(const AsmArgs &a, hipStream_t st) {
    const int64_t total = int64_t(a.nblk) * (a.nb + a.ng) + a.ng;
    const int64_t grid = (total + 255) / 256;
    hipLaunchKernelGGL(k_assemble, dim3(unsigned(grid)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_factor_blocks(const FactorArgs &fa, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_factor_blocks, dim3(nblk), dim3(kFactorThreads), 0, st, fa);
    return hipGetLastError();
}

hipError_t launch_factor_border(const BorderArgs &ba, hipStream_t st) {
    if (ba.nbd == 0) return hipSuccess;
    const int64_t npk = int64_t(ba.nbd) * (ba.nbd + 1) / 2;
    hipLaunchKernelGGL(k_border_sum, dim3(unsigned((npk + 255) / 256)), dim3(256), 0, st, ba);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lbytes = size_t(npk) * sizeof(double);
    const int use_lds = lbytes <= 160 * 1024 - 4096 ? 1 : 0;
    hipLaunchKernelGGL(k_border_factor, dim3(1), dim3(kBorderThreads), use_lds ? lbytes : 0, st, ba, use_lds);
    return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_solve_fwd, dim3(a.nblk), dim3(kSolveThreads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.nbd > 0) {
        hipLaunchKernelGGL(k_solve_border, dim3(1), dim3(kBorderThreads), size_t(a.nbd) * sizeof(double), st, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_solve_bwd, dim3(a.nblk), dim3(kSolveThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace ncl
