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
#include <mutex>
#include <type_traits>

#include "kernels.h"

namespace ncl {

constexpr int kWG = 256;                 // threads per workgroup of the list kernels (4 wavefronts)
constexpr int kBorderThreads = 1024;

// Schedule tables are read-only during a launch and indexed uniformly across
// a wavefront; reading them through the constant address space lets the
// compiler use scalar loads (one per wavefront, through the scalar cache)
// instead of per-lane vector loads that each wait for memory.
template <class T>
__device__ inline const __attribute__((address_space(4))) T *cs(const T *p) {
    return (const __attribute__((address_space(4))) T *)p;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b mod 8).  The list kernels renumber them so that each XCD takes one
// contiguous range of the work list (a bijection of [0, gridDim.x)): items
// that share data then share an L2.
constexpr int kXcd = 8;

// Element idx of a per-template array whose byte offsets fit 32 bits (a
// bound checked at analysis): the uniform base stays in scalar registers
// and the offset is one 32-bit vector value, so an address costs one
// scalar multiply-add and one vector add instead of 64-bit scalar
// arithmetic.
__device__ inline double ld32(const double *base, uint32_t idx) {
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + (idx << 3));
}
__device__ inline void st32(double *base, uint32_t idx, double v) {
    *reinterpret_cast<double *>(reinterpret_cast<char *>(base) + (idx << 3)) = v;
}

__device__ inline int xcd_workgroup() {
    const int G = int(gridDim.x), b = int(blockIdx.x);
    const int q = G / kXcd, r = G % kXcd;
    const int x = b % kXcd, i = b / kXcd;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ inline int wave_id() {
    return __builtin_amdgcn_readfirstlane(xcd_workgroup() * (kWG / 64) + int(threadIdx.x >> 6));
}
__device__ inline int lane_id() { return int(threadIdx.x & 63); }

// Update sums over a contiguous run of terms [t0, t1).  Terms are taken in
// rounds of 8, then 4, 2 and 1: each round loads its (uniform) descriptors,
// then issues every vector load of the round before the first use, so that
// a wavefront keeps many loads in flight instead of waiting on each product
// in turn, and no load is wasted on padding.

// U[a] L[c] (= L[a] d[k] L[c], U = L D) for R consecutive terms, added
// into R partial sums
template <int R>
__device__ inline void tdot_round(const double *__restrict__ Lb, const double *__restrict__ Ub, uint32_t nb,
                                  uint32_t bl, const Term *__restrict__ tm, double *s) {
    double p[R];
#pragma unroll
    for (int u = 0; u < R; u++) {
        const auto *q = cs(tm) + u;
        p[u] = ld32(Ub, uint32_t(q->a) * nb + bl) * ld32(Lb, uint32_t(q->c) * nb + bl);
    }
#pragma unroll
    for (int u = 0; u < R; u++) s[u] += p[u];
}

// sum over terms of U[a] L[c] (template bases Lb, Ub; the lane's block bl)
__device__ inline double tdot(const double *__restrict__ Lb, const double *__restrict__ Ub, uint32_t nb, uint32_t bl,
                              const Term *__restrict__ tm, int t0, int t1) {
    double s[8];
#pragma unroll
    for (int u = 0; u < 8; u++) s[u] = 0.0;
    int t = t0;
    for (; t + 8 <= t1; t += 8) tdot_round<8>(Lb, Ub, nb, bl, tm + t, s);
    if (t + 4 <= t1) { tdot_round<4>(Lb, Ub, nb, bl, tm + t, s); t += 4; }
    if (t + 2 <= t1) { tdot_round<2>(Lb, Ub, nb, bl, tm + t, s + 4); t += 2; }
    if (t < t1) tdot_round<1>(Lb, Ub, nb, bl, tm + t, s + 6);
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// L[a] y[k] for R consecutive terms
template <int R>
__device__ inline void ydot_round(const double *__restrict__ Lb, const double *yb, uint32_t nb, uint32_t bl,
                                  const Term *__restrict__ tm, double *s) {
    double p[R];
#pragma unroll
    for (int u = 0; u < R; u++) {
        const auto *q = cs(tm) + u;
        p[u] = ld32(Lb, uint32_t(q->a) * nb + bl) * ld32(yb, uint32_t(q->k) * nb + bl);
    }
#pragma unroll
    for (int u = 0; u < R; u++) s[u] += p[u];
}

// Split sums.  A long run of terms is summed as four partials: full rounds
// of 8 go round-robin to partials 0..3, the tail (rounds of 4, 2, 1) to
// partial 0, and the total is (p0 + p1) + (p2 + p3).  One wavefront can
// compute all four in turn, or four wavefronts one each (then a workgroup
// combines them through LDS): the bits are the same either way, so a
// launch may pick the split by how many tasks it has.
constexpr int kSplit = 4;

// partial q of the split sum of L[a] y[k] over terms [t0, t1) (template
// bases Lb, yb; the lane's block bl)
__device__ inline double ydot_q(const double *__restrict__ Lb, const double *yb, uint32_t nb, uint32_t bl,
                                const Term *__restrict__ tm, int t0, int t1, int q) {
    double s[8];
#pragma unroll
    for (int u = 0; u < 8; u++) s[u] = 0.0;
    const int nc = (t1 - t0) >> 3;
    for (int c = q; c < nc; c += kSplit) ydot_round<8>(Lb, yb, nb, bl, tm + t0 + 8 * c, s);
    if (q == 0) {
        int t = t0 + 8 * nc;
        if (t + 4 <= t1) { ydot_round<4>(Lb, yb, nb, bl, tm + t, s); t += 4; }
        if (t + 2 <= t1) { ydot_round<2>(Lb, yb, nb, bl, tm + t, s + 4); t += 2; }
        if (t < t1) ydot_round<1>(Lb, yb, nb, bl, tm + t, s + 6);
    }
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Task and partial of the calling wavefront: NW = 1, one task per
// wavefront computing every partial; NW = kSplit, one task per workgroup,
// wavefront q computing partial q.
template <int NW>
__device__ inline int split_task() {
    if (NW == 1) return wave_id();
    return xcd_workgroup();
}

// Combine the partials of the split sum: v holds partial q (NW = kSplit) or
// the caller's own total (NW = 1).  Returns the total in wavefront 0; the
// other wavefronts get false and must not write.
template <int NW>
__device__ inline bool split_combine(double &v) {
    if (NW == 1) return true;
    __shared__ double red[kSplit][64];
    const int q = int(threadIdx.x >> 6), lane = lane_id();
    red[q][lane] = v;
    __syncthreads();
    if (q != 0) return false;
    v = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    return true;
}

template <int NW, class F>
__device__ inline double split_sum(F &&part) {
    if (NW == 1) return (part(0) + part(1)) + (part(2) + part(3));
    return part(int(threadIdx.x >> 6));
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

// instance owning a flat index of a concatenated per-instance array
__device__ inline int find_inst(const DevArgs &a, int64_t idx, int64_t InstDev::*base) {
    int lo = 0, hi = a.ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.insts[mid].*base <= idx) lo = mid;
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
// kSwap: the sending end is the branch's to-end, so variable a of the end
// (v_s, v_o, th_s, th_o) is variable a ^ 1 of the branch order.
template <bool kSwap>
__device__ inline void branch_end(double g, double b, double vs, double vo, double ts, double to, double wP,
                                  double wQ, double wF, double W[4][4], EndDeriv &e) {
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
            const int ia = kSwap ? (a ^ 1) : a, ic = kSwap ? (c ^ 1) : c;
            W[ia][ic] += h;
            if (ia != ic) W[ic][ia] += h;
        }
}

// The state z and Sigma (layout order) transposed to the interleaved order
// of the factor storage, layout-local element j of a template's block bl at
// dbase + j * nblk + bl; the border values of every instance follow at
// dint + bd0.  Per template the state is an [nblk][n] array (blocks of a
// template are contiguous in layout order, one block after the other),
// moved through LDS in tiles of kTileJ columns x kTileB blocks: reads run
// along j (kTileJ contiguous values of one block), writes along bl (kTileB
// contiguous values of one column).  The tile is narrow in j so that a
// launch holds several workgroups per compute unit.
struct TileIx {
    const TemplDev *T;
    int j0, b0;
};

__device__ inline TileIx tile_index(const DevArgs &a, int64_t t) {
    const TemplDev &T = a.tmpls[find_tmpl(a, t, &TemplDev::tile0)];
    const int64_t tt = t - T.tile0;
    const int nbt = (T.nblk + kTileB - 1) / kTileB;
    return TileIx{&T, int(tt / nbt) * kTileJ, int(tt % nbt) * kTileB};
}

// per thread: kTileJ * kTileB / 256 values in each phase
constexpr int kTileR = kTileJ * kTileB / 256;
constexpr int kTileRows = 256 / kTileJ;   // blocks read per pass in the first phase
static_assert(kTileB == 64 && 256 % kTileJ == 0 && kTileR * 4 == kTileJ, "tile shape");

__global__ __launch_bounds__(256) void k_interleave(DevArgs a, const double *__restrict__ z,
                                                    const double *__restrict__ sig, double *__restrict__ zd,
                                                    double *__restrict__ sd) {
    __shared__ double tile[kTileB][kTileJ + 1];
    const int64_t t = blockIdx.x;
    if (t >= a.tiles) {
        // border values: a plain copy
        const int64_t i = (t - a.tiles) * 256 + threadIdx.x;
        if (i < a.nbd_tot) {
            const InstDev &I = a.insts[find_inst(a, i, &InstDev::bd0)];
            const int64_t col = I.bstart + (i - I.bd0);
            zd[a.dint + i] = z[col];
            sd[a.dint + i] = sig[col];
        }
        return;
    }
    const TileIx x = tile_index(a, t);
    const TemplDev &T = *x.T;
    const int cj = threadIdx.x % kTileJ, rb = threadIdx.x / kTileJ;
    const int cb = threadIdx.x & 63, rj = threadIdx.x >> 6;
    // every load of both arrays is issued before the first barrier
    double vz[kTileR], vs[kTileR];
#pragma unroll
    for (int q = 0; q < kTileR; q++) {
        const int bl = x.b0 + rb + kTileRows * q, j = x.j0 + cj;
        const bool ok = bl < T.nblk && j < T.n;
        const int64_t src = ok ? a.blks[T.blocks[bl]].col0 + j : 0;
        vz[q] = ok ? z[src] : 0.0;
        vs[q] = ok ? sig[src] : 0.0;
    }
    for (int pass = 0; pass < 2; pass++) {
        double *dst = pass ? sd : zd;
#pragma unroll
        for (int q = 0; q < kTileR; q++) tile[rb + kTileRows * q][cj] = pass ? vs[q] : vz[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kTileR; q++) {
            const int j = x.j0 + rj + 4 * q, bl = x.b0 + cb;
            if (bl < T.nblk && j < T.n) dst[T.dbase + int64_t(j) * T.nblk + bl] = tile[cb][rj + 4 * q];
        }
        __syncthreads();
    }
}

struct AsmCtx {
    const DevArgs *a;
    int64_t kb;      // template K base + the lane's block
    int64_t nb;      // blocks of the template (stride)
    int64_t kbb;     // the instance's K_bb values
    bool on;         // the lane holds a block (idle lanes write nothing)
};

__device__ inline void put(const AsmCtx &c, int32_t slot, double v) {
    if (slot < 0 || !c.on) return;
    if (slot & kBorderFlag) c.a->kval[c.kbb + (slot & ~kBorderFlag)] = v;
    else c.a->kval[c.kb + int64_t(uint32_t(slot) * uint32_t(c.nb))] = v;   // a template's K fits 2^29
}

__device__ inline int64_t zi(int64_t bstart, const BlockDev &B, int n, int32_t x) {
    return x < n ? B.col0 + x : bstart + (x - n);
}

// Threads: per template, one wavefront per (bus, group of 64 blocks), then
// per (generator, group), the lane running over the blocks of the group so
// that neighbouring lanes write neighbouring interleaved values; then the
// border pg diagonal of every instance.
// index of layout-local element x of the lane's block in the interleaved state
struct StateIx {
    int64_t base, nb, bord;
    int n;
    // x * nb in 32 bits: a template's pivots fit 2^29 (checked at analysis)
    __device__ int64_t operator()(int32_t x) const {
        return x < n ? base + int64_t(uint32_t(x) * uint32_t(nb)) : bord + (x - n);
    }
};

__global__ __launch_bounds__(256) void k_assemble(DevArgs a, const double *__restrict__ z,
                                                  const double *__restrict__ sig, double rho, int noshift) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const double irho = 1.0 / rho;
    const double shift = noshift ? 0.0 : 1.0;    // diagonal-dominance shift on (1) or off (0)
    if (tid >= a.asm_wthreads) {
        const int64_t gg = tid - a.asm_wthreads;
        if (gg >= a.gp_tot) return;
        const InstDev &I = a.insts[find_inst(a, gg, &InstDev::gp0)];
        const int g = int(gg - I.gp0);
        if (I.nbd == 0 || g >= I.ng) return;
        const int bidx = I.border_pg[g];
        const int32_t p = I.kbb_pos[size_t(bidx) * I.nbd + bidx];
        const double h = 2.0 * I.gen_c2[g];
        if (p >= 0) a.kval[a.kint + I.kbb0 + p] = h + shift * fmax(0.0, -h) + a.sint[a.dint + I.bd0 + bidx];
        return;
    }
    // one wavefront per (bus or generator j, group of 64 blocks): j and every
    // table index are uniform, so the tables are read through scalar loads
    const int64_t wt0 = int64_t(blockIdx.x) * blockDim.x + 64 * __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const TemplDev &T = a.tmpls[find_tmpl(a, wt0, &TemplDev::awbase)];
    const int ngr = (T.nblk + 63) >> 6;
    const int wloc = int((wt0 - T.awbase) >> 6);
    const int j = wloc / ngr;
    const int b = (wloc - j * ngr) * 64 + lane_id();
    const bool on = b < T.nblk;
    const int bl = on ? b : T.nblk - 1;           // idle lanes read a valid block and write nothing
    const int64_t kbb = a.kint + a.insts[T.inst].kbb0;
    const double *__restrict__ zs = a.zint;
    const double *__restrict__ ss = a.sint;
    if (j < T.nbus) {
        const int i = j;
        const BlockDev B = a.blks[T.blocks[bl]];
        const int n = T.n;
        const AsmCtx cx{&a, T.kbase + bl, T.nblk, kbb, on};
        const StateIx ix{T.dbase + bl, T.nblk, a.dint + T.bd0, n};
        const auto *bi = cs(T.bus_idx) + size_t(i) * BI_N;
        double Hvv = 0, Haa = 0, Hva = 0, dPv = 0, dPa = 0, dQv = 0, dQa = 0, absv = 0, absa = 0;
        for (int q = cs(T.bus_adj_ptr)[i]; q < cs(T.bus_adj_ptr)[i + 1]; q++) {
            const int32_t e = cs(T.bus_adj)[q];
            const bool self_from = e >= 0;
            const int l = self_from ? e : ~e;
            const auto *br = cs(T.br_idx) + size_t(l) * 4;
            const int f = br[2], t = br[3];
            const auto *bf = cs(T.bus_idx) + size_t(f) * BI_N, *bt = cs(T.bus_idx) + size_t(t) * BI_N;
            const double vf = zs[ix(bf[BI_VM])], vt = zs[ix(bt[BI_VM])];
            const double tf = zs[ix(bf[BI_VA])], tt = zs[ix(bt[BI_VA])];
            const double yPf = zs[ix(bf[BI_P])], yQf = zs[ix(bf[BI_Q])];
            const double yPt = zs[ix(bt[BI_P])], yQt = zs[ix(bt[BI_Q])];
            const double yFf = zs[ix(br[0])], yFt = zs[ix(br[1])];
            const double st = (l == B.outage) ? 0.0 : 1.0;
            const double r = cs(T.br_r)[l], x = cs(T.br_x)[l];
            const double den = r * r + x * x;
            const double g = st * (r / den), b = st * (-x / den);
            double W[4][4] = {};
            EndDeriv ef, et;
            branch_end<false>(g, b, vf, vt, tf, tt, yPf, yQf, yFf, W, ef);
            branch_end<true>(g, b, vt, vf, tt, tf, yPt, yQt, yFt, W, et);
            // this bus's variables are (v, th) = branch variables (0, 2) at the
            // from end, (1, 3) at the to end; selects keep W in registers
            Hvv += self_from ? W[0][0] : W[1][1];
            Haa += self_from ? W[2][2] : W[3][3];
            Hva += self_from ? W[0][2] : W[1][3];
            absv += self_from ? fabs(W[0][1]) + fabs(W[0][3]) : fabs(W[1][0]) + fabs(W[1][2]);
            absa += self_from ? fabs(W[2][1]) + fabs(W[2][3]) : fabs(W[3][0]) + fabs(W[3][2]);
            dPv += self_from ? ef.gP[0] : et.gP[0];
            dPa += self_from ? ef.gP[2] : et.gP[2];
            dQv += self_from ? ef.gQ[0] : et.gQ[0];
            dQa += self_from ? ef.gQ[2] : et.gQ[2];
            if (self_from) {
                const auto *s = cs(T.br_slot) + size_t(l) * LS_N;
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
                put(cx, s[LS_FFFF], -(irho + ss[ix(br[0])]));
                put(cx, s[LS_FTFT], -(irho + ss[ix(br[1])]));
            }
        }
        const double dv = shift * fmax(0.0, absv + fabs(Hva) - Hvv);
        const double da = shift * fmax(0.0, absa + fabs(Hva) - Haa);
        const auto *bs = cs(T.bus_slot) + size_t(i) * BS_N;
        put(cx, bs[BS_VMVM], Hvv + dv + ss[ix(bi[BI_VM])]);
        put(cx, bs[BS_VAVA], Haa + da + ss[ix(bi[BI_VA])]);
        put(cx, bs[BS_VMVA], Hva);
        put(cx, bs[BS_PVM], dPv);
        put(cx, bs[BS_PVA], dPa);
        put(cx, bs[BS_QVM], dQv);
        put(cx, bs[BS_QVA], dQa);
        put(cx, bs[BS_PP], -(irho + ss[ix(bi[BI_P])]));
        put(cx, bs[BS_QQ], -(irho + ss[ix(bi[BI_Q])]));
        return;
    }
    {
        const int g = j - T.nbus;
        const int n = T.n;
        const AsmCtx cx{&a, T.kbase + bl, T.nblk, kbb, on};
        const StateIx ix{T.dbase + bl, T.nblk, a.dint + T.bd0, n};
        const auto *gi = cs(T.gen_idx) + size_t(g) * GI_N;
        const auto *gs = cs(T.gen_slot) + size_t(g) * GS_N;
        put(cx, gs[GS_PPG], -1.0);
        put(cx, gs[GS_QQG], -1.0);
        put(cx, gs[GS_QGQG], ss[ix(gi[GI_QG])]);
        if (T.has_pg_local) {
            const double h = 2.0 * cs(T.gen_c2)[g];
            put(cx, gs[GS_PGPG], h + shift * fmax(0.0, -h) + ss[ix(gi[GI_PG])]);
        }
        if (T.pvpq_rows) {
            const double nup = zs[ix(gi[GI_NUP])], num = zs[ix(gi[GI_NUM])];
            const double sup = zs[ix(gi[GI_SUP])], slo = zs[ix(gi[GI_SLO])];
            const int64_t cu = ix(gi[GI_CUP]), cl = ix(gi[GI_CLO]);
            const double n0u = zs[cu], n0l = zs[cl];
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
            put(cx, gs[GS_NUPNUP], shift * fabs(n0l) + ss[ix(gi[GI_NUP])]);
            put(cx, gs[GS_NUMNUM], shift * fabs(n0u) + ss[ix(gi[GI_NUM])]);
            put(cx, gs[GS_SUPSUP], shift * fabs(n0u) + ss[ix(gi[GI_SUP])]);
            put(cx, gs[GS_SLOSLO], shift * fabs(n0l) + ss[ix(gi[GI_SLO])]);
            put(cx, gs[GS_LL], -(irho + ss[ix(gi[GI_LIN])]));
            put(cx, gs[GS_UU], -(irho + ss[ix(gi[GI_DUP])]));
            put(cx, gs[GS_DD], -(irho + ss[ix(gi[GI_DLO])]));
            put(cx, gs[GS_CUCU], -(irho + ss[cu] / n0u));
            put(cx, gs[GS_CLCL], -(irho + ss[cl] / n0l));
        }
        if (T.agc_rows) {
            // eq. (droopmpec): ALIN = pi+ - pi- - pgk + pg0 + alpha delta, the
            // two slack rows, and the products pi- sp_up, pi+ sp_lo with their
            // nu0 Hessian pairs; pgk and delta have no Hessian (no shift)
            const double pip = zs[ix(gi[GI_PIP])], pim = zs[ix(gi[GI_PIM])];
            const double spu = zs[ix(gi[GI_SPU])], spl = zs[ix(gi[GI_SPL])];
            const int64_t au = ix(gi[GI_ACUP]), al = ix(gi[GI_ACLO]);
            const double n0u = zs[au], n0l = zs[al];
            put(cx, gs[GS_ALIN_PIP], 1.0);
            put(cx, gs[GS_ALIN_PIM], -1.0);
            put(cx, gs[GS_ALIN_PGK], -1.0);
            put(cx, gs[GS_ALIN_PG0], 1.0);
            put(cx, gs[GS_ALIN_DEL], cs(T.gen_alpha)[g]);
            put(cx, gs[GS_ADUP_SPU], 1.0);
            put(cx, gs[GS_ADUP_PGK], 1.0);
            put(cx, gs[GS_ADLO_SPL], 1.0);
            put(cx, gs[GS_ADLO_PGK], -1.0);
            put(cx, gs[GS_ACUP_PIM], spu);
            put(cx, gs[GS_ACUP_SPU], pim);
            put(cx, gs[GS_ACLO_PIP], spl);
            put(cx, gs[GS_ACLO_SPL], pip);
            put(cx, gs[GS_H_PIM_SPU], n0u);
            put(cx, gs[GS_H_PIP_SPL], n0l);
            put(cx, gs[GS_PIPPIP], shift * fabs(n0l) + ss[ix(gi[GI_PIP])]);
            put(cx, gs[GS_PIMPIM], shift * fabs(n0u) + ss[ix(gi[GI_PIM])]);
            put(cx, gs[GS_SPUSPU], shift * fabs(n0u) + ss[ix(gi[GI_SPU])]);
            put(cx, gs[GS_SPLSPL], shift * fabs(n0l) + ss[ix(gi[GI_SPL])]);
            put(cx, gs[GS_PGKPGK], ss[ix(gi[GI_PG])]);
            put(cx, gs[GS_AL], -(irho + ss[ix(gi[GI_ALIN])]));
            put(cx, gs[GS_AU], -(irho + ss[ix(gi[GI_ADUP])]));
            put(cx, gs[GS_AD], -(irho + ss[ix(gi[GI_ADLO])]));
            put(cx, gs[GS_ACUACU], -(irho + ss[au] / n0u));
            put(cx, gs[GS_ACLACL], -(irho + ss[al] / n0l));
            if (gs[GS_DELDEL] >= 0) put(cx, gs[GS_DELDEL], ss[ix(gi[GI_DELTA])]);
        }
    }
}

// Public lower-CSC values <-> internal (interleaved blocks, then each
// instance's K_bb).
__global__ __launch_bounds__(256) void k_values(DevArgs a, const double *__restrict__ src, double *__restrict__ dst,
                                                int to_internal) {
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
    } else if (idx < a.kint + a.nbb_tot) {
        const int64_t p = idx - a.kint;
        const InstDev &I = a.insts[find_inst(a, p, &InstDev::kbb0)];
        const int64_t c = I.kcsc_border + (p - I.kbb0);
        if (to_internal) dst[idx] = src[c];
        else dst[c] = src[idx];
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
// supernodes that hold the entry's row and column (one term per column of
// each descendant).
__global__ __launch_bounds__(kWG) void k_fac_gather(DevArgs a, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const int e = W.k;
    const int kp = cs(T.ent_kpos)[e];
    double v = kp >= 0 ? a.kval[T.kbase + W.bl + int64_t(kp) * nb] : 0.0;
    v -= tdot(a.lpan + T.lbase, a.upan + T.lbase, uint32_t(nb), uint32_t(W.bl), T.terms, cs(T.ent_tptr)[e],
              cs(T.ent_tptr)[e + 1]);
    if (W.on) a.lpan[T.lbase + W.bl + int64_t(cs(T.ent_out)[e]) * nb] = v;
}

// Width classes: kernels that walk the columns of a supernode are
// instantiated for W = 1, 2, 4, 8, 12, 16, 24, 32 and run the smallest class
// holding the supernode's width w (a uniform branch).  Inside a class every
// loop bound is a compile-time constant; loads past w are clamped to column
// w-1 (a valid address) and their contributions masked, so no load waits on
// a run-time branch.
// the same, for widths up to WMAX only (a launch whose items are all that
// narrow keeps the register count of its narrow paths)
template <int WMAX, class F>
__device__ inline void by_width_max(int w, F &&f) {
    if (w <= 1) f(std::integral_constant<int, 1>());
    else if (w <= 2) f(std::integral_constant<int, 2>());
    else if (w <= 4) f(std::integral_constant<int, 4>());
    else if (w <= 8 || WMAX <= 8) f(std::integral_constant<int, 8>());
    else if (w <= 12) f(std::integral_constant<int, (WMAX < 12 ? WMAX : 12)>());
    else if (w <= 16 || WMAX <= 16) f(std::integral_constant<int, (WMAX < 16 ? WMAX : 16)>());
    else if (w <= 24) f(std::integral_constant<int, (WMAX < 24 ? WMAX : 24)>());
    else f(std::integral_constant<int, WMAX>());
}

template <class F>
__device__ inline void by_width(int w, F &&f) {
    if (w <= 1) f(std::integral_constant<int, 1>());
    else if (w <= 2) f(std::integral_constant<int, 2>());
    else if (w <= 4) f(std::integral_constant<int, 4>());
    else if (w <= 8) f(std::integral_constant<int, 8>());
    else if (w <= 12) f(std::integral_constant<int, 12>());
    else if (w <= 16) f(std::integral_constant<int, 16>());
    else if (w <= 24) f(std::integral_constant<int, 24>());
    else f(std::integral_constant<int, 32>());
}

// B: LDL^T of the diagonal block of a wide supernode.  Two blocks per
// wavefront; lane i of each half holds row i of its block's diagonal block
// in registers.  Right-looking: at step j each row publishes its column-j
// value through LDS, every lane reads the pivot and the column by broadcast
// reads, and row i takes l_ij = a_ij / d_j and a_ik -= l_ij a_kj (k <= i).
// Row i ends with l_ik (k < i) and d_i.
// Width-1 supernodes, one per wavefront (in the diagonal-block launch, not
// in the row kernel, whose wide classes would set their occupancy): d =
// P(0,0) and L(p,0) = P(p,0) / d for the rows p below it, their loads all in
// flight together; U(p,0) = L(p,0) d is the row's value before the division.
__device__ inline void fac_pivots(const DevArgs &a, const TemplDev &T, int s, int g) {
    const uint32_t nb = uint32_t(T.nblk);
    const uint32_t bl = uint32_t(g * 64 + lane_id());
    if (bl >= nb) return;
    const int r = cs(T.sup_rowptr)[s + 1] - cs(T.sup_rowptr)[s];
    double *Lb = a.lpan + T.lbase, *Ub = a.upan + T.lbase;
    const uint32_t po = uint32_t(cs(T.panel_off)[s]);
    const double d = ld32(Lb, po * nb + bl);
    st32(a.dval + T.dbase, uint32_t(cs(T.sup_first)[s]) * nb + bl, d);
    int p = 1;
    for (; p + 4 <= r; p += 4) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = ld32(Lb, (po + uint32_t(p + u)) * nb + bl);
#pragma unroll
        for (int u = 0; u < 4; u++) {
            st32(Lb, (po + uint32_t(p + u)) * nb + bl, v[u] / d);
            st32(Ub, (po + uint32_t(p + u)) * nb + bl, v[u]);
        }
    }
    for (; p < r; p++) {
        const double v = ld32(Lb, (po + uint32_t(p)) * nb + bl);
        st32(Lb, (po + uint32_t(p)) * nb + bl, v / d);
        st32(Ub, (po + uint32_t(p)) * nb + bl, v);
    }
}

// Narrow diagonal blocks (w <= kNarrowW): one block per lane, the whole
// block in registers, the same right-looking steps (and so the same bits)
// as the wide path.
template <int W>
__device__ inline void diag_narrow(const DevArgs &a, const TemplDev &T, int s, int g) {
    const uint32_t nb = uint32_t(T.nblk);
    const uint32_t b = uint32_t(g * 64 + lane_id());
    if (b >= nb) return;
    const int f = cs(T.sup_first)[s], w = cs(T.sup_first)[s + 1] - f;
    const int r = cs(T.sup_rowptr)[s + 1] - cs(T.sup_rowptr)[s];
    double *Lb = a.lpan + T.lbase;
    const uint32_t po = uint32_t(cs(T.panel_off)[s]);
    // element (row, col) of the panel for this lane's block
    auto at = [&](int col, int row) { return (po + uint32_t(col) * uint32_t(r) + uint32_t(row)) * nb + b; };
    const int wl1 = w - 1;
    double A[W][W];
#pragma unroll
    for (int i = 0; i < W; i++)
#pragma unroll
        for (int k = 0; k <= i; k++) {
            const double v = ld32(Lb, at(k < w ? k : wl1, i < w ? i : wl1));   // clamped inside the panel
            A[i][k] = (i < w) ? v : 0.0;
        }
#pragma unroll
    for (int j = 0; j < W; j++) {
        if (j < w) {
            const double dj = A[j][j];
            double l[W];
#pragma unroll
            for (int i = j + 1; i < W; i++) l[i] = A[i][j] / dj;
            // A[k][j] is read before any row's column j is scaled
#pragma unroll
            for (int i = j + 1; i < W; i++)
#pragma unroll
                for (int k = j + 1; k <= i; k++) A[i][k] -= l[i] * A[k][j];
#pragma unroll
            for (int i = j + 1; i < W; i++) A[i][j] = l[i];
        }
    }
#pragma unroll
    for (int i = 0; i < W; i++) {
        if (i < w) {
#pragma unroll
            for (int k = 0; k < i; k++) st32(Lb, at(k, i), A[i][k]);
            st32(a.dval + T.dbase, uint32_t(f + i) * nb + b, A[i][i]);
        }
    }
}

__global__ __launch_bounds__(kWG) void k_fac_diag(DevArgs a, const Work *__restrict__ wl, int nw) {
    __shared__ double cbuf[kWG / 64][2][2][kMaxW];     // wavefront, step parity, half, row
    const int wid = wave_id();
    if (wid >= nw) return;
    const int lane = lane_id(), wv = int(threadIdx.x >> 6);
    const int half = lane >> 5, i = lane & 31;
    const Work wk = wl[wid];
    const TemplDev &T = a.tmpls[wk.tg >> 16];
    if (wk.k & kPivotFlag) {
        fac_pivots(a, T, wk.k & ~kPivotFlag, wk.tg & 0xffff);
        return;
    }
    if (wk.k & kNarrowFlag) {
        const int sn = wk.k & ~kNarrowFlag;
        const int wn = cs(T.sup_first)[sn + 1] - cs(T.sup_first)[sn];
        const int g = wk.tg & 0xffff;
        if (wn <= 2) diag_narrow<2>(a, T, sn, g);
        else if (wn <= 4) diag_narrow<4>(a, T, sn, g);
        else diag_narrow<kNarrowW>(a, T, sn, g);
        return;
    }
    const int nb = T.nblk;
    const int b = (wk.tg & 0xffff) * 2 + half;
    const int bl = b < nb ? b : 0;
    const int s = wk.k;
    const int f = cs(T.sup_first)[s], w = cs(T.sup_first)[s + 1] - f;
    const int r = cs(T.sup_rowptr)[s + 1] - cs(T.sup_rowptr)[s];
    const bool on = b < nb && i < w;
    double *Lb = a.lpan + T.lbase;
    const uint32_t po = uint32_t(cs(T.panel_off)[s]), nbu = uint32_t(nb), blu = uint32_t(bl);
    // element (row, col) of the panel for this lane's block
    auto at = [&](int col, int row) { return (po + uint32_t(col) * uint32_t(r) + uint32_t(row)) * nbu + blu; };
    by_width(w, [&](auto Wc) {
        constexpr int W = decltype(Wc)::value;
        const int wl1 = w - 1, ic = i < w ? i : wl1;
        double row[W];
#pragma unroll
        for (int k = 0; k < W; k++) {
            const double v = ld32(Lb, at(k < w ? k : wl1, ic));
            row[k] = (k <= i && i < w && k < w) ? v : 0.0;
        }
#pragma unroll
        for (int j = 0; j < W; j++) {
            if (j < w) {
                double *cb = cbuf[wv][j & 1][half];
                if (i >= j && i < w) cb[i] = row[j];
                __builtin_amdgcn_wave_barrier();
                const double dj = cb[j];
                const double lij = i > j ? row[j] / dj : 0.0;
#pragma unroll
                for (int k = j + 1; k < W; k++) {
                    const double ak = cb[k];
                    const double upd = row[k] - lij * ak;
                    row[k] = (i >= k && k < w) ? upd : row[k];          // select, no divergent branch
                }
                row[j] = i > j ? lij : row[j];
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (on) {
            double di = 0.0;
#pragma unroll
            for (int k = 0; k < W; k++) {
                if (k < i) st32(Lb, at(k, i), row[k]);
                if (k == i) di = row[k];
            }
            st32(a.dval + T.dbase, uint32_t(f + i) * nbu + blu, di);
        }
    });
}


// C: off-diagonal rows of wide supernodes (U(p,j) = u_j is kept too).  Row p >= w: u_j = L(p,j) d_j
// satisfies u_j = P(p,j) - sum_{k<j} L(j,k) u_k, solved right-looking
// (u_k -= L(k,j) u_j for k > j; the loads of L do not depend on u), then
// L(p,j) = u_j / d_j.
__global__ __launch_bounds__(kWG) void k_fac_rows(DevArgs a, const Work *__restrict__ wl, int nw) {
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const uint32_t nb = uint32_t(W.nb), bl = uint32_t(W.bl);
    const int s = cs(T.task_s)[W.k], p = cs(T.task_p)[W.k];
    const int f = cs(T.sup_first)[s], w = cs(T.sup_first)[s + 1] - f;
    const int r = cs(T.sup_rowptr)[s + 1] - cs(T.sup_rowptr)[s];
    double *Lb = a.lpan + T.lbase;
    double *Db = a.dval + T.dbase;
    const uint32_t po = uint32_t(cs(T.panel_off)[s]);
    // element (row, col) of the panel for this lane's block
    auto at = [&](int col, int row) { return (po + uint32_t(col) * uint32_t(r) + uint32_t(row)) * nb + bl; };
    by_width(w, [&](auto Wc) {
        constexpr int W_ = decltype(Wc)::value;
        const int wl1 = w - 1;
        double u[W_];
#pragma unroll
        for (int j = 0; j < W_; j++) u[j] = ld32(Lb, at(j < w ? j : wl1, p));
        // u_k -= L(k,j) u_j for j < k, row by row in increasing j.  Each row
        // of the diagonal block is loaded whole before its products, and
        // rows past the width (clamped loads) update values that are never
        // stored, with no select on the loaded values: with a select per
        // product the compiler kept one load in flight at a time in the
        // widest classes (hundreds of L2 round trips in a row); this way
        // about ten are.
#pragma unroll
        for (int k = 1; k < W_; k++) {
            const int kc = k < w ? k : wl1;
            double l[W_];
#pragma unroll
            for (int j = 0; j < k; j++) l[j] = ld32(Lb, at(j < w ? j : wl1, kc));
#pragma unroll
            for (int j = 0; j < k; j++) u[k] -= l[j] * u[j];
        }
        if (W.on) {
            double *Ub = a.upan + T.lbase;
#pragma unroll
            for (int j = 0; j < W_; j++) {
                const double d = ld32(Db, uint32_t(f + (j < w ? j : wl1)) * nb + bl);
                if (j < w) {
                    st32(Lb, at(j, p), u[j] / d);
                    st32(Ub, at(j, p), u[j]);
                }
            }
        }
    });
}

// Border Schur products on the matrix cores.  One wavefront per slice: a
// run of one tile pair's items (supernodes of one template holding rows of
// both border tiles I >= J) and one chunk of kMC blocks.  It sums
//     P[m][n] += U[I_m, k] L[J_n, k]        (U = L D on the panel rows)
// over the items' columns k and the chunk's blocks with v_mfma_f64_16x16x4:
// A[m][q] (the q-th of four products) sits in lane m + 16 q, B[q][n] in lane
// n + 16 q, and D[m][n] comes back in lane n + 16 (m % 4), register m / 4.
// A full chunk puts four blocks of one column on the inner dimension (two
// accumulators alternate over the column's four block quads); a chunk of
// fewer blocks (the base case's single block, the last chunk of a template)
// runs over (column, block) pairs in order, four at a time.  Rows an item
// does not hold enter as zeros.  Each slice writes its own partial tile to
// spart, and k_border_sum adds a pair's slices in order, so every entry has
// one fixed order of additions.
typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

// Slices are taken by a grid of workgroups each wave of which takes every
// (grid waves)-th slice: one wave per slice alone, at most kSchurGrid
// workgroups when the kernel runs beside the blocks' forward substitution
// (the combined factor and solve), so that it leaves compute units to it.
// A slice's result does not depend on which wave takes it.
constexpr int kSchurGrid = 128;

__device__ __attribute__((always_inline)) inline void border_schur_slice(const DevArgs &a, int64_t wg) {
    const InstDev &I = a.insts[find_inst(a, wg, &InstDev::mw0)];
    const int64_t wl = wg - I.mw0;
    const auto *dsc = cs(I.mdesc) + wl;
    const int ib = dsc->ib, ie = dsc->ie, chunk = dsc->chunk;
    const int lane = lane_id(), m = lane & 15, qd = lane >> 4;
    mfma_f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const auto *items = cs(I.mitems);
    // the next item's tile rows are loaded while the current item runs
    int ra_n = items[ib].ri[m], rb_n = items[ib].rj[m];
    for (int it = ib; it < ie; it++) {
        const TemplDev &T = a.tmpls[items[it].tmpl];
        const int nb = T.nblk, b0 = kMC * chunk, csz = min(kMC, nb - b0);
        const int ra = ra_n, rb = rb_n;
        if (it + 1 < ie) {
            ra_n = items[it + 1].ri[m];
            rb_n = items[it + 1].rj[m];
        }
        const int r = items[it].r, w = items[it].w, poff = items[it].poff;
        const double *__restrict__ Ub = a.upan + T.lbase;
        const double *__restrict__ Lb = a.lpan + T.lbase;
        const uint32_t nbu = uint32_t(nb), step = uint32_t(r) * nbu;
        const uint32_t ba = uint32_t(poff + (ra < 0 ? 0 : ra)) * nbu + uint32_t(b0);
        const uint32_t bb = uint32_t(poff + (rb < 0 ? 0 : rb)) * nbu + uint32_t(b0);
        const bool va = ra >= 0, vb = rb >= 0;
        if (csz == kMC) {
            uint32_t oa = ba + uint32_t(qd), ob = bb + uint32_t(qd);
            // two columns a round: 16 loads in flight before their 8 products
            int k = 0;
            for (; k + 2 <= w; k += 2, oa += 2 * step, ob += 2 * step) {
                double av[8], bv[8];
#pragma unroll
                for (int g = 0; g < 8; g++) {
                    const uint32_t o = (g < 4 ? 0u : step) + 4u * uint32_t(g & 3);
                    av[g] = va ? ld32(Ub, oa + o) : 0.0;
                    bv[g] = vb ? ld32(Lb, ob + o) : 0.0;
                }
#pragma unroll
                for (int g = 0; g < 8; g += 2) {
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g], bv[g], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g + 1], bv[g + 1], acc1, 0, 0, 0);
                }
            }
            if (k < w) {
                double av[4], bv[4];
#pragma unroll
                for (int g = 0; g < 4; g++) {
                    av[g] = va ? ld32(Ub, oa + 4 * g) : 0.0;
                    bv[g] = vb ? ld32(Lb, ob + 4 * g) : 0.0;
                }
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], bv[0], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], bv[1], acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[2], bv[2], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[3], bv[3], acc1, 0, 0, 0);
            }
        } else {
            // (column, block) pair t = k * csz + bl; lane quad qd takes t = t0 + qd
            const int tot = w * csz;
            int k = qd / csz, bl = qd - k * csz;
            for (int t0 = 0; t0 < tot; t0 += 4) {
                const bool in = t0 + qd < tot;
                const uint32_t o = uint32_t(k) * step + uint32_t(bl);
                const double av = (in && va) ? ld32(Ub, ba + o) : 0.0;
                const double bv = (in && vb) ? ld32(Lb, bb + o) : 0.0;
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc0, 0, 0, 0);
                bl += 4;
                while (bl >= csz) {
                    bl -= csz;
                    k++;
                }
            }
        }
    }
    double *out = a.spart + I.sp0 + wl * (kMT * kMT);
#pragma unroll
    for (int q = 0; q < 4; q++) out[(4 * q + qd) * kMT + m] = acc0[q] + acc1[q];
}

__global__ __launch_bounds__(kWG) void k_border_schur(DevArgs a) {
    const int64_t stride = int64_t(gridDim.x) * (kWG / 64);
    for (int64_t wg = int64_t(blockIdx.x) * (kWG / 64) + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
         wg < a.mw_tot; wg += stride)
        border_schur_slice(a, wg);
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

constexpr int kBB = 32;          // column block of the dense border factor and solves
constexpr int kPS = kBB + 1;     // LDS row stride of a staged block column

// S = K_bb - (the partial tiles of each tile pair summed in slice order):
// one thread per entry of every tile pair (neighbouring threads read
// neighbouring entries of each partial tile, up to 16 in flight).  Tile
// position q holds border row bperm[q]; an entry goes to the packed lower
// triangle at (max, min) of its two border rows, each unordered pair once
// (on a diagonal tile pair, the entries with m >= n).
__global__ __launch_bounds__(256) void k_border_sum(DevArgs a) {
    const int64_t tg = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (tg >= a.pe_tot) return;
    const InstDev &I = a.insts[find_inst(a, tg, &InstDev::pe0)];
    const int64_t u = tg - I.pe0;
    const int pq = int(u / (kMT * kMT)), e = int(u % (kMT * kMT));
    int ti = int((sqrt(8.0 * double(pq) + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > pq) ti--;
    while ((ti + 1) * (ti + 2) / 2 <= pq) ti++;
    const int tj = pq - ti * (ti + 1) / 2;
    const int qi = ti * kMT + e / kMT, qj = tj * kMT + e % kMT;
    if (qi >= I.nbd || qj >= I.nbd || (ti == tj && qj > qi)) return;
    const double *src = a.spart + I.sp0 + e;
    double s = 0.0;
    const int d1 = I.mdesc_ptr[pq + 1];
    int d = I.mdesc_ptr[pq];
    for (; d + 16 <= d1; d += 16) {
        double x[16];
#pragma unroll
        for (int q = 0; q < 16; q++) x[q] = src[int64_t(d + q) * (kMT * kMT)];
#pragma unroll
        for (int q = 0; q < 16; q++) s += x[q];
    }
    for (; d < d1; d++) s += src[int64_t(d) * (kMT * kMT)];
    const int bi = I.bperm[qi], bj = I.bperm[qj];
    const int i = max(bi, bj), j = min(bi, bj);
    const int32_t p = I.kbb_pos[size_t(i) * I.nbd + j];
    a.sbb[I.sbb0 + int64_t(i) * (i + 1) / 2 + j] = (p >= 0 ? a.kval[a.kint + I.kbb0 + p] : 0.0) - s;
}

// Dense LDL^T of the packed border matrix S (lower triangle packed by
// rows); the factor L (unit lower, packed the same way) goes to lbb and D to
// dval.  Borders of up to kBorderRegMax rows: k_border_factor, one
// workgroup per instance with the whole matrix in registers.  Larger ones:
// k_border_step, right-looking by column blocks of kBB, one launch per
// block, S left as the trailing matrices.
//   launch b = -1: one workgroup factors the diagonal block 0.
//   launch b >= 0: one workgroup per tile (I, K), b < K <= I, of the
//     trailing lower triangle.  It solves the rows of tiles I and K in block
//     column b against the block's factor (W = A L^-T, L = W D^-1, one
//     thread a row), takes S_IK -= W_I L_K^T, and, on the diagonal tile
//     I = K, writes L of tile I's rows in block column b.  The workgroup of
//     tile (b + 1, b + 1) then factors that updated diagonal block.
// Every workgroup reads only block column b of S and writes only its own
// tile, and L goes to a separate array, so no workgroup reads what another
// writes in the same launch.  Each entry's sums run in column order.

// LDL^T of the kBB x kBB block T (LDS, rows < bs, lower part valid) by
// wavefront 0, lane i holding row i, column j published through T's column
// j; L (strict lower, 1 on the diagonal) to Lg rows b0.., pivots to Dg.
__device__ inline void border_diag_ldlt(double (*T)[kPS], int bs, int b0, double *Lg, double *Dg) {
    const int i = lane_id();
    const bool on = i < bs;
    double row[kBB];
#pragma unroll
    for (int k = 0; k < kBB; k++) row[k] = (on && k <= i) ? T[on ? i : 0][k] : 0.0;
#pragma unroll
    for (int j = 0; j < kBB; j++) {
        if (j < bs) {
            if (on && i >= j) T[i][j] = row[j];
            __builtin_amdgcn_wave_barrier();
            const double dj = T[j][j];
            const double lij = i > j ? row[j] / dj : 0.0;
#pragma unroll
            for (int k = j + 1; k < kBB; k++) {
                const double ak = T[k][j];
                const double upd = row[k] - lij * ak;
                row[k] = (i >= k && k < bs) ? upd : row[k];
            }
            row[j] = i > j ? lij : row[j];
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (on) {
#pragma unroll
        for (int k = 0; k < kBB; k++) {
            if (k < i) Lg[pk(b0 + i, b0 + k)] = row[k];
            if (k == i) {
                Lg[pk(b0 + i, b0 + i)] = 1.0;
                Dg[b0 + i] = row[k];
            }
        }
    }
}

constexpr int kBFThreads = 512;    // 8 wavefronts: up to 256 registers each, no spills

// Dense LDL^T of a border matrix held in registers.  The lower triangle is
// cut into 4x4 tiles numbered column by column; thread t holds tiles t,
// t + kBFThreads, ... (at most T).  For each panel p of 4 columns:
//  (1) the owner of tile (p, p) factors it (pivots d_p, unit lower L_pp)
//      and publishes it in LDS;
//  (2) the owner of each tile (I, p), I > p, forms W = A_Ip L_pp^{-T}
//      (= L_Ip D_p) and L_Ip = W D_p^{-1}, and publishes both rows;
//  (3) every tile (I, K) with I >= K > p takes A_IK -= W_I L_K^T.
// Two barriers a panel and no copy of the matrix in LDS.  Rows padded past
// nbd carry pivot 1 and no coupling; only real entries are written out.
constexpr int kBFRegMaxNt = 54;    // tile rows a thread's 3 tiles cover: 54 * 55 / 2 <= 3 * kBFThreads (nbd <= 216)
static_assert(4 * kBFRegMaxNt == kBorderRegMax && kBB == kBorderBlock, "border factor split");

template <int T>
__device__ inline void border_factor_reg(const DevArgs &a, const InstDev &I, double *piv, double *pan) {
    const int nbd = I.nbd, tid = threadIdx.x;
    if (nbd == 0) return;
    const int mt = (nbd + 3) >> 2, npad = 4 * mt, ntl = mt * (mt + 1) / 2;
    const double *Sg = a.sbb + I.sbb0;
    double *Lo = a.lbb + I.sbb0;
    double *Db = a.dval + a.dint + I.bd0;
    double *Wp = pan, *Lp = pan + 4 * npad;      // [k][row] for k < 4, rows < npad
    double A[T][16];
    int ti[T], tk[T];
#pragma unroll
    for (int j = 0; j < T; j++) {
        const int q = tid + j * kBFThreads;
        int K = -1, i0 = -1;
        if (q < ntl) {
            int off = 0;
            K = 0;
            while (off + (mt - K) <= q) {
                off += mt - K;
                K++;
            }
            i0 = K + (q - off);
        }
        ti[j] = i0;
        tk[j] = K;
        // every load is issued (entries outside the matrix read entry (0, 0)
        // and are replaced after), so that the tiles' loads are in flight
        // together rather than one guarded group at a time
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int i = 4 * i0 + r, k = 4 * K + c;
                const bool in = q < ntl && i < nbd && k <= i;
                A[j][4 * r + c] = Sg[in ? pk(i, k) : 0];
            }
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int i = 4 * i0 + r, k = 4 * K + c;
                const bool in = q < ntl && i < nbd && k <= i;
                if (!in) A[j][4 * r + c] = (q < ntl && i == k) ? 1.0 : 0.0;
            }
    }
    for (int p = 0; p < mt; p++) {
#pragma unroll
        for (int j = 0; j < T; j++) {
            if (tk[j] == p && ti[j] == p) {
                const double *x = A[j];
                const double d0 = x[0], r0 = 1.0 / d0;
                const double l10 = x[4] * r0, l20 = x[8] * r0, l30 = x[12] * r0;
                const double d1 = x[5] - l10 * x[4], r1 = 1.0 / d1;
                const double w21 = x[9] - l20 * x[4], w31 = x[13] - l30 * x[4];
                const double l21 = w21 * r1, l31 = w31 * r1;
                const double d2 = x[10] - l20 * x[8] - l21 * w21, r2 = 1.0 / d2;
                const double w32 = x[14] - l30 * x[8] - l31 * w21;
                const double l32 = w32 * r2;
                const double d3 = x[15] - l30 * x[12] - l31 * w31 - l32 * w32, r3 = 1.0 / d3;
                piv[0] = d0; piv[1] = d1; piv[2] = d2; piv[3] = d3;
                piv[4] = r0; piv[5] = r1; piv[6] = r2; piv[7] = r3;
                piv[8] = l10; piv[9] = l20; piv[10] = l21; piv[11] = l30; piv[12] = l31; piv[13] = l32;
                // the tile now holds D on its diagonal and L below it
                A[j][0] = d0; A[j][5] = d1; A[j][10] = d2; A[j][15] = d3;
                A[j][4] = l10; A[j][8] = l20; A[j][9] = l21; A[j][12] = l30; A[j][13] = l31; A[j][14] = l32;
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < T; j++) {
            if (tk[j] == p && ti[j] > p) {
                const double l10 = piv[8], l20 = piv[9], l21 = piv[10], l30 = piv[11], l31 = piv[12], l32 = piv[13];
                const double r0 = piv[4], r1 = piv[5], r2 = piv[6], r3 = piv[7];
                const int row0 = 4 * ti[j];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const double *x = A[j] + 4 * r;
                    const double w0 = x[0];
                    const double w1 = x[1] - w0 * l10;
                    const double w2 = x[2] - w0 * l20 - w1 * l21;
                    const double w3 = x[3] - w0 * l30 - w1 * l31 - w2 * l32;
                    const double y0 = w0 * r0, y1 = w1 * r1, y2 = w2 * r2, y3 = w3 * r3;
                    const int i = row0 + r;
                    Wp[i] = w0; Wp[npad + i] = w1; Wp[2 * npad + i] = w2; Wp[3 * npad + i] = w3;
                    Lp[i] = y0; Lp[npad + i] = y1; Lp[2 * npad + i] = y2; Lp[3 * npad + i] = y3;
                    A[j][4 * r] = y0; A[j][4 * r + 1] = y1; A[j][4 * r + 2] = y2; A[j][4 * r + 3] = y3;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < T; j++) {
            if (tk[j] > p) {
                const int ri = 4 * ti[j], rk = 4 * tk[j];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const double2 wa = *reinterpret_cast<const double2 *>(Wp + k * npad + ri);
                    const double2 wb = *reinterpret_cast<const double2 *>(Wp + k * npad + ri + 2);
                    const double2 la = *reinterpret_cast<const double2 *>(Lp + k * npad + rk);
                    const double2 lb = *reinterpret_cast<const double2 *>(Lp + k * npad + rk + 2);
                    const double w[4] = {wa.x, wa.y, wb.x, wb.y};
                    const double l[4] = {la.x, la.y, lb.x, lb.y};
#pragma unroll
                    for (int r = 0; r < 4; r++)
#pragma unroll
                        for (int c = 0; c < 4; c++) A[j][4 * r + c] -= w[r] * l[c];
                }
            }
        }
    }
    // write the factor out once, after the last barrier: global stores
    // inside the panel loop would make every barrier wait for them
#pragma unroll
    for (int j = 0; j < T; j++) {
        if (tk[j] < 0) continue;
        const int c0 = 4 * tk[j];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int i = 4 * ti[j] + r;
            if (i >= nbd) continue;
            double *si = Lo + pk(i, c0);
#pragma unroll
            for (int c = 0; c < 4; c++) {
                if (c0 + c > i) continue;
                if (c0 + c == i) {
                    si[c] = 1.0;
                    Db[i] = A[j][5 * r];
                } else {
                    si[c] = A[j][4 * r + c];
                }
            }
        }
    }
}

// One workgroup per instance.  Each instance takes the register-tiled factor
// when its tiles fit T per thread, else the blocked one (k_border_step), so
// that the path an instance takes depends on its own border only (a batched
// launch and a launch for that instance alone compute the same bits).
template <int T>
__global__ __launch_bounds__(kBFThreads) void k_border_factor(DevArgs a) {
    __shared__ double piv[16];    // d (0..3), 1/d (4..7), l10 l20 l21 l30 l31 l32 (8..13)
    extern __shared__ __align__(16) double lds[];
    const InstDev &I = a.insts[blockIdx.x];
    const int mt = (I.nbd + 3) >> 2;
    if (mt <= kBFRegMaxNt) border_factor_reg<T>(a, I, piv, lds);   // larger: k_border_step
}


constexpr int kBSThreads = 256;

__global__ __launch_bounds__(kBSThreads) void k_border_step(DevArgs a, int b) {
    __shared__ double Lbb[kBB][kPS];   // L of block b's diagonal block
    __shared__ double db[kBB];         // its pivots
    __shared__ double Wi[kBB][kPS];    // W of tile I's rows in block column b
    __shared__ double Lk[kBB][kPS];    // L of tile K's rows in block column b
    __shared__ double Tn[kBB][kPS];    // the next diagonal block, updated
    const InstDev &I = a.insts[blockIdx.y];
    const int n = I.nbd, nbk = (n + kBB - 1) / kBB, tid = threadIdx.x;
    if (n <= kBorderRegMax) return;
    double *S = a.sbb + I.sbb0;
    double *Lg = a.lbb + I.sbb0;
    double *Dg = a.dval + a.dint + I.bd0;
    // the diagonal block this workgroup factors at the end (none: -1)
    int dg0 = -1, dgs = 0;
    if (b < 0) {
        if (blockIdx.x != 0 || n == 0) return;
        dgs = n < kBB ? n : kBB;
        dg0 = 0;
        for (int e = tid; e < kBB * kBB; e += kBSThreads) {
            const int r = e / kBB, c = e % kBB;
            Tn[r][c] = (r < dgs && c <= r) ? S[pk(r, c)] : 0.0;
        }
    } else {
        const int rem = nbk - b - 1;
        if (rem <= 0 || int(blockIdx.x) >= rem * (rem + 1) / 2) return;
        int ti, tk;
        unpack(blockIdx.x, ti, tk);
        const int TI = b + 1 + ti, TK = b + 1 + tk;
        const int b0 = b * kBB, i0 = TI * kBB, k0 = TK * kBB;
        const int bsb = n - b0 < kBB ? n - b0 : kBB;
        const int bsi = n - i0 < kBB ? n - i0 : kBB;
        const int bsk = n - k0 < kBB ? n - k0 : kBB;
        for (int e = tid; e < kBB * kBB; e += kBSThreads) {
            const int r = e / kBB, c = e % kBB;
            Lbb[r][c] = (r < bsb && c < r) ? Lg[pk(b0 + r, b0 + c)] : (r == c ? 1.0 : 0.0);
        }
        if (tid < kBB) db[tid] = tid < bsb ? Dg[b0 + tid] : 1.0;
        __syncthreads();
        // rows of tile I (threads 0..31, into Wi) and of tile K (threads 32..63,
        // K != I, into Lk): w_j = a_j - sum_{k<j} w_k L_jk, the row in
        // registers (every index known at compile time)
        if (tid < 2 * kBB) {
            const bool rowsI = tid < kBB;
            const int rr = tid & (kBB - 1);
            const int bsr = rowsI ? bsi : bsk, r0 = rowsI ? i0 : k0;
            if (rowsI || TK != TI) {
                const bool on = rr < bsr;
                const double *src = S + pk(on ? r0 + rr : r0, b0);
                double w[kBB];
#pragma unroll
                for (int j = 0; j < kBB; j++) w[j] = (on && j < bsb) ? src[j] : 0.0;
#pragma unroll
                for (int j = 1; j < kBB; j++) {
                    double v = w[j];
#pragma unroll
                    for (int k = 0; k < j; k++) v -= w[k] * Lbb[j][k];
                    w[j] = v;
                }
                double *dst = rowsI ? Wi[rr] : Lk[rr];
#pragma unroll
                for (int j = 0; j < kBB; j++) dst[j] = w[j];
            }
        }
        __syncthreads();
        // L_K = W_K D^-1 (the I rows themselves on a diagonal tile); the diagonal
        // tile writes L of tile I's rows in block column b
        for (int e = tid; e < kBB * kBB; e += kBSThreads) {
            const int rr = e / kBB, j = e % kBB;
            if (TK == TI) {
                const double l = Wi[rr][j] / db[j];
                Lk[rr][j] = l;
                if (rr < bsi && j < bsb) Lg[pk(i0 + rr, b0 + j)] = l;
            } else {
                Lk[rr][j] = Lk[rr][j] / db[j];
            }
        }
        __syncthreads();
        // S_IK -= W_I L_K^T: thread t takes row t / 8 and columns 4 (t % 8) .. + 3
        const bool next = TI == b + 1 && TK == b + 1;
        {
            const int r = tid >> 3, c0 = (tid & 7) * 4;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int j = 0; j < bsb; j++) {
                const double wv = Wi[r][j];
#pragma unroll
                for (int u = 0; u < 4; u++) acc[u] += wv * Lk[c0 + u][j];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int c = c0 + u;
                const bool in = r < bsi && c < bsk && (TI != TK || c <= r);
                double v = 0.0;
                if (in) {
                    v = S[pk(i0 + r, k0 + c)] - acc[u];
                    S[pk(i0 + r, k0 + c)] = v;
                }
                if (next) Tn[r][c] = v;
            }
        }
        if (next) {
            dg0 = i0;
            dgs = bsi;
        }
    }
    if (dg0 < 0) return;
    __syncthreads();
    if (tid < 64) border_diag_ldlt(Tn, dgs, dg0, Lg, Dg);
}

// Pivot signs and magnitudes of the whole factorisation (integer atomics only).
__global__ __launch_bounds__(64) void k_status_init(DevArgs a) {
    if (threadIdx.x == 0) {
        a.stat[0 * kStatStride] = 0;
        a.stat[1 * kStatStride] = 0;
        a.stat[2 * kStatStride] = 0;
        a.stat[3 * kStatStride] = INT64_MAX;
        a.stat[4 * kStatStride] = INT64_MAX;
        a.stat[5 * kStatStride] = 0;
        a.stat[6 * kStatStride] = 0;
        a.stat[7 * kStatStride] = 0;
    }
}

__device__ inline int pivot_code(double d, bool primal) {
    if (!isfinite(d)) return 3;                 // non-finite
    if (d == 0.0) return 2;                     // zero
    if ((d > 0.0) != primal) return 1;          // wrong sign
    return 0;
}

// Inertia and pivot report.  Each wavefront takes kStatusChunk consecutive
// pivots and their expected signs (coalesced reads, all in flight before
// any is used); the column of a pivot is formed only for a bad one.
constexpr int kStatusChunk = 1024;

__global__ __launch_bounds__(256) void k_status(DevArgs a) {
    int64_t np = 0, nn = 0, nz = 0, nf = 0, bad = INT64_MAX, mn = INT64_MAX, mx = 0;
    const int64_t total = a.dint + a.nbd_tot;
    const int64_t c0 = (int64_t(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6))) * kStatusChunk;
    const int lane = lane_id();
    // indices past the end re-read the last pivot and are not counted
    constexpr int kQ = kStatusChunk / 64;
    double dv[kQ];
    uint8_t pf[kQ];
#pragma unroll
    for (int k = 0; k < kQ; k++) {
        const int64_t idx = c0 + k * 64 + lane;
        const int64_t ic = idx < total ? idx : total - 1;
        dv[k] = a.dval[ic];
        pf[k] = a.bprim[ic];
    }
#pragma unroll
    for (int k = 0; k < kQ; k++) {
        const int64_t idx = c0 + k * 64 + lane;
        if (idx >= total) continue;
        const double d = dv[k];
        const int code = pivot_code(d, pf[k] != 0);
        if (code == 0 || code == 1) {
            if (d > 0) np++;
            else nn++;
        } else if (code == 2) nz++;
        else if (code == 3) nf++;
        if (code) {
            int64_t col;
            if (idx < a.dint) {
                const TemplDev &T = a.tmpls[find_tmpl(a, idx, &TemplDev::dbase)];
                const uint32_t off = uint32_t(idx - T.dbase), nb = uint32_t(T.nblk), j = off / nb;
                col = a.blks[T.blocks[off - j * nb]].col0 + j;
            } else {
                const int64_t j = idx - a.dint;
                const InstDev &I = a.insts[find_inst(a, j, &InstDev::bd0)];
                col = I.bstart + (j - I.bd0);
            }
            if (col * 8 + code < bad) bad = col * 8 + code;
        }
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
        nf += __shfl_xor(nf, o);
        const int64_t ob = __shfl_xor(bad, o), om = __shfl_xor(mn, o), ox = __shfl_xor(mx, o);
        bad = ob < bad ? ob : bad;
        mn = om < mn ? om : mn;
        mx = ox > mx ? ox : mx;
    }
    __shared__ int64_t red[7][4];
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) {
        red[0][wv] = np; red[1][wv] = nn; red[2][wv] = nz; red[3][wv] = bad; red[4][wv] = mn; red[5][wv] = mx;
        red[6][wv] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; q++) {
            red[0][0] += red[0][q];
            red[1][0] += red[1][q];
            red[2][0] += red[2][q];
            red[6][0] += red[6][q];
            red[3][0] = red[3][q] < red[3][0] ? red[3][q] : red[3][0];
            red[4][0] = red[4][q] < red[4][0] ? red[4][q] : red[4][0];
            red[5][0] = red[5][q] > red[5][0] ? red[5][q] : red[5][0];
        }
        unsigned long long *u = reinterpret_cast<unsigned long long *>(a.stat);
        if (red[0][0]) atomicAdd(u + 0 * kStatStride, (unsigned long long)red[0][0]);
        if (red[1][0]) atomicAdd(u + 1 * kStatStride, (unsigned long long)red[1][0]);
        if (red[2][0]) atomicAdd(u + 2 * kStatStride, (unsigned long long)red[2][0]);
        if (red[3][0] != INT64_MAX)
            atomicMin(reinterpret_cast<long long *>(a.stat + 3 * kStatStride), (long long)red[3][0]);
        if (red[4][0] != INT64_MAX)
            atomicMin(reinterpret_cast<long long *>(a.stat + 4 * kStatStride), (long long)red[4][0]);
        if (red[5][0]) atomicMax(reinterpret_cast<long long *>(a.stat + 5 * kStatStride), (long long)red[5][0]);
        if (red[6][0]) atomicAdd(u + 6 * kStatStride, (unsigned long long)red[6][0]);
    }
}

// Whether the last factorisation may be solved with: no zero or non-finite
// pivot and the inertia (n, m) (read from the status words k_status left).
__device__ inline bool factor_usable(const DevArgs &a) {
    return a.stat[2 * kStatStride] == 0 && a.stat[6 * kStatStride] == 0 && a.stat[0 * kStatStride] == a.nprimal;
}

// ------------------------------------------------------------------ solve

// Right-hand side into the solve vector and solution out of it: the
// caller's order (block by block, layout-local columns) and the factor's
// interleaved order are transposed through the LDS tiles of k_interleave,
// so that both the reads and the writes are coalesced.
// A factorisation that may not be solved with (see factor_usable) makes
// the solve write NaN: the caller who never read the status still sees it.
__global__ __launch_bounds__(256) void k_sol_load(DevArgs a, const double *__restrict__ b, double *__restrict__ y,
                                                  int64_t bld, int64_t ys, int check) {
    __shared__ double tile[kTileB][kTileJ + 1];
    b += blockIdx.y * bld;
    y += blockIdx.y * ys;
    const TileIx x = tile_index(a, blockIdx.x);
    const TemplDev &T = *x.T;
    const bool ok = !check || factor_usable(a);
    const int cj = threadIdx.x % kTileJ, rb = threadIdx.x / kTileJ;
    const int cb = threadIdx.x & 63, rj = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kTileR; q++) {
        const int bl = x.b0 + rb + kTileRows * q, j = x.j0 + cj;
        if (bl < T.nblk && j < T.n) tile[rb + kTileRows * q][cj] = b[a.blks[T.blocks[bl]].col0 + j];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTileR; q++) {
        const int j = x.j0 + rj + 4 * q, bl = x.b0 + cb;
        if (bl < T.nblk && j < T.n)
            y[T.dbase + int64_t(T.iperm[j]) * T.nblk + bl] = ok ? tile[cb][rj + 4 * q] : __builtin_nan("");
    }
}

// The same from a right-hand side already interleaved in layout order (the
// residual of a refinement step): a permutation inside each template, one
// element per thread, reads and writes along the blocks.
__global__ __launch_bounds__(256) void k_sol_load_int(DevArgs a, const double *__restrict__ r, double *__restrict__ y) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= a.dint) return;
    const TemplDev &T = a.tmpls[find_tmpl(a, idx, &TemplDev::dbase)];
    const int64_t off = idx - T.dbase;
    const int j = int(off / T.nblk), bl = int(off - int64_t(j) * T.nblk);
    y[T.dbase + int64_t(T.iperm[j]) * T.nblk + bl] = factor_usable(a) ? r[idx] : __builtin_nan("");
}

template <bool kAdd>
__global__ __launch_bounds__(256) void k_sol_store(DevArgs a, const double *__restrict__ y, double *__restrict__ xo,
                                                   int64_t ys, int64_t bld) {
    __shared__ double tile[kTileB][kTileJ + 1];
    y += blockIdx.y * ys;
    xo += blockIdx.y * bld;
    const TileIx x = tile_index(a, blockIdx.x);
    const TemplDev &T = *x.T;
    const bool ok = factor_usable(a);
    const int cj = threadIdx.x % kTileJ, rb = threadIdx.x / kTileJ;
    const int cb = threadIdx.x & 63, rj = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kTileR; q++) {
        const int j = x.j0 + rj + 4 * q, bl = x.b0 + cb;
        if (bl < T.nblk && j < T.n) tile[cb][rj + 4 * q] = y[T.dbase + int64_t(T.iperm[j]) * T.nblk + bl];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTileR; q++) {
        const int bl = x.b0 + rb + kTileRows * q, j = x.j0 + cj;
        if (bl < T.nblk && j < T.n) {
            const int64_t c = a.blks[T.blocks[bl]].col0 + j;
            const double v = ok ? tile[rb + kTileRows * q][cj] : __builtin_nan("");
            xo[c] = kAdd ? xo[c] + v : v;
        }
    }
}

// Solves.  Forward (L y = b, levels upwards): per level, every diagonal
// row gathers the products of its descendants' columns (pull), then the
// wide supernodes' unit lower diagonal blocks are solved.  Backward: one
// launch takes every column's border rows and D^-1, then one launch per
// level (downwards) takes each supernode's block rows and its diagonal
// block (see k_sol_bwd_border and k_sol_bwd below).

// forward gather of a diagonal row: y_row -= sum over descendants L_d[row,:] y_d
// (the terms of the row's diagonal panel entry)
template <int NW>
__global__ __launch_bounds__(kWG) void k_sol_fwd_gather(DevArgs a, double *y, const Work *__restrict__ wl, int nw,
                                                        int64_t ys) {
    y += blockIdx.y * ys;
    const int task = split_task<NW>();
    if (task >= nw) return;
    const Lane W = lane_work(a, wl, task);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    double *yb = y + T.dbase + W.bl;
    const int s = cs(T.task_s)[W.k], p = cs(T.task_p)[W.k];
    const int col = cs(T.sup_first)[s] + p;
    const int e = cs(T.task_cbase)[W.k] + p;
    const int t0 = cs(T.ent_tptr)[e], t1 = cs(T.ent_tptr)[e + 1];
    const double *Lb = a.lpan + T.lbase, *y0 = y + T.dbase;
    const uint32_t nbu = uint32_t(nb), blu = uint32_t(W.bl);
    double v = split_sum<NW>([&](int q) { return ydot_q(Lb, y0, nbu, blu, T.terms, t0, t1, q); });
    if (!split_combine<NW>(v)) return;
    if (W.on) yb[int64_t(col) * nb] -= v;
}

// unit lower triangular solve with a wide supernode's diagonal block,
// right-looking: y_k -= L(k,j) y_j for k > j (the loads of L do not depend
// on y)
__global__ __launch_bounds__(kWG) void k_sol_fwd_diag(DevArgs a, double *y, const Work *__restrict__ wl, int nw,
                                                      int64_t ys) {
    y += blockIdx.y * ys;
    const int wid = wave_id();
    if (wid >= nw) return;
    const Lane W = lane_work(a, wl, wid);
    const TemplDev &T = *W.T;
    const int64_t nb = W.nb;
    const int s = W.k;
    const int f = cs(T.sup_first)[s], w = cs(T.sup_first)[s + 1] - f;
    const int r = cs(T.sup_rowptr)[s + 1] - cs(T.sup_rowptr)[s];
    const double *P = a.lpan + T.lbase + W.bl + int64_t(cs(T.panel_off)[s]) * nb;
    double *yb = y + T.dbase + W.bl + int64_t(f) * nb;
    by_width(w, [&](auto Wc) {
        constexpr int W_ = decltype(Wc)::value;
        const int wl1 = w - 1;
        double x[W_];
#pragma unroll
        for (int j = 0; j < W_; j++) x[j] = yb[int64_t(j < w ? j : wl1) * nb];
        // row by row: x_k -= L(k,j) x_j for j < k, in increasing j (the
        // order of the column sweep, so the same bits)
#pragma unroll
        for (int k = 1; k < W_; k++) {
            const int kc = k < w ? k : wl1;
#pragma unroll
            for (int j = 0; j < k; j++) {
                const double l = P[(int64_t(j < w ? j : wl1) * r + kc) * nb];
                x[k] -= (k < w ? l : 0.0) * x[j];
            }
        }
        if (W.on) {
#pragma unroll
            for (int j = 1; j < W_; j++)
                if (j < w) yb[int64_t(j) * nb] = x[j];
        }
    });
}

struct SolTask {
    const TemplDev *T;
    int s, f, w, r, rnb;     // rows: 0 .. w-1 diagonal block, w .. rnb-1 block rows, rnb .. r-1 border rows
    uint32_t nb, bl, po;
    bool on;
};

__device__ __attribute__((always_inline)) inline SolTask sol_task(const DevArgs &a, const Work *wl, int item) {
    const Lane W = lane_work(a, wl, item);
    SolTask t;
    t.T = W.T;
    t.s = W.k & ~kWideFlag;
    t.f = cs(W.T->sup_first)[t.s];
    t.w = cs(W.T->sup_first)[t.s + 1] - t.f;
    t.r = cs(W.T->sup_rowptr)[t.s + 1] - cs(W.T->sup_rowptr)[t.s];
    t.rnb = cs(W.T->sup_rnb)[t.s];
    t.nb = uint32_t(W.nb);
    t.bl = uint32_t(W.bl);
    t.po = uint32_t(cs(W.T->panel_off)[t.s]);
    t.on = W.on;
    return t;
}

// Work of a level launch: narrow items first (one wavefront each, four to a
// workgroup), then wide ones (a workgroup each).  Returns false for a
// wavefront with nothing to do.
__device__ __attribute__((always_inline)) inline bool sol_item(int nw, int nnar, int &item, int &q, int &nwv) {
    const int g = xcd_workgroup(), wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int ngn = (nnar + 3) >> 2;
    if (g < ngn) {
        item = 4 * g + wv;
        q = 0;
        nwv = 1;
        return item < nnar;
    }
    item = nnar + (g - ngn);
    q = wv;
    nwv = 4;
    return item < nw;
}

// this block's part of the border right-hand side: cpart[b][block] = L_bk y_k
template <int NW>
__global__ __launch_bounds__(kWG) void k_sol_bpart(DevArgs a, const double *y, double *cpart,
                                                   const Work *__restrict__ wl, int nw, int64_t ys, int64_t cps) {
    y += blockIdx.y * ys;
    cpart += blockIdx.y * cps;
    const int task = split_task<NW>();
    if (task >= nw) return;
    const Lane W = lane_work(a, wl, task);
    const TemplDev &T = *W.T;
    const int bi = W.k;
    const int t0 = cs(T.bterm_ptr)[bi], t1 = cs(T.bterm_ptr)[bi + 1];
    const double *Lb = a.lpan + T.lbase, *y0 = y + T.dbase;
    const uint32_t nbu = uint32_t(W.nb), blu = uint32_t(W.bl);
    double v = split_sum<NW>([&](int q) { return ydot_q(Lb, y0, nbu, blu, T.bterms, t0, t1, q); });
    if (!split_combine<NW>(v)) return;
    const InstDev &I = a.insts[T.inst];
    if (W.on) cpart[I.cp0 + int64_t(bi) * I.nblk + (T.blocks[W.bl] - I.blk0)] = v;
}

// border: c = b_b - sum_k cpart; forward with L_bb, D_b^{-1}, backward with
// L_bb^T.  The block sum runs one wavefront per border row (lane-strided
// partial sums, then a fixed shuffle tree).  The substitutions are blocked
// by kBB rows: wavefront 0 solves a diagonal block with cross-lane shuffles
// (lane = row, its kBB factor entries preloaded into registers), then the
// workgroup updates the remaining rows.
// Value of v in lane k (k uniform), through two scalar lane reads.
__device__ inline double lane_bcast(double v, int k) {
    const int64_t b = __double_as_longlong(v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(b), k));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(b >> 32), k));
    return __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

// kRes: the packed factor is first copied into LDS (one coalesced sweep), so
// that the substitutions wait on LDS rather than on global memory; taken by
// each instance whose factor fits the LDS the launch provides.
template <bool kRes>
__device__ inline void sol_border(const DevArgs &a, const InstDev &I, double *c, double *x, double *y, bool add) {
    const int nbd = I.nbd, tid = threadIdx.x, lane = lane_id();
    const double *Db = a.dval + a.dint + I.bd0;
    const double *Lg = a.lbb + I.sbb0;
    double *Ll = c + a.max_nbd;
    if (kRes) {
        const int npk = nbd * (nbd + 1) / 2;
#pragma unroll 8
        for (int e = tid; e < npk; e += kBorderThreads) Ll[e] = Lg[e];
    }
    const double *Lb = kRes ? Ll : Lg;
    // the border right-hand side (k_sol_bsum left it in y's border part)
    for (int i = tid; i < nbd; i += kBorderThreads) c[i] = y[a.dint + I.bd0 + i];
    __syncthreads();
    // forward: L y = c
    for (int b0 = 0; b0 < nbd; b0 += kBB) {
        const int bs = nbd - b0 < kBB ? nbd - b0 : kBB;
        if (tid < 64) {
            const int i = b0 + lane;
            double l[kBB];
#pragma unroll
            for (int k = 0; k < kBB; k++) l[k] = (lane < bs && k < lane) ? Lb[pk(i, b0 + k)] : 0.0;
            double ci = lane < bs ? c[i] : 0.0;
#pragma unroll
            for (int k = 0; k < kBB - 1; k++) {
                const double xk = lane_bcast(ci, k);
                ci -= l[k] * xk;
            }
            if (lane < bs) c[i] = ci;
        }
        __syncthreads();
        for (int i = b0 + bs + tid; i < nbd; i += kBorderThreads) {
            const double *li = Lb + pk(i, b0);
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
            for (int k = 0; k < kBB; k += 4) {
                if (k < bs) s0 += li[k] * c[b0 + k];
                if (k + 1 < bs) s1 += li[k + 1] * c[b0 + k + 1];
                if (k + 2 < bs) s2 += li[k + 2] * c[b0 + k + 2];
                if (k + 3 < bs) s3 += li[k + 3] * c[b0 + k + 3];
            }
            c[i] -= (s0 + s1) + (s2 + s3);
        }
        __syncthreads();
    }
    for (int i = tid; i < nbd; i += kBorderThreads) c[i] /= Db[i];
    __syncthreads();
    // backward: L^T x = y, last block first
    for (int b0 = ((nbd - 1) / kBB) * kBB; b0 >= 0; b0 -= kBB) {
        const int bs = nbd - b0 < kBB ? nbd - b0 : kBB;
        if (tid < 64) {
            double l[kBB];
#pragma unroll
            for (int i = 0; i < kBB; i++) l[i] = (i < bs && lane < i) ? Lb[pk(b0 + i, b0 + lane)] : 0.0;
            double cj = lane < bs ? c[b0 + lane] : 0.0;
#pragma unroll
            for (int i = kBB - 1; i > 0; i--) {
                const double xi = lane_bcast(cj, i);
                cj -= l[i] * xi;
            }
            if (lane < bs) c[b0 + lane] = cj;
        }
        __syncthreads();
        for (int j = tid; j < b0; j += kBorderThreads) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
            for (int k = 0; k < kBB; k += 4) {
                if (k < bs) s0 += Lb[pk(b0 + k, j)] * c[b0 + k];
                if (k + 1 < bs) s1 += Lb[pk(b0 + k + 1, j)] * c[b0 + k + 1];
                if (k + 2 < bs) s2 += Lb[pk(b0 + k + 2, j)] * c[b0 + k + 2];
                if (k + 3 < bs) s3 += Lb[pk(b0 + k + 3, j)] * c[b0 + k + 3];
            }
            c[j] -= (s0 + s1) + (s2 + s3);
        }
        __syncthreads();
    }
    const bool ok = factor_usable(a);
    for (int i = tid; i < nbd; i += kBorderThreads) {
        const double v = ok ? c[i] : __builtin_nan("");
        y[a.dint + I.bd0 + i] = v;
        x[I.bstart + i] = add ? x[I.bstart + i] + v : v;
    }
}

// The border right-hand side c_i = b_i - (sum over the blocks of the
// partials k_sol_bpart left), one wavefront per border row of every
// instance: lane-strided in two partials (blocks lane, lane + 128, ... and
// lane + 64, lane + 192, ...), then a fixed shuffle tree; into y's border
// part, which the border solve reads.
__global__ __launch_bounds__(256) void k_sol_bsum(DevArgs a, const double *__restrict__ b, double *y,
                                                  const double *__restrict__ cpart, int64_t bld, int64_t ys,
                                                  int64_t cps) {
    const int64_t q = int64_t(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    if (q >= a.nbd_tot) return;
    b += blockIdx.y * bld;
    y += blockIdx.y * ys;
    cpart += blockIdx.y * cps;
    const InstDev &I = a.insts[find_inst(a, q, &InstDev::bd0)];
    const int i = int(q - I.bd0), nblk = I.nblk, lane = lane_id();
    const double *ci = cpart + I.cp0 + int64_t(i) * nblk;
    double s0 = 0.0, s1 = 0.0;
    for (int k = lane; k < nblk; k += 128) {
        s0 += ci[k];
        if (k + 64 < nblk) s1 += ci[k + 64];
    }
    double v = s0 + s1;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) y[a.dint + I.bd0 + i] = b[I.bstart + i] - v;
}

__global__ __launch_bounds__(kBorderThreads) void k_sol_border(DevArgs a, double *x, double *y, int64_t lds_bytes,
                                                               int add, int64_t bld, int64_t ys) {
    extern __shared__ double c[];
    x += blockIdx.y * bld;
    y += blockIdx.y * ys;
    const InstDev &I = a.insts[blockIdx.x];
    const int64_t need = (int64_t(a.max_nbd) + int64_t(I.nbd) * (I.nbd + 1) / 2) * int64_t(sizeof(double));
    if (need <= lds_bytes) sol_border<true>(a, I, c, x, y, add != 0);
    else sol_border<false>(a, I, c, x, y, add != 0);
}

// Backward (D L^T x = y).  One launch over every block column first takes
// the border rows (k_sol_bwd_border below), the border solution being
// final.  Then the levels
// downwards: v_p = sum over the block rows i below the diagonal block of
// L(i, p) x_row(i) (ancestors, final), x_p = y_p - v_p, and the transposed
// unit diagonal block, right-looking from the last column.  Both sums run
// over a row range [i0, i1) as four partials (partial k takes rows i0 + k,
// i0 + k + 4, ... in order, one accumulator per column), combined
// (v0 + v1) + (v2 + v3).  A narrow task's wavefront computes all four
// partials, a wide task's wavefront k partial k (exchanged through local
// memory, 3 * w * 64 doubles); only wavefront 0 of a wide task returns true.
template <int W_, int NP>
__device__ __attribute__((always_inline)) inline bool bwd_rowsum(const DevArgs &a, const SolTask &t, const double *y,
                                                                  int q, int i0, int i1, double *red, double v[W_]) {
    const TemplDev &T = *t.T;
    const double *Lb = a.lpan + T.lbase;
    const double *y0 = y + T.dbase;
    const double *xb = y + a.dint + T.bd0;
    const int n = T.n, w = t.w;
    const uint32_t nb = t.nb, bl = t.bl, po = t.po, ur = uint32_t(t.r);
    const int32_t *__restrict__ R_ = T.sup_rows + cs(T.sup_rowptr)[t.s];
    auto at = [&](int col, int row) { return (po + uint32_t(col) * ur + uint32_t(row)) * nb + bl; };
    double acc[NP][W_];
#pragma unroll
    for (int k = 0; k < NP; k++)
#pragma unroll
        for (int p = 0; p < W_; p++) acc[k][p] = 0.0;
    // rows in groups of four (one per partial); a pass loads KP rows of a
    // group (all four partials: KP = 2 or 4 by width) or G_ groups' row of
    // the wavefront's own partial, so that about 16 loads are in flight
    constexpr int KP = NP == 4 ? (W_ >= 8 ? 2 : 4) : 1;
    constexpr int G_ = NP == 4 ? 1 : (W_ <= 4 ? 4 : (W_ <= 8 ? 2 : 1));
    const int k0 = NP == 4 ? 0 : q;
    for (int g0 = i0; g0 < i1; g0 += 4 * G_) {
#pragma unroll
        for (int kh = 0; kh < NP; kh += KP) {
            double xv[G_][KP], l[G_][KP][W_];
#pragma unroll
            for (int gg = 0; gg < G_; gg++)
#pragma unroll
                for (int k = 0; k < KP; k++) {
                    const int i = g0 + 4 * gg + k0 + kh + k, ic = i < i1 ? i : i1 - 1;
                    const int ri = cs(R_)[ic];
                    xv[gg][k] = ri < n ? ld32(y0, uint32_t(ri) * nb + bl) : xb[ri - n];
#pragma unroll
                    for (int p = 0; p < W_; p++) l[gg][k][p] = p < w ? ld32(Lb, at(p, ic)) : 0.0;
                }
#pragma unroll
            for (int gg = 0; gg < G_; gg++)
#pragma unroll
                for (int k = 0; k < KP; k++) {
                    if (g0 + 4 * gg + k0 + kh + k >= i1) continue;
#pragma unroll
                    for (int p = 0; p < W_; p++)
                        if (p < w) acc[kh + k][p] = fma(l[gg][k][p], xv[gg][k], acc[kh + k][p]);
                }
        }
    }
    if constexpr (NP == 4) {
#pragma unroll
        for (int p = 0; p < W_; p++) v[p] = (acc[0][p] + acc[1][p]) + (acc[2][p] + acc[3][p]);
        return true;
    } else {
        const int lane = lane_id();
        if (q > 0) {
#pragma unroll
            for (int p = 0; p < W_; p++)
                if (p < w) red[((q - 1) * w + p) * 64 + lane] = acc[0][p];
        }
        __syncthreads();
        if (q > 0) return false;
#pragma unroll
        for (int p = 0; p < W_; p++)
            v[p] = p < w ? (acc[0][p] + red[p * 64 + lane]) + (red[(w + p) * 64 + lane] + red[(2 * w + p) * 64 + lane])
                         : 0.0;
        return true;
    }
}

template <int W_, int NP>
__device__ __attribute__((always_inline)) inline void sol_bwd_task(const DevArgs &a, const SolTask &t, double *y, int q,
                                                                    double *red) {
    double v[W_];
    if (!bwd_rowsum<W_, NP>(a, t, y, q, t.w, t.rnb, red, v)) return;
    const TemplDev &T = *t.T;
    const double *Lb = a.lpan + T.lbase;
    double *y0 = y + T.dbase;
    const int w = t.w, wl1 = w - 1;
    const uint32_t nb = t.nb, bl = t.bl, po = t.po, ur = uint32_t(t.r);
    auto at = [&](int col, int row) { return (po + uint32_t(col) * ur + uint32_t(row)) * nb + bl; };
    double x[W_];
#pragma unroll
    for (int j = 0; j < W_; j++) x[j] = ld32(y0, uint32_t(t.f + (j < w ? j : wl1)) * nb + bl) - v[j];
#pragma unroll
    for (int j = W_ - 1; j > 0; j--) {
        const int jc = j < w ? j : wl1;
#pragma unroll
        for (int k = 0; k < j; k++) {
            const double l = ld32(Lb, at(k < w ? k : wl1, jc));
            x[k] = fma(-(j < w ? l : 0.0), x[j], x[k]);
        }
    }
    if (t.on) {
#pragma unroll
        for (int j = 0; j < W_; j++)
            if (j < w) st32(y0, uint32_t(t.f + j) * nb + bl, x[j]);
    }
}

// Border step of the backward pass, one task per block column j (of a group
// of 64 blocks): y_j <- y_j / d_j - t_j, t_j = sum over the border rows b of
// j's panel column of L(b, j) x_b, as four partials over those rows (partial
// k takes rows k, k + 4, ... in order) combined (t0 + t1) + (t2 + t3).  The
// rows of one panel column are contiguous.  A narrow task's wavefront
// computes all four partials; a wide task (long border column) is a
// workgroup whose wavefront k computes partial k.
template <int NP>
__device__ __attribute__((always_inline)) inline void bwd_col_partials(const DevArgs &a, const TemplDev &T, const double *y,
                                                                        int s, int p, uint32_t nb, uint32_t bl, int k0,
                                                                        double acc[NP]) {
    const int r = cs(T.sup_rowptr)[s + 1] - cs(T.sup_rowptr)[s], rnb = cs(T.sup_rnb)[s];
    const int32_t *__restrict__ R_ = T.sup_rows + cs(T.sup_rowptr)[s];
    const double *Lc = a.lpan + T.lbase;
    const uint32_t c0 = uint32_t(cs(T.panel_off)[s] + p * r);
    const double *xb = y + a.dint + T.bd0;
    const int n = T.n;
#pragma unroll
    for (int k = 0; k < NP; k++) acc[k] = 0.0;
    constexpr int G_ = NP == 4 ? 2 : 8;          // row groups of four per pass (8 rows in flight)
    for (int g0 = rnb; g0 < r; g0 += 4 * G_) {
        double l[G_][NP], xv[G_][NP];
#pragma unroll
        for (int gg = 0; gg < G_; gg++)
#pragma unroll
            for (int k = 0; k < NP; k++) {
                const int i = g0 + 4 * gg + k0 + k, ic = i < r ? i : r - 1;
                l[gg][k] = ld32(Lc, (c0 + uint32_t(ic)) * nb + bl);
                xv[gg][k] = xb[cs(R_)[ic] - n];
            }
#pragma unroll
        for (int gg = 0; gg < G_; gg++)
#pragma unroll
            for (int k = 0; k < NP; k++)
                if (g0 + 4 * gg + k0 + k < r) acc[k] = fma(l[gg][k], xv[gg][k], acc[k]);
    }
}

__global__ __launch_bounds__(kWG) void k_sol_bwd_border(DevArgs a, double *y, const Work *__restrict__ wl, int nw,
                                                        int nnar, int64_t ys) {
    __shared__ double red[3][64];
    y += blockIdx.y * ys;
    int item, q, nwv;
    if (!sol_item(nw, nnar, item, q, nwv)) return;
    const Lane W = lane_work(a, wl, item);
    const TemplDev &T = *W.T;
    const int j = W.k & ~kWideFlag;
    const int s = cs(T.col_sup)[j], p = j - cs(T.sup_first)[s];
    const uint32_t nb = uint32_t(W.nb), bl = uint32_t(W.bl);
    double v;
    if (nwv == 1) {
        double acc[4];
        bwd_col_partials<4>(a, T, y, s, p, nb, bl, 0, acc);
        v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    } else {
        double acc[1];
        bwd_col_partials<1>(a, T, y, s, p, nb, bl, q, acc);
        const int lane = lane_id();
        if (q > 0) red[q - 1][lane] = acc[0];
        __syncthreads();
        if (q > 0) return;
        v = (acc[0] + red[0][lane]) + (red[1][lane] + red[2][lane]);
    }
    if (!W.on) return;
    double *y0 = y + T.dbase;
    const double *d0 = a.dval + T.dbase;
    const uint32_t c = uint32_t(j) * nb + bl;
    st32(y0, c, ld32(y0, c) / ld32(d0, c) - v);
}

template <int WMAX>
__global__ __launch_bounds__(kWG, WMAX <= 8 ? 4 : 2) void k_sol_bwd(DevArgs a, double *y, const Work *__restrict__ wl,
                                                                    int nw, int nnar, int64_t ys) {
    extern __shared__ double red[];
    y += blockIdx.y * ys;
    int item, q, nwv;
    if (!sol_item(nw, nnar, item, q, nwv)) return;
    const SolTask t = sol_task(a, wl, item);
    if (nwv == 1) {
        by_width_max<kNarrowW>(t.w, [&](auto Wc) { sol_bwd_task<decltype(Wc)::value, 4>(a, t, y, q, red); });
    } else {
        by_width_max<WMAX>(t.w, [&](auto Wc) { sol_bwd_task<decltype(Wc)::value, 1>(a, t, y, q, red); });
    }
}

// ------------------------------------------------------------------ backward error

// Residual r = b - K x of one column and the quantities of its backward
// errors: |r_i|, |r_i| / (|K||x| + |b|)_i, the row norm sum_j |K_ij|, |x_i|
// and |b_i|.  Each workgroup leaves their maxima (non-negative, so order
// does not matter; a NaN propagates) in epart[8 * workgroup + q]; the final
// kernel reduces them.  x and b come interleaved (k_interleave into xint,
// bint); r goes to rint (blocks) and rbuf (border, layout order), where a
// refinement step's solve picks it up.
enum { BE_R, BE_Q, BE_ROWN, BE_X, BE_B, BE_N };
constexpr int kFinalThreads = 1024;

__device__ inline double nanmax(double p, double q) { return (p > q || p != p) ? p : q; }

__device__ inline void berr_commit(const DevArgs &a, int64_t slot, double v[BE_N]) {
#pragma unroll
    for (int q = 0; q < BE_N; q++)
        for (int o = 32; o > 0; o >>= 1) v[q] = nanmax(v[q], __shfl_xor(v[q], o));
    __shared__ double red[4][BE_N];
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0)
        for (int q = 0; q < BE_N; q++) red[wv][q] = v[q];
    __syncthreads();
    if (threadIdx.x < BE_N) {
        const int q = threadIdx.x;
        a.epart[8 * slot + q] = nanmax(nanmax(red[0][q], red[1][q]), nanmax(red[2][q], red[3][q]));
    }
}

__device__ inline double ratio(double r, double den) { return den > 0.0 ? r / den : (r > 0.0 ? INFINITY : r); }

// one wavefront per (template row, group of 64 blocks), lane = block
__global__ __launch_bounds__(256) void k_berr_rows(DevArgs a) {
    const int64_t w = int64_t(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    double v[BE_N] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (w < a.rows_waves) {
        const TemplDev &T = a.tmpls[find_tmpl(a, w, &TemplDev::rwbase)];
        const int ngr = (T.nblk + 63) >> 6;
        const int64_t wl = w - T.rwbase;
        const int j = int(wl / ngr), g = int(wl - int64_t(j) * ngr);
        const int b = g * 64 + lane_id();
        const bool on = b < T.nblk;
        const uint32_t bl = on ? uint32_t(b) : 0u, nb = uint32_t(T.nblk);
        const double *xb = a.xint + T.dbase, *Kb = a.kval + T.kbase;
        const double *xbd = a.xint + a.dint + T.bd0;
        const int n = T.n;
        double s0 = 0.0, s1 = 0.0, d0 = 0.0, d1 = 0.0, rn = 0.0;
        const int e1 = cs(T.rr_ptr)[j + 1];
        int e = cs(T.rr_ptr)[j];
        for (; e + 2 <= e1; e += 2) {
            const int k0 = cs(T.rr_ent)[2 * e], c0 = cs(T.rr_ent)[2 * e + 1];
            const int k1 = cs(T.rr_ent)[2 * e + 2], c1 = cs(T.rr_ent)[2 * e + 3];
            const double v0 = ld32(Kb, uint32_t(k0) * nb + bl), v1 = ld32(Kb, uint32_t(k1) * nb + bl);
            const double x0 = c0 < n ? ld32(xb, uint32_t(c0) * nb + bl) : xbd[c0 - n];
            const double x1 = c1 < n ? ld32(xb, uint32_t(c1) * nb + bl) : xbd[c1 - n];
            s0 += v0 * x0;
            s1 += v1 * x1;
            d0 += fabs(v0) * fabs(x0);
            d1 += fabs(v1) * fabs(x1);
            rn += fabs(v0) + fabs(v1);
        }
        if (e < e1) {
            const int k0 = cs(T.rr_ent)[2 * e], c0 = cs(T.rr_ent)[2 * e + 1];
            const double v0 = ld32(Kb, uint32_t(k0) * nb + bl);
            const double x0 = c0 < n ? ld32(xb, uint32_t(c0) * nb + bl) : xbd[c0 - n];
            s0 += v0 * x0;
            d0 += fabs(v0) * fabs(x0);
            rn += fabs(v0);
        }
        const uint32_t o = uint32_t(j) * nb + bl;
        const double bv = ld32(a.bint + T.dbase, o), xj = ld32(xb, o);
        const double r = bv - (s0 + s1);
        if (on) {
            st32(a.rint + T.dbase, o, r);
            v[BE_R] = fabs(r);
            v[BE_Q] = ratio(fabs(r), (d0 + d1) + fabs(bv));
            v[BE_ROWN] = rn;
            v[BE_X] = fabs(xj);
            v[BE_B] = fabs(bv);
        }
    }
    berr_commit(a, blockIdx.x, v);
}

// one wavefront per border row of every instance: the blocks' entries of
// the row (lane = block, templates and groups in order), then K_bb's (lanes
// strided), summed by a fixed shuffle tree
__global__ __launch_bounds__(256) void k_berr_border(DevArgs a) {
    const int64_t q = int64_t(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    double v[BE_N] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (q < a.nbd_tot) {
        const InstDev &I = a.insts[find_inst(a, q, &InstDev::bd0)];
        const int bi = int(q - I.bd0), lane = lane_id();
        double s = 0.0, den = 0.0, rn = 0.0;
        for (int ti = I.t0; ti < I.t0 + I.nt; ti++) {
            const TemplDev &T = a.tmpls[ti];
            const int e0 = cs(T.rb_ptr)[bi], e1 = cs(T.rb_ptr)[bi + 1];
            for (int g0 = 0; g0 < T.nblk; g0 += 64) {
                const int b = g0 + lane;
                if (b >= T.nblk) continue;
                for (int e = e0; e < e1; e++) {
                    const int kp = cs(T.rb_ent)[2 * e], c = cs(T.rb_ent)[2 * e + 1];
                    const double kv = a.kval[T.kbase + int64_t(kp) * T.nblk + b];
                    const double xv = a.xint[T.dbase + int64_t(c) * T.nblk + b];
                    s += kv * xv;
                    den += fabs(kv) * fabs(xv);
                    rn += fabs(kv);
                }
            }
        }
        const double *xbd = a.xint + a.dint + I.bd0;
        for (int e = I.kbr_ptr[bi] + lane; e < I.kbr_ptr[bi + 1]; e += 64) {
            const double kv = a.kval[a.kint + I.kbb0 + I.kbr_ent[2 * e]];
            const double xv = xbd[I.kbr_ent[2 * e + 1]];
            s += kv * xv;
            den += fabs(kv) * fabs(xv);
            rn += fabs(kv);
        }
        for (int o = 32; o > 0; o >>= 1) {
            s += __shfl_xor(s, o);
            den += __shfl_xor(den, o);
            rn += __shfl_xor(rn, o);
        }
        const double bv = a.bint[a.dint + I.bd0 + bi], xv = xbd[bi];
        const double r = bv - s;
        if (lane == 0) a.rbuf[I.bstart + bi] = r;
        v[BE_R] = fabs(r);
        v[BE_Q] = ratio(fabs(r), den + fabs(bv));
        v[BE_ROWN] = rn;
        v[BE_X] = fabs(xv);
        v[BE_B] = fabs(bv);
    }
    berr_commit(a, a.rows_wg + blockIdx.x, v);
}

// eta = max|r| / (max_i sum_j |K_ij| * max|x| + max|b|), omega = max ratio
__global__ __launch_bounds__(kFinalThreads) void k_berr_final(DevArgs a, double *out) {
    const int np = a.rows_wg + int((a.nbd_tot + 3) / 4);
    double v[BE_N] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < np; i += kFinalThreads)
#pragma unroll
        for (int q = 0; q < BE_N; q++) v[q] = nanmax(v[q], a.epart[8 * int64_t(i) + q]);
#pragma unroll
    for (int q = 0; q < BE_N; q++)
        for (int o = 32; o > 0; o >>= 1) v[q] = nanmax(v[q], __shfl_xor(v[q], o));
    __shared__ double red[kFinalThreads / 64][BE_N];
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0)
        for (int q = 0; q < BE_N; q++) red[wv][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kFinalThreads / 64; w++)
            for (int q = 0; q < BE_N; q++) red[0][q] = nanmax(red[0][q], red[w][q]);
        const double den = red[0][BE_ROWN] * red[0][BE_X] + red[0][BE_B];
        out[0] = ratio(red[0][BE_R], den);
        out[1] = red[0][BE_Q];
    }
}

// ------------------------------------------------------------------ dispatch map

// Flow leaving end s of a branch (value and gradient in v_s, v_o, th_s, th_o).
struct Flow {
    double P, Q, gP[4], gQ[4];
};

__device__ inline void branch_flow(double g, double b, double vs, double vo, double ts, double to, Flow &e) {
    double sn, cs;
    sincos(ts - to, &sn, &cs);
    const double A = g * cs + b * sn, Bq = g * sn - b * cs, vv = vs * vo;
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
}

// F(z; pd) and the barrier / dual diagonal sigma of the NCL subproblem
// without PV/PQ rows.  Threads as in the assembly: per template (bus,
// block) then (generator, block), then the border pg of every instance.
// Every position of F and sigma is written by exactly one thread: a bus
// thread writes its vm, va, P and Q rows and, for branches it is the from
// end of, both flow rows; a generator thread its qg (and a single-block
// network's pg); a border thread the shared pg, summing its balance-row
// multipliers over the instance's blocks in block order.
__global__ __launch_bounds__(256) void k_residual(DevArgs a, const double *__restrict__ z, ncl_nlp q,
                                                  double *__restrict__ F, double *__restrict__ sg, double rho) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const double irho = 1.0 / rho, mu = q.mu;
    if (tid >= a.asm_threads) {
        const int64_t gg = tid - a.asm_threads;
        if (gg >= a.gp_tot) return;
        const InstDev &I = a.insts[find_inst(a, gg, &InstDev::gp0)];
        const int g = int(gg - I.gp0);
        if (I.nbd == 0 || g >= I.ng) return;
        const int64_t col = I.bstart + I.border_pg[g];
        double ysum = 0.0;
        for (int blk = I.blk0; blk < I.blk0 + I.nblk; blk++) {
            const BlockDev &B = a.blks[blk];
            const TemplDev &T = a.tmpls[B.tmpl];
            const int bus = T.gen_idx[size_t(g) * GI_N + GI_BUS];
            ysum += z[zi(I.bstart, B, T.n, T.bus_idx[size_t(bus) * BI_N + BI_P])];
        }
        const double pg = z[col], lo = pg, hi = q.pmax - pg;
        F[col] = 2.0 * I.gen_c2[g] * pg - ysum - mu / lo + mu / hi;
        sg[col] = mu / (lo * lo) + mu / (hi * hi);
        return;
    }
    const TemplDev &T = a.tmpls[find_tmpl(a, tid, &TemplDev::abase)];
    const int64_t u0 = tid - T.abase;
    const int64_t nbus_t = int64_t(T.nblk) * T.nbus;
    const int64_t bstart = a.insts[T.inst].bstart;
    const int n = T.n;
    if (u0 < nbus_t) {
        const int bl = int(u0 % T.nblk), i = int(u0 / T.nblk);
        const BlockDev B = a.blks[T.blocks[bl]];
        const int32_t *bi = T.bus_idx + size_t(i) * BI_N;
        const double vi = z[zi(bstart, B, n, bi[BI_VM])], ti = z[zi(bstart, B, n, bi[BI_VA])];
        const double yPi = z[zi(bstart, B, n, bi[BI_P])], yQi = z[zi(bstart, B, n, bi[BI_Q])];
        double Pinj = 0.0, Qinj = 0.0, Fv = 0.0, Fa = 0.0;
        for (int qa = T.bus_adj_ptr[i]; qa < T.bus_adj_ptr[i + 1]; qa++) {
            const int32_t e = T.bus_adj[qa];
            const bool self_from = e >= 0;
            const int l = self_from ? e : ~e;
            const int32_t *br = T.br_idx + size_t(l) * 4;
            const int o = self_from ? br[3] : br[2];
            const int32_t *bo = T.bus_idx + size_t(o) * BI_N;
            const double vo = z[zi(bstart, B, n, bo[BI_VM])], to = z[zi(bstart, B, n, bo[BI_VA])];
            const double yPo = z[zi(bstart, B, n, bo[BI_P])], yQo = z[zi(bstart, B, n, bo[BI_Q])];
            const int64_t rs = zi(bstart, B, n, self_from ? br[0] : br[1]);   // flow row of the end at i
            const int64_t ro = zi(bstart, B, n, self_from ? br[1] : br[0]);   // flow row of the other end
            const double yFs = z[rs], yFo = z[ro];
            const double st = (l == B.outage) ? 0.0 : 1.0;
            const double r = T.br_r[l], x = T.br_x[l], den = r * r + x * x;
            const double g = st * (r / den), b = st * (-x / den);
            Flow es, eo;
            branch_flow(g, b, vi, vo, ti, to, es);     // leaving i
            branch_flow(g, b, vo, vi, to, ti, eo);     // leaving o
            Pinj += es.P;
            Qinj += es.Q;
            // d/dv_i and d/dth_i: index 0/2 of es (i is its sending end), 1/3 of eo
            const double hs0 = 2.0 * (es.P * es.gP[0] + es.Q * es.gQ[0]);
            const double hs2 = 2.0 * (es.P * es.gP[2] + es.Q * es.gQ[2]);
            const double ho1 = 2.0 * (eo.P * eo.gP[1] + eo.Q * eo.gQ[1]);
            const double ho3 = 2.0 * (eo.P * eo.gP[3] + eo.Q * eo.gQ[3]);
            Fv += yPi * es.gP[0] + yQi * es.gQ[0] + yPo * eo.gP[1] + yQo * eo.gQ[1] + yFs * hs0 + yFo * ho1;
            Fa += yPi * es.gP[2] + yQi * es.gQ[2] + yPo * eo.gP[3] + yQo * eo.gQ[3] + yFs * hs2 + yFo * ho3;
            if (self_from) {
                const double hs = es.P * es.P + es.Q * es.Q, ho = eo.P * eo.P + eo.Q * eo.Q;
                F[rs] = hs - q.smax2 - yFs * irho + mu / yFs;
                sg[rs] = mu / (yFs * yFs);
                F[ro] = ho - q.smax2 - yFo * irho + mu / yFo;
                sg[ro] = mu / (yFo * yFo);
            }
        }
        const int gat = T.bus_gen[i];
        double pgv = 0.0, qgv = 0.0;
        if (gat >= 0) {
            const int32_t *gi = T.gen_idx + size_t(gat) * GI_N;
            pgv = z[zi(bstart, B, n, gi[GI_PG])];
            qgv = z[zi(bstart, B, n, gi[GI_QG])];
        }
        const double pd = q.pd[i];
        const int64_t cP = zi(bstart, B, n, bi[BI_P]), cQ = zi(bstart, B, n, bi[BI_Q]);
        F[cP] = Pinj - pgv + pd - yPi * irho;
        sg[cP] = 0.0;
        F[cQ] = Qinj - qgv + q.qd_ratio * pd - yQi * irho;
        sg[cQ] = 0.0;
        const int64_t cv = zi(bstart, B, n, bi[BI_VM]), ca = zi(bstart, B, n, bi[BI_VA]);
        const double lo = vi - q.vmin, hi = q.vmax - vi;
        F[cv] = Fv - mu / lo + mu / hi;
        sg[cv] = mu / (lo * lo) + mu / (hi * hi);
        F[ca] = Fa + (i == 0 ? q.eps * ti : 0.0);
        sg[ca] = i == 0 ? q.eps : 0.0;
        return;
    }
    {
        const int64_t u = u0 - nbus_t;
        const int bl = int(u % T.nblk), g = int(u / T.nblk);
        const BlockDev B = a.blks[T.blocks[bl]];
        const int32_t *gi = T.gen_idx + size_t(g) * GI_N;
        const int bus = gi[GI_BUS];
        const int32_t *bb = T.bus_idx + size_t(bus) * BI_N;
        const int64_t cq = zi(bstart, B, n, gi[GI_QG]);
        const double qg = z[cq], lo = qg + q.qmax, hi = q.qmax - qg;
        F[cq] = -z[zi(bstart, B, n, bb[BI_Q])] - mu / lo + mu / hi;
        sg[cq] = mu / (lo * lo) + mu / (hi * hi);
        if (T.has_pg_local) {
            const int64_t cp = zi(bstart, B, n, gi[GI_PG]);
            const double pg = z[cp], pl = pg, ph = q.pmax - pg;
            F[cp] = 2.0 * T.gen_c2[g] * pg - z[zi(bstart, B, n, bb[BI_P])] - mu / pl + mu / ph;
            sg[cp] = mu / (pl * pl) + mu / (ph * ph);
        }
    }
}

// Fraction-to-boundary step over every barrier argument (one workgroup:
// the elements are strided over its threads, then reduced in a fixed order).
constexpr int kStepThreads = 1024;

__device__ inline double step_limit(double x, double dx, double lo, double hi, double tau) {
    double al = 1.0;
    if (dx < 0.0 && lo > -INFINITY) al = fmin(al, tau * (x - lo) / -dx);
    if (dx > 0.0 && hi < INFINITY) al = fmin(al, tau * (hi - x) / dx);
    return al;
}

// Global column and layout kind of interleaved index idx < dint + nbd_tot
// (dispatch-map networks: the border holds pg).
__device__ inline void col_kind(const DevArgs &a, int64_t idx, int64_t &col, uint8_t &kind) {
    if (idx < a.dint) {
        const TemplDev &T = a.tmpls[find_tmpl(a, idx, &TemplDev::dbase)];
        const int64_t off = idx - T.dbase;
        const int j = int(off / T.nblk), bl = int(off % T.nblk);
        col = a.blks[T.blocks[bl]].col0 + j;
        kind = T.lkind[j];
    } else {
        const int64_t j = idx - a.dint;
        const InstDev &I = a.insts[find_inst(a, j, &InstDev::bd0)];
        col = I.bstart + (j - I.bd0);
        kind = j - I.bd0 < I.ng ? LK_PG : LK_VM0;
    }
}

__global__ __launch_bounds__(kStepThreads) void k_max_step(DevArgs a, const double *__restrict__ z,
                                                          const double *__restrict__ dz, ncl_nlp q, double tau,
                                                          double *alpha) {
    __shared__ double red[kStepThreads / 64];
    double al = 1.0;
    const int64_t total = a.dint + a.nbd_tot;
    for (int64_t idx = threadIdx.x; idx < total; idx += kStepThreads) {
        int64_t col;
        uint8_t kind;
        col_kind(a, idx, col, kind);
        const double x = z[col], dx = dz[col];
        switch (kind) {
            case LK_VM: al = fmin(al, step_limit(x, dx, q.vmin, q.vmax, tau)); break;
            case LK_QG: al = fmin(al, step_limit(x, dx, -q.qmax, q.qmax, tau)); break;
            case LK_PG: al = fmin(al, step_limit(x, dx, 0.0, q.pmax, tau)); break;
            case LK_FLOW: al = fmin(al, step_limit(x, dx, 0.0, INFINITY, tau)); break;
            default: break;
        }
    }
    for (int o = 32; o > 0; o >>= 1) al = fmin(al, __shfl_xor(al, o));
    if (lane_id() == 0) red[threadIdx.x >> 6] = al;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kStepThreads / 64; w++) m = fmin(m, red[w]);
        *alpha = m;
    }
}

// ------------------------------------------------------------------ dispatch map: Newton steps

// Elementwise steps of the dispatch map's Newton method over the N columns
// (layout order), and its deterministic reductions: every sum has a fixed
// order (each workgroup sums kRedPer consecutive elements, thread t taking
// t, t + 256, ... in turn, then a fixed shuffle tree; the final kernel sums
// the workgroups' partials in the same way), so results repeat bit for bit.
constexpr int kRedPer = 4096;
constexpr int kRedFinal = 1024;

__device__ inline double tree_sum256(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// out = y + a x  (y may be null: out = a x)
__global__ __launch_bounds__(256) void k_vec_axpy(int64_t n, double al, const double *__restrict__ x,
                                                  const double *__restrict__ y, double *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) out[i] = y ? fma(al, x[i], y[i]) : al * x[i];
}

// partial sums of squares (mode 0) or partial maxima of |dz_i| - tol (1 + |z_i|) (mode 1)
__global__ __launch_bounds__(256) void k_vec_reduce(int64_t n, const double *__restrict__ x,
                                                    const double *__restrict__ z, double tol, int mode,
                                                    double *__restrict__ part) {
    __shared__ double red[4];
    const int64_t i0 = int64_t(blockIdx.x) * kRedPer;
    double v = mode ? -INFINITY : 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i0 + kRedPer && i < n; i += 256) {
        if (mode == 0) v = fma(x[i], x[i], v);
        else {
            const double e = fabs(x[i]) - tol * (1.0 + fabs(z[i]));
            v = (e > v || e != e) ? e : v;
        }
    }
    if (mode == 0) {
        const double s = tree_sum256(v, red);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    } else {
        for (int o = 32; o > 0; o >>= 1) {
            const double w = __shfl_xor(v, o);
            v = (w > v || w != w) ? w : v;
        }
        if (lane_id() == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = red[0];
            for (int q = 1; q < 4; q++) m = (red[q] > m || red[q] != red[q]) ? red[q] : m;
            part[blockIdx.x] = m;
        }
    }
}

// out[0] = sqrt(sum of the partials) (mode 0) or their maximum (mode 1)
__global__ __launch_bounds__(kRedFinal) void k_vec_reduce_final(int64_t np, const double *__restrict__ part, int mode,
                                                                double *__restrict__ out) {
    __shared__ double red[kRedFinal / 64];
    double v = mode ? -INFINITY : 0.0;
    for (int64_t i = threadIdx.x; i < np; i += kRedFinal) v = mode ? ((part[i] > v || part[i] != part[i]) ? part[i] : v)
                                                                  : v + part[i];
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o);
        v = mode ? ((w > v || w != w) ? w : v) : v + w;
    }
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int q = 1; q < kRedFinal / 64; q++) t = mode ? ((red[q] > t || red[q] != red[q]) ? red[q] : t) : t + red[q];
        out[0] = mode ? t : sqrt(t);
    }
}

// the default start (vm = 1, pg = pmax / 2, flow-row multipliers mu / smax2,
// everything else 0) and the primal shift out = sig + dw on vm, va, qg, pg
__global__ __launch_bounds__(256) void k_disp_point(DevArgs a, ncl_nlp q, const double *__restrict__ sig, double dw,
                                                    int mode, double *__restrict__ out) {
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= a.dint + a.nbd_tot) return;
    int64_t col;
    uint8_t kind;
    col_kind(a, idx, col, kind);
    if (mode == 0) {
        out[col] = kind == LK_VM ? 1.0 : kind == LK_PG ? 0.5 * q.pmax : kind == LK_FLOW ? q.mu / q.smax2 : 0.0;
    } else {
        const bool primal = kind == LK_VM || kind == LK_VA || kind == LK_QG || kind == LK_PG;
        out[col] = primal ? sig[col] + dw : sig[col];
    }
}

// phi = sum_g c2_g pg_g^2 (generators in order) and pg (one thread)
__global__ __launch_bounds__(64) void k_disp_outputs(DevArgs a, const double *__restrict__ z, double *__restrict__ phi,
                                                     double *__restrict__ pg) {
    if (threadIdx.x != 0) return;
    const InstDev &I = a.insts[0];
    double f = 0.0;
    for (int g = 0; g < a.ng_disp; g++) {
        const double p = z[a.pg_col[g]];
        f = fma(I.gen_c2[g] * p, p, f);
        if (pg) pg[g] = p;
    }
    *phi = f;
}

// adjoint right-hand side g = d(gphi phi + gpg . pg)/dz: 2 c2 pg gphi + gpg
// on the pg columns, 0 elsewhere (mode 0 fills the zeros, then mode 1 the
// pg columns)
__global__ __launch_bounds__(256) void k_disp_adjoint_rhs(DevArgs a, const double *__restrict__ z,
                                                          const double *__restrict__ gphi,
                                                          const double *__restrict__ gpg, int mode,
                                                          double *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (mode == 0) {
        if (i < a.N) out[i] = 0.0;
    } else if (i < a.ng_disp) {
        const InstDev &I = a.insts[0];
        const int64_t c = a.pg_col[i];
        const double p = z[c];
        out[c] = fma(2.0 * I.gen_c2[i] * p, *gphi, gpg ? gpg[i] : 0.0);
    }
}

// load gradient: gpd_i = -(sum over blocks of adj at bus i's P row + qd
// times the same sum at its Q row), blocks in order
__global__ __launch_bounds__(256) void k_disp_load_grad(DevArgs a, const double *__restrict__ adj, double qd,
                                                        double *__restrict__ gpd) {
    const int i = int(blockIdx.x) * 256 + threadIdx.x;
    if (i >= a.nbus_disp) return;
    double sp = 0.0, sq = 0.0;
    for (int b = 0; b < a.nblk; b++) {
        sp += adj[a.row_pq[2 * (int64_t(b) * a.nbus_disp + i)]];
        sq += adj[a.row_pq[2 * (int64_t(b) * a.nbus_disp + i) + 1]];
    }
    gpd[i] = -(sp + qd * sq);
}

hipError_t launch_vec_axpy(int64_t n, double al, const double *x, const double *y, double *out, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_vec_axpy, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, n, al, x, y, out);
    return hipGetLastError();
}

hipError_t launch_vec_reduce(int64_t n, const double *x, const double *z, double tol, int mode, double *part,
                             double *out, hipStream_t st) {
    const int64_t np = (n + kRedPer - 1) / kRedPer;
    if (np > 0) hipLaunchKernelGGL(k_vec_reduce, dim3(unsigned(np)), dim3(256), 0, st, n, x, z, tol, mode, part);
    hipLaunchKernelGGL(k_vec_reduce_final, dim3(1), dim3(kRedFinal), 0, st, np, part, mode, out);
    return hipGetLastError();
}

int64_t vec_reduce_partials(int64_t n) { return (n + kRedPer - 1) / kRedPer; }

hipError_t launch_disp_point(const DevArgs &a, const ncl_nlp &q, const double *sig, double dw, int mode, double *out,
                             hipStream_t st) {
    const int64_t n = a.dint + a.nbd_tot;
    if (n > 0) hipLaunchKernelGGL(k_disp_point, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, a, q, sig, dw, mode, out);
    return hipGetLastError();
}

hipError_t launch_disp_outputs(const DevArgs &a, const double *z, double *phi, double *pg, hipStream_t st) {
    hipLaunchKernelGGL(k_disp_outputs, dim3(1), dim3(64), 0, st, a, z, phi, pg);
    return hipGetLastError();
}

hipError_t launch_disp_adjoint(const DevArgs &a, const double *z, const double *gphi, const double *gpg, double *out,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_disp_adjoint_rhs, dim3(unsigned((a.N + 255) / 256)), dim3(256), 0, st, a, z, gphi, gpg, 0, out);
    hipLaunchKernelGGL(k_disp_adjoint_rhs, dim3(unsigned((a.ng_disp + 255) / 256)), dim3(256), 0, st, a, z, gphi, gpg, 1,
                       out);
    return hipGetLastError();
}

hipError_t launch_disp_load_grad(const DevArgs &a, const double *adj, double qd, double *gpd, hipStream_t st) {
    hipLaunchKernelGGL(k_disp_load_grad, dim3(unsigned((a.nbus_disp + 255) / 256)), dim3(256), 0, st, a, adj, qd, gpd);
    return hipGetLastError();
}

// ------------------------------------------------------------------ IPM step

// Block (or border), residual index and kind of layout column col of a
// network handle: the last block starting at or before col holds it, or,
// past that block's columns, the border of its network follows.
struct LayPos {
    int64_t rint;                 // interleaved residual index, -1 in the border
    uint8_t kind;
    bool vref;                    // bus 0's angle of its block
};

__device__ inline LayPos lay_pos(const DevArgs &a, int64_t col) {
    int lo = 0, hi = a.nblk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.blks[mid].col0 <= col) lo = mid;
        else hi = mid - 1;
    }
    const BlockDev &B = a.blks[lo];
    const TemplDev &T = a.tmpls[B.tmpl];
    const int64_t j = col - B.col0;
    LayPos p;
    if (j < T.n) {
        p.rint = T.dbase + j * T.nblk + B.bl;
        p.kind = T.lkind[j];
        p.vref = j == T.bus_idx[BI_VA];
    } else {
        const InstDev &I = a.insts[T.inst];
        p.rint = -1;
        p.kind = col - I.bstart < I.ng ? LK_PG : LK_VM0;
        p.vref = false;
    }
    return p;
}

// Elementwise steps of the IPM direction, one thread per layout column:
// sigma of the Newton matrix, the multiplier vector (z on dual rows, 0 on
// primal positions), the reduced right-hand side from c / grad phi (in)
// and the residual -J'y the row kernels left in rint / rbuf, the recovery
// of the eliminated directions from dz (in), and the primal shift of a
// sigma (in).
__global__ __launch_bounds__(256) void k_ipm_point(DevArgs a, IpmArgs q, int mode, const double *__restrict__ in,
                                                   double dw, double *__restrict__ o0, double *__restrict__ o1,
                                                   double *__restrict__ o2, double *__restrict__ o3) {
    const int64_t col = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (col >= a.N) return;
    const LayPos p = lay_pos(a, col);
    const bool primal = lk_primal(p.kind);
    const bool comp = p.kind == LK_CUP || p.kind == LK_CLO || p.kind == LK_ACUP || p.kind == LK_ACLO;
    const bool flow = p.kind == LK_FLOW;
    if (mode == IPM_SHIFT) {
        o0[col] = primal ? in[col] + dw : in[col];
        return;
    }
    const double z = q.z[col];
    if (mode == IPM_MASK) {
        o0[col] = primal ? 0.0 : z;
    } else if (mode == IPM_YN) {
        // the first-order multiplier update: y_n takes y at the dual rows
        if (!primal) o0[col] = z;
    } else if (mode == IPM_INTERIOR) {
        // 1 where the point is not strictly interior (or not finite), else 0
        bool ok = z == z && fabs(z) < INFINITY;
        if (primal) {
            const double lo = q.lo[col], hi = q.hi[col];
            if (lo > -INFINITY) ok = ok && z > lo && q.zl[col] > 0.0;
            if (hi < INFINITY) ok = ok && z < hi && q.zu[col] > 0.0;
        } else {
            const double rt = q.rt[col];
            ok = ok && rt == rt && fabs(rt) < INFINITY;
            if (comp || flow) ok = ok && z > 0.0 && q.s[col] > 0.0;
        }
        o0[col] = ok ? 0.0 : 1.0;
    } else if (mode == IPM_ERROR) {
        // the barrier KKT residual G at this position, at mu (o0) and at 0
        // (o1), as the largest magnitude of its components, and |rt| at dual
        // rows (o2); in = c(w) and grad phi, J'y from the residual buffers
        double em = 0.0, e0 = 0.0, ar = 0.0;
        if (primal) {
            const double lo = q.lo[col], hi = q.hi[col];
            double gw = in[col] - (p.rint >= 0 ? a.rint[p.rint] : a.rbuf[col]);
            if (lo > -INFINITY) {
                const double c = (z - lo) * q.zl[col];
                gw -= q.zl[col];
                em = fmax(em, fabs(c - q.mu));
                e0 = fmax(e0, fabs(c));
            }
            if (hi < INFINITY) {
                const double c = (hi - z) * q.zu[col];
                gw += q.zu[col];
                em = fmax(em, fabs(c - q.mu));
                e0 = fmax(e0, fabs(c));
            }
            em = fmax(em, fabs(gw));
            e0 = fmax(e0, fabs(gw));
        } else {
            const double rt = q.rt[col];
            double gy = in[col] - rt;
            const double grt = q.yn[col] + q.rho * rt - z;
            if (comp || flow) {
                const double sv = q.s[col];
                gy += sv;
                em = fmax(em, fabs(sv * z - q.mu));
                e0 = fmax(e0, fabs(sv * z));
            }
            em = fmax(em, fmax(fabs(gy), fabs(grt)));
            e0 = fmax(e0, fmax(fabs(gy), fabs(grt)));
            ar = fabs(rt);
        }
        o0[col] = em;
        o1[col] = e0;
        o2[col] = ar;
    } else if (mode == IPM_SIGMA) {
        double v = 0.0;
        if (primal) {
            const double lo = q.lo[col], hi = q.hi[col];
            if (lo > -INFINITY) v += q.zl[col] / (z - lo);
            if (hi < INFINITY) v += q.zu[col] / (hi - z);
            if (p.vref) v += q.eps;
        } else if (comp) {
            v = q.s[col];
        } else if (flow) {
            v = q.s[col] / z;
        }
        o0[col] = v;
    } else if (mode == IPM_RHS) {
        double v;
        if (primal) {
            v = -in[col] + (p.rint >= 0 ? a.rint[p.rint] : a.rbuf[col]);
            const double lo = q.lo[col], hi = q.hi[col];
            if (lo > -INFINITY) v += q.mu / (z - lo);
            if (hi < INFINITY) v -= q.mu / (hi - z);
        } else {
            v = -in[col] + (z - q.yn[col]) / q.rho;
            if (comp || flow) v -= q.mu / z;
        }
        o0[col] = v;
    } else {
        const double dz = in[col];
        double drt = 0.0, ds = 0.0, dzl = 0.0, dzu = 0.0;
        if (primal) {
            const double lo = q.lo[col], hi = q.hi[col];
            if (lo > -INFINITY) {
                const double gap = z - lo, zl = q.zl[col];
                dzl = (q.mu - gap * zl - zl * dz) / gap;
            }
            if (hi < INFINITY) {
                const double gap = hi - z, zu = q.zu[col];
                dzu = (q.mu - gap * zu + zu * dz) / gap;
            }
        } else {
            drt = (dz + z - q.yn[col] - q.rho * q.rt[col]) / q.rho;
            if (comp || flow) {
                const double sv = q.s[col];
                ds = q.mu / z - sv - sv / z * dz;
            }
        }
        o0[col] = drt;
        o1[col] = ds;
        o2[col] = dzl;
        o3[col] = dzu;
    }
}

// Constraint values c(w) at every dual row and grad phi at every primal
// position.  Threads as in the assembly: per template (bus, block), then
// (generator, block), then one per generator of the network's border.  A
// bus thread writes its vm (when in the block), va, P and Q rows and, for
// the branches it is the from end of, both flow rows; a generator thread
// its qg (and a single block's pg) and, with PV/PQ rows, its four
// complementarity variables and five rows, with AGC rows its pgk, pi+-,
// the two slacks (generator 0 also delta) and the five AGC rows; a border
// thread pg and vm0.
__global__ __launch_bounds__(256) void k_ipm_cons(DevArgs a, IpmArgs q, double *__restrict__ cg) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const double *z = q.z;
    if (tid >= a.asm_threads) {
        const int64_t gg = tid - a.asm_threads;
        if (gg >= a.gp_tot) return;
        const InstDev &I = a.insts[find_inst(a, gg, &InstDev::gp0)];
        const int g = int(gg - I.gp0);
        if (I.nbd == 0 || g >= I.ng) return;
        const int64_t col = I.bstart + I.border_pg[g];
        cg[col] = 2.0 * I.gen_c2[g] * z[col];
        if (I.nbd > I.ng) cg[I.bstart + I.ng + g] = 0.0;
        return;
    }
    const TemplDev &T = a.tmpls[find_tmpl(a, tid, &TemplDev::abase)];
    const int64_t u0 = tid - T.abase;
    const int64_t nbus_t = int64_t(T.nblk) * T.nbus;
    const int64_t bstart = a.insts[T.inst].bstart;
    const int n = T.n;
    if (u0 < nbus_t) {
        const int bl = int(u0 % T.nblk), i = int(u0 / T.nblk);
        const BlockDev B = a.blks[T.blocks[bl]];
        const int32_t *bi = T.bus_idx + size_t(i) * BI_N;
        const double vi = z[zi(bstart, B, n, bi[BI_VM])], ti = z[zi(bstart, B, n, bi[BI_VA])];
        double Pinj = 0.0, Qinj = 0.0;
        for (int qa = T.bus_adj_ptr[i]; qa < T.bus_adj_ptr[i + 1]; qa++) {
            const int32_t e = T.bus_adj[qa];
            const bool self_from = e >= 0;
            const int l = self_from ? e : ~e;
            const int32_t *br = T.br_idx + size_t(l) * 4;
            const int o = self_from ? br[3] : br[2];
            const int32_t *bo = T.bus_idx + size_t(o) * BI_N;
            const double vo = z[zi(bstart, B, n, bo[BI_VM])], to = z[zi(bstart, B, n, bo[BI_VA])];
            const double st = (l == B.outage) ? 0.0 : 1.0;
            const double r = T.br_r[l], x = T.br_x[l], den = r * r + x * x;
            const double g = st * (r / den), b = st * (-x / den);
            Flow es, eo;
            branch_flow(g, b, vi, vo, ti, to, es);
            Pinj += es.P;
            Qinj += es.Q;
            if (self_from) {
                branch_flow(g, b, vo, vi, to, ti, eo);
                cg[zi(bstart, B, n, br[0])] = es.P * es.P + es.Q * es.Q - q.smax2;
                cg[zi(bstart, B, n, br[1])] = eo.P * eo.P + eo.Q * eo.Q - q.smax2;
            }
        }
        const int gat = T.bus_gen[i];
        double pgv = 0.0, qgv = 0.0;
        if (gat >= 0) {
            const int32_t *gi = T.gen_idx + size_t(gat) * GI_N;
            // a screening block without AGC rows has no pg column: pg0 is data
            pgv = gi[GI_PG] >= 0 ? z[zi(bstart, B, n, gi[GI_PG])] : q.pg0[gat];
            qgv = z[zi(bstart, B, n, gi[GI_QG])];
        }
        const double pd = q.pd[i];
        cg[zi(bstart, B, n, bi[BI_P])] = Pinj - pgv + pd;
        cg[zi(bstart, B, n, bi[BI_Q])] = Qinj - qgv + q.qd_ratio * pd;
        if (bi[BI_VM] < n) cg[zi(bstart, B, n, bi[BI_VM])] = 0.0;
        cg[zi(bstart, B, n, bi[BI_VA])] = i == 0 ? q.eps * ti : 0.0;
        return;
    }
    const int64_t u = u0 - nbus_t;
    const int bl = int(u % T.nblk), g = int(u / T.nblk);
    const BlockDev B = a.blks[T.blocks[bl]];
    const int32_t *gi = T.gen_idx + size_t(g) * GI_N;
    const int64_t cq = zi(bstart, B, n, gi[GI_QG]);
    cg[cq] = 0.0;
    if (T.has_pg_local) {
        const int64_t cp = zi(bstart, B, n, gi[GI_PG]);
        cg[cp] = 2.0 * T.gen_c2[g] * z[cp];
    }
    if (T.pvpq_rows) {
        const int64_t cnup = zi(bstart, B, n, gi[GI_NUP]), cnum = zi(bstart, B, n, gi[GI_NUM]);
        const int64_t csup = zi(bstart, B, n, gi[GI_SUP]), cslo = zi(bstart, B, n, gi[GI_SLO]);
        const double nup = z[cnup], num = z[cnum], sup = z[csup], slo = z[cslo], qg = z[cq];
        const int32_t *bb = T.bus_idx + size_t(gi[GI_BUS]) * BI_N;
        const double vi = z[zi(bstart, B, n, bb[BI_VM])];
        const double v0 = gi[GI_VM0] >= 0 ? z[zi(bstart, B, n, gi[GI_VM0])] : q.vm0[g];
        cg[cnup] = 0.0;
        cg[cnum] = 0.0;
        cg[csup] = 0.0;
        cg[cslo] = 0.0;
        cg[zi(bstart, B, n, gi[GI_LIN])] = nup - num - vi + v0;
        cg[zi(bstart, B, n, gi[GI_DUP])] = sup - (q.qmax - qg);
        cg[zi(bstart, B, n, gi[GI_DLO])] = slo - (qg + q.qmax);
        cg[zi(bstart, B, n, gi[GI_CUP])] = num * sup;
        cg[zi(bstart, B, n, gi[GI_CLO])] = nup * slo;
    }
    if (T.agc_rows) {
        // eq. (droopmpec); phi does not depend on pgk, pi+-, the slacks or delta
        const int64_t cpk = zi(bstart, B, n, gi[GI_PG]);
        const int64_t cpip = zi(bstart, B, n, gi[GI_PIP]), cpim = zi(bstart, B, n, gi[GI_PIM]);
        const int64_t cspu = zi(bstart, B, n, gi[GI_SPU]), cspl = zi(bstart, B, n, gi[GI_SPL]);
        const int64_t cdel = zi(bstart, B, n, gi[GI_DELTA]);
        const double pk = z[cpk], pip = z[cpip], pim = z[cpim], spu = z[cspu], spl = z[cspl];
        const double p0 = gi[GI_PG0] >= 0 ? z[zi(bstart, B, n, gi[GI_PG0])] : q.pg0[g];
        cg[cpk] = 0.0;
        cg[cpip] = 0.0;
        cg[cpim] = 0.0;
        cg[cspu] = 0.0;
        cg[cspl] = 0.0;
        if (g == 0) cg[cdel] = 0.0;
        cg[zi(bstart, B, n, gi[GI_ALIN])] = pip - pim - pk + p0 + T.gen_alpha[g] * z[cdel];
        cg[zi(bstart, B, n, gi[GI_ADUP])] = spu - (q.pmax - pk);
        cg[zi(bstart, B, n, gi[GI_ADLO])] = spl - pk;
        cg[zi(bstart, B, n, gi[GI_ACUP])] = pim * spu;
        cg[zi(bstart, B, n, gi[GI_ACLO])] = pip * spl;
    }
}

hipError_t launch_ipm_point(const DevArgs &a, const IpmArgs &q, int mode, const double *in, double dw, double *o0,
                            double *o1, double *o2, double *o3, hipStream_t st) {
    if (a.N > 0)
        hipLaunchKernelGGL(k_ipm_point, dim3(unsigned((a.N + 255) / 256)), dim3(256), 0, st, a, q, mode, in, dw, o0, o1,
                           o2, o3);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_ipm_line(DevArgs a, IpmArgs q, IpmMove m, int mode, double t,
                                                  double ad, double *__restrict__ o0, double *__restrict__ o1) {
    const int64_t col = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (col >= a.N) return;
    const LayPos p = lay_pos(a, col);
    const bool primal = lk_primal(p.kind);
    const bool ineq = p.kind == LK_CUP || p.kind == LK_CLO || p.kind == LK_ACUP || p.kind == LK_ACLO ||
                      p.kind == LK_FLOW;
    const double dz = m.dz[col];
    if (mode == IPM_FTB) {
        // 1 / alpha limits: x + alpha dx >= (1 - tau) x for x > 0, dx < 0
        const double tau = t;
        double ip = 1.0, id = 1.0;
        if (primal) {
            const double w = m.z[col], lo = q.lo[col], hi = q.hi[col];
            if (lo > -INFINITY) {
                if (dz < 0.0) ip = fmax(ip, -dz / (tau * (w - lo)));
                const double dl = m.dzl[col];
                if (dl < 0.0) id = fmax(id, -dl / (tau * m.zl[col]));
            }
            if (hi < INFINITY) {
                if (dz > 0.0) ip = fmax(ip, dz / (tau * (hi - w)));
                const double du = m.dzu[col];
                if (du < 0.0) id = fmax(id, -du / (tau * m.zu[col]));
            }
        } else if (ineq) {
            const double ds = m.ds[col];
            if (ds < 0.0) ip = fmax(ip, -ds / (tau * m.s[col]));
            if (dz < 0.0) id = fmax(id, -dz / (tau * m.z[col]));
        }
        o0[col] = ip;
        o1[col] = id;
        return;
    }
    const double ap = t;
    if (primal) {
        m.z[col] += ap * dz;
        if (q.lo[col] > -INFINITY) m.zl[col] += ad * m.dzl[col];
        if (q.hi[col] < INFINITY) m.zu[col] += ad * m.dzu[col];
    } else {
        m.z[col] += (ineq ? ad : ap) * dz;
        m.rt[col] += ap * m.drt[col];
        if (ineq) m.s[col] += ap * m.ds[col];
    }
}

hipError_t launch_ipm_line(const DevArgs &a, const IpmArgs &q, const IpmMove &m, int mode, double tau_or_ap,
                           double ad, double *o0, double *o1, hipStream_t st) {
    if (a.N > 0)
        hipLaunchKernelGGL(k_ipm_line, dim3(unsigned((a.N + 255) / 256)), dim3(256), 0, st, a, q, m, mode, tau_or_ap,
                           ad, o0, o1);
    return hipGetLastError();
}

hipError_t launch_ipm_cons(const DevArgs &a, const IpmArgs &q, double *cg, hipStream_t st) {
    const int64_t n = a.asm_threads + a.gp_tot;
    if (n > 0) hipLaunchKernelGGL(k_ipm_cons, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, a, q, cg);
    return hipGetLastError();
}

// ------------------------------------------------------------------ streaming copy

// Plain copy d = s of n2 16-byte elements: each thread moves kCopyPer
// elements strided by the workgroup, all loads issued before the stores.
// Used to measure the bandwidth a streaming kernel reaches on this GPU.
constexpr int kCopyPer = 4;

__global__ __launch_bounds__(256) void k_copy(const double2 *__restrict__ s, double2 *__restrict__ d, int64_t n2) {
    const int64_t i0 = int64_t(blockIdx.x) * (256 * kCopyPer) + threadIdx.x;
    double2 v[kCopyPer];
#pragma unroll
    for (int q = 0; q < kCopyPer; q++) {
        const int64_t i = i0 + 256 * q;
        if (i < n2) v[q] = s[i];
    }
#pragma unroll
    for (int q = 0; q < kCopyPer; q++) {
        const int64_t i = i0 + 256 * q;
        if (i < n2) d[i] = v[q];
    }
}

hipError_t launch_copy(const double *src, double *dst, int64_t n, hipStream_t st) {
    const int64_t n2 = n / 2;
    const int64_t g = (n2 + 256 * kCopyPer - 1) / (256 * kCopyPer);
    if (g) hipLaunchKernelGGL(k_copy, dim3(unsigned(g)), dim3(256), 0, st, reinterpret_cast<const double2 *>(src),
                              reinterpret_cast<double2 *>(dst), n2);
    return hipGetLastError();
}

// ------------------------------------------------------------------ library-held scratch

// Device memory of the entry points that allocate nothing: one array per
// GPU, held from module load until the process ends.  In host code the
// array's name is only a stand-in for its device address; the address of
// each device's copy comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is ever passed to a
// kernel or a copy.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_address(double **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

// ------------------------------------------------------------------ launchers

// Task lists at most this long run one task per workgroup (four wavefronts
// splitting each sum), longer ones one task per wavefront: either way the
// GPU holds a few waves per SIMD.
constexpr int kSplitTasks = 2048;

static inline unsigned waves_grid(int nw) { return unsigned((nw + (kWG / 64) - 1) / (kWG / 64)); }
static inline unsigned elems_grid(int64_t n) { return unsigned((n + 255) / 256); }

// Dynamic LDS a workgroup may use on the current device (queried once).
static int max_lds_per_workgroup() {
    static int bytes = -1;
    if (bytes < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        bytes = v;
    }
    return bytes;
}

// One kernel per call, so that a caller can bracket exactly one kernel
// with events.
hipError_t launch(int kind, const DevArgs &a, const LaunchArgs &l, hipStream_t st) {
    switch (kind) {
        case NCL_K_ASSEMBLE: {
            const int64_t total = a.asm_wthreads + a.gp_tot;
            if (total)
                hipLaunchKernelGGL(k_assemble, dim3(elems_grid(total)), dim3(256), 0, st, a, l.z, l.sig, l.rho,
                                   (l.flags & NCL_NO_SHIFT) ? 1 : 0);
            break;
        }
        case NCL_K_VALUES: {
            const int64_t total = a.kint + a.nbb_tot;
            if (total)
                hipLaunchKernelGGL(k_values, dim3(elems_grid(total)), dim3(256), 0, st, a, l.src, l.dst,
                                   l.to_internal ? 1 : 0);
            break;
        }
        case NCL_K_FAC_GATHER:
            if (l.nw) hipLaunchKernelGGL(k_fac_gather, dim3(waves_grid(l.nw)), dim3(kWG), 0, st, a, l.wl, l.nw);
            break;
        case NCL_K_FAC_DIAG:
            if (l.nw) hipLaunchKernelGGL(k_fac_diag, dim3(waves_grid(l.nw)), dim3(kWG), 0, st, a, l.wl, l.nw);
            break;
        case NCL_K_FAC_ROWS:
            if (l.nw) hipLaunchKernelGGL(k_fac_rows, dim3(waves_grid(l.nw)), dim3(kWG), 0, st, a, l.wl, l.nw);
            break;
        case NCL_K_BORDER_SCHUR:
            if (a.mw_tot) {
                const int64_t need = (a.mw_tot + kWG / 64 - 1) / (kWG / 64);
                const int64_t grid = l.shared_gpu && need > kSchurGrid ? kSchurGrid : need;
                hipLaunchKernelGGL(k_border_schur, dim3(unsigned(grid)), dim3(kWG), 0, st, a);
            }
            break;
        case NCL_K_BORDER_SUM:
            if (a.pe_tot) hipLaunchKernelGGL(k_border_sum, dim3(unsigned((a.pe_tot + 255) / 256)), dim3(256), 0, st, a);
            break;
        case NCL_K_BORDER_FACTOR:
            if (!a.max_nbd) break;
            if (l.b0 == -2) {
                // the register path; tiles per thread: enough for the largest border that takes it
                const int nreg = a.max_nbd < 4 * kBFRegMaxNt ? a.max_nbd : 4 * kBFRegMaxNt;
                const int mt = (nreg + 3) / 4, tpt = (mt * (mt + 1) / 2 + kBFThreads - 1) / kBFThreads;
                const size_t lb = size_t(8) * 4 * mt * sizeof(double);
                const void *fn = tpt <= 1 ? reinterpret_cast<const void *>(&k_border_factor<1>)
                               : tpt == 2 ? reinterpret_cast<const void *>(&k_border_factor<2>)
                                          : reinterpret_cast<const void *>(&k_border_factor<3>);
                if (lb > 65536) {
                    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lb));
                    if (e != hipSuccess) return e;
                }
                switch (tpt) {
                    case 1: hipLaunchKernelGGL(k_border_factor<1>, dim3(a.ninst), dim3(kBFThreads), lb, st, a); break;
                    case 2: hipLaunchKernelGGL(k_border_factor<2>, dim3(a.ninst), dim3(kBFThreads), lb, st, a); break;
                    default: hipLaunchKernelGGL(k_border_factor<3>, dim3(a.ninst), dim3(kBFThreads), lb, st, a); break;
                }
            } else {
                // blocked path: column block b = -1 .. (blocks of the largest border) - 2
                const int nbk = (a.max_nbd + kBB - 1) / kBB, rem = nbk - l.b0 - 1;
                const unsigned nt = l.b0 < 0 ? 1u : unsigned(rem > 0 ? rem * (rem + 1) / 2 : 0);
                if (nt) hipLaunchKernelGGL(k_border_step, dim3(nt, unsigned(a.ninst)), dim3(kBSThreads), 0, st, a, l.b0);
            }
            break;
        case NCL_K_STATUS_INIT:
            hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, st, a);
            break;
        case NCL_K_STATUS: {
            const int64_t ne = a.dint + a.nbd_tot;
            const unsigned sg = unsigned((ne + 4 * kStatusChunk - 1) / (4 * kStatusChunk));
            if (sg) hipLaunchKernelGGL(k_status, dim3(sg), dim3(256), 0, st, a);
            break;
        }
        case NCL_K_SOL_LOAD:
            if (a.dint && l.src)
                hipLaunchKernelGGL(k_sol_load_int, dim3(elems_grid(a.dint)), dim3(256), 0, st, a, l.src, l.y);
            else if (a.dint)
                hipLaunchKernelGGL(k_sol_load, dim3(unsigned(a.tiles), unsigned(l.nrhs)), dim3(256), 0, st, a, l.b, l.y,
                                   l.bld, l.ys, l.nocheck ? 0 : 1);
            break;
        case NCL_K_SOL_FWD_GATHER:
            if (l.nw > kSplitTasks)
                hipLaunchKernelGGL(k_sol_fwd_gather<1>, dim3(waves_grid(l.nw), unsigned(l.nrhs)), dim3(kWG), 0, st, a, l.y,
                                   l.wl, l.nw, l.ys);
            else if (l.nw)
                hipLaunchKernelGGL(k_sol_fwd_gather<kSplit>, dim3(unsigned(l.nw), unsigned(l.nrhs)), dim3(kWG), 0, st, a,
                                   l.y, l.wl, l.nw, l.ys);
            break;
        case NCL_K_SOL_FWD_DIAG:
            if (l.nw)
                hipLaunchKernelGGL(k_sol_fwd_diag, dim3(waves_grid(l.nw), unsigned(l.nrhs)), dim3(kWG), 0, st, a, l.y, l.wl,
                                   l.nw, l.ys);
            break;
        case NCL_K_SOL_BPART:
            if (l.nw > kSplitTasks)
                hipLaunchKernelGGL(k_sol_bpart<1>, dim3(waves_grid(l.nw), unsigned(l.nrhs)), dim3(kWG), 0, st, a, l.y,
                                   l.cpart, l.wl, l.nw, l.ys, l.cps);
            else if (l.nw)
                hipLaunchKernelGGL(k_sol_bpart<kSplit>, dim3(unsigned(l.nw), unsigned(l.nrhs)), dim3(kWG), 0, st, a, l.y,
                                   l.cpart, l.wl, l.nw, l.ys, l.cps);
            break;
        case NCL_K_SOL_BORDER:
            if (a.max_nbd > 0) {
                // LDS for the largest factor that fits one workgroup; larger
                // instances read theirs from global memory
                const size_t cap = size_t(max_lds_per_workgroup());
                size_t lb = size_t(a.max_nbd + a.max_nbd * (a.max_nbd + 1) / 2) * sizeof(double);
                if (lb > cap) lb = cap;
                if (lb > 65536) {
                    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sol_border),
                                                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lb));
                    if (e != hipSuccess) return e;
                }
                hipLaunchKernelGGL(k_sol_bsum, dim3(unsigned((a.nbd_tot + 3) / 4), unsigned(l.nrhs)), dim3(256), 0, st, a, l.b,
                                   l.y, l.cpart, l.bld, l.ys, l.cps);
                hipLaunchKernelGGL(k_sol_border, dim3(unsigned(a.ninst), unsigned(l.nrhs)), dim3(kBorderThreads), lb, st, a,
                                   l.x, l.y, int64_t(lb), l.accumulate ? 1 : 0, l.bld, l.ys);
            }
            break;
        case NCL_K_SOL_BWD_BORDER:
            if (l.nw)
                hipLaunchKernelGGL(k_sol_bwd_border, dim3(unsigned((l.nnar + 3) / 4 + (l.nw - l.nnar)), unsigned(l.nrhs)),
                                   dim3(kWG), 0, st, a, l.y, l.wl, l.nw, l.nnar, l.ys);
            break;
        case NCL_K_SOL_BWD:
            if (l.nw) {
                const size_t lb = l.nw > l.nnar ? size_t(3) * size_t(l.wmax) * 64 * sizeof(double) : 0;
                const dim3 g(unsigned((l.nnar + 3) / 4 + (l.nw - l.nnar)), unsigned(l.nrhs));
                if (l.wmax <= 8) hipLaunchKernelGGL(k_sol_bwd<8>, g, dim3(kWG), lb, st, a, l.y, l.wl, l.nw, l.nnar, l.ys);
                else if (l.wmax <= 16)
                    hipLaunchKernelGGL(k_sol_bwd<16>, g, dim3(kWG), lb, st, a, l.y, l.wl, l.nw, l.nnar, l.ys);
                else hipLaunchKernelGGL(k_sol_bwd<32>, g, dim3(kWG), lb, st, a, l.y, l.wl, l.nw, l.nnar, l.ys);
            }
            break;
        case NCL_K_SOL_STORE:
            if (a.dint && l.accumulate)
                hipLaunchKernelGGL(k_sol_store<true>, dim3(unsigned(a.tiles), unsigned(l.nrhs)), dim3(256), 0, st, a, l.y, l.x,
                                   l.ys, l.bld);
            else if (a.dint)
                hipLaunchKernelGGL(k_sol_store<false>, dim3(unsigned(a.tiles), unsigned(l.nrhs)), dim3(256), 0, st, a, l.y,
                                   l.x, l.ys, l.bld);
            break;
        case NCL_K_BERR_ROWS:
            if (a.rows_waves)
                hipLaunchKernelGGL(k_berr_rows, dim3(unsigned(a.rows_wg)), dim3(256), 0, st, a);
            break;
        case NCL_K_BERR_BORDER:
            if (a.nbd_tot)
                hipLaunchKernelGGL(k_berr_border, dim3(unsigned((a.nbd_tot + 3) / 4)), dim3(256), 0, st, a);
            break;
        case NCL_K_BERR_FINAL:
            hipLaunchKernelGGL(k_berr_final, dim3(1), dim3(kFinalThreads), 0, st, a, l.dst);
            break;
        case NCL_K_RESIDUAL: {
            const int64_t total = a.asm_threads + a.gp_tot;
            if (total)
                hipLaunchKernelGGL(k_residual, dim3(elems_grid(total)), dim3(256), 0, st, a, l.z, l.nlp, l.F,
                                   l.sigma_out, l.rho);
            break;
        }
        case NCL_K_INTERLEAVE: {
            const int64_t nt = a.tiles + (a.nbd_tot + 255) / 256;
            if (nt) hipLaunchKernelGGL(k_interleave, dim3(unsigned(nt)), dim3(256), 0, st, a, l.z, l.sig, l.zdst, l.sdst);
            break;
        }
        case NCL_K_MAX_STEP:
            hipLaunchKernelGGL(k_max_step, dim3(1), dim3(kStepThreads), 0, st, a, l.z, l.dz, l.nlp, l.tau, l.alpha);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ncl
