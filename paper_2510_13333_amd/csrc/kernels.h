// Arguments and launchers of the device kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include "ncl_internal.h"

namespace ncl {

// Device state shared by every kernel (pointers into the workspace).
struct DevArgs {
    const TemplDev *tmpls;
    const BlockDev *blks;
    const InstDev *insts;
    int ntmpl, nblk, ninst, max_nbd;
    int64_t N;
    int64_t kint;               // interleaved K values; the border K_bb values of every instance follow
    int64_t dint;               // interleaved pivots; the border pivots of every instance follow
    int64_t nbd_tot, nbb_tot, npk_tot;
    int64_t asm_threads, gp_tot;   // residual threads of the templates, then of the border pg values
    int64_t asm_wthreads;          // assembly threads of the templates (wavefront-aligned), then border pg
    int64_t mw_tot;                // border Schur wavefronts of all instances
    int64_t pe_tot;                // border partial-sum threads (tile-pair entries) of all instances
    int64_t tiles;              // state transpose tiles of all templates
    double *kval, *lpan, *dval, *spart, *sbb, *ybuf, *cpart;
    double *lbb;                   // the border factor L (packed like sbb)
    double *upan;                  // U = L D on the off-diagonal panel rows (rows >= w), panel layout
    double *zint, *sint;        // interleaved copies of the state and Sigma (assembly input)
    int64_t *stat;              // npos, nneg, nzero, first bad key, min |d| bits, max |d| bits, non-finite
    const uint8_t *bprim;       // [dint + nbd_tot] expected sign of every pivot (1: positive), in dval's order
    int64_t rows_waves;         // residual-row wavefronts of all templates
    int64_t nprimal;            // expected positive pivots
    int rows_wg;                // workgroups of the residual-row kernel
    double *xint, *bint, *rint; // residual: x, b and r in the interleaved layout order
    double *rbuf;               // residual in layout order (border part)
    double *epart;              // partial maxima of the backward error, 8 per workgroup
    // dispatch map (a single network without PV/PQ rows)
    int ng_disp, nbus_disp;
    const int64_t *pg_col;      // [ng] global column of each generator's pg
    const int64_t *row_pq;      // [nblk][nbus][2] global P and Q rows of each bus in each block
};

// Arguments of one launch (only those the kernel kind uses are read).
// Dense border factor: borders of up to kBorderRegMax rows in registers by
// one workgroup (b0 = -2); larger ones right-looking by column blocks of
// kBorderBlock, one launch per block (b0 = block index, -1 for the first
// diagonal block).
constexpr int kBorderBlock = 32;
constexpr int kBorderRegMax = 216;
// status words: 6 counters, each on a cache line of its own so that the
// workgroups' atomics on different counters do not queue on one line
constexpr int kStatStride = 16;
constexpr int kStatWords = 8;

struct LaunchArgs {
    const Work *wl = nullptr;   // work list and its length
    int nw = 0;
    int b0 = 0;                 // border column block of a border factor launch (-1: the first diagonal block)
    const double *z = nullptr, *sig = nullptr;   // assembly state
    double rho = 0.0;
    uint32_t flags = 0;                          // NCL_NO_SHIFT
    ncl_nlp nlp{};                               // dispatch map: parameters, outputs, step
    double *F = nullptr, *sigma_out = nullptr;
    const double *dz = nullptr;
    double tau = 0.0;
    double *alpha = nullptr;
    double *zdst = nullptr, *sdst = nullptr;     // interleave: destinations of z and sig
    const double *src = nullptr;                 // value conversion; solve load: interleaved right-hand side
    double *dst = nullptr;                       // value conversion; backward error: (eta, omega)
    bool to_internal = false;
    bool accumulate = false;                     // solve store: x += solution
    bool nocheck = false;                        // solve load: do not consult the factorisation status
    bool shared_gpu = false;                     // border Schur: cap the grid, for running beside other work (the library's call paths run it alone)
    const double *b = nullptr;                   // solve: right-hand side, solution, work vectors
    double *x = nullptr, *y = nullptr, *cpart = nullptr;
    int nnar = 0;                                // solve levels: narrow items first in the list
    int wmax = 0;                                // solve levels: widest supernode of the level (8, 16 or 32 class)
    int nrhs = 1;                                // solve: right-hand sides of the launch (grid dimension y)
    int64_t bld = 0, ys = 0, cps = 0;            // solve: strides between right-hand sides of b and x, y, cpart
};

// Launch one kernel of the given kind (NCL_K_* of ncl_kkt.h) on stream st.
hipError_t launch(int kind, const DevArgs &a, const LaunchArgs &l, hipStream_t st);

// Library-held device scratch (doubles) of the entry points that allocate
// nothing, and its address on the current device (looked up once per device).
constexpr int64_t kScratchDoubles = int64_t(6) << 20;
hipError_t scratch_address(double **out);

// Dispatch map: vector steps of its Newton method (deterministic reductions
// use part[] of vec_reduce_partials(n) doubles).
hipError_t launch_vec_axpy(int64_t n, double al, const double *x, const double *y, double *out, hipStream_t st);
hipError_t launch_vec_reduce(int64_t n, const double *x, const double *z, double tol, int mode, double *part,
                             double *out, hipStream_t st);
int64_t vec_reduce_partials(int64_t n);
hipError_t launch_disp_point(const DevArgs &a, const ncl_nlp &q, const double *sig, double dw, int mode, double *out,
                             hipStream_t st);
hipError_t launch_disp_outputs(const DevArgs &a, const double *z, double *phi, double *pg, hipStream_t st);
hipError_t launch_disp_adjoint(const DevArgs &a, const double *z, const double *gphi, const double *gpg, double *out,
                               hipStream_t st);
hipError_t launch_disp_load_grad(const DevArgs &a, const double *adj, double qd, double *gpd, hipStream_t st);

// IPM step of the NCL subproblem: its data and point (layout order) and
// the elementwise modes of launch_ipm_point.
struct IpmArgs {
    const double *pd = nullptr, *lo = nullptr, *hi = nullptr, *yn = nullptr;
    const double *z = nullptr, *rt = nullptr, *s = nullptr, *zl = nullptr, *zu = nullptr;
    const double *pg0 = nullptr, *vm0 = nullptr;   // fixed first stage (screening networks)
    double qd_ratio = 0.0, qmax = 0.0, pmax = 0.0, smax2 = 0.0, eps = 0.0, mu = 0.0, rho = 0.0;
};
enum IpmMode { IPM_SIGMA = 0, IPM_MASK, IPM_RHS, IPM_RECOVER, IPM_SHIFT, IPM_ERROR, IPM_YN, IPM_INTERIOR };
hipError_t launch_ipm_point(const DevArgs &a, const IpmArgs &q, int mode, const double *in, double dw, double *o0,
                            double *o1, double *o2, double *o3, hipStream_t st);
hipError_t launch_ipm_cons(const DevArgs &a, const IpmArgs &q, double *cg, hipStream_t st);
// The IPM state (written in place by IPM_UPDATE) and a direction.
struct IpmMove {
    double *z = nullptr, *rt = nullptr, *s = nullptr, *zl = nullptr, *zu = nullptr;
    const double *dz = nullptr, *drt = nullptr, *ds = nullptr, *dzl = nullptr, *dzu = nullptr;
};
enum IpmLineMode { IPM_FTB = 0, IPM_UPDATE };
// IPM_FTB: per position the reciprocals of the largest primal (o0) and dual
// (o1) steps in (0, 1] that keep the bounded quantities above (1 - tau) of
// their values (1 where nothing limits); IPM_UPDATE: the state moves by ap
// (w, y at equality rows, rt, s) and ad (zl, zu, y at inequality rows).
hipError_t launch_ipm_line(const DevArgs &a, const IpmArgs &q, const IpmMove &m, int mode, double tau_or_ap,
                           double ad, double *o0, double *o1, hipStream_t st);

// Streaming copy of n doubles (n even, both pointers 16-byte aligned).
hipError_t launch_copy(const double *src, double *dst, int64_t n, hipStream_t st);

}  // namespace ncl
