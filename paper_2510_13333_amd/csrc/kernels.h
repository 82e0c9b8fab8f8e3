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
    int64_t asm_threads, gp_tot;   // assembly threads of the templates, then of the border pg values
    double *kval, *lpan, *dval, *spart, *sbb, *ybuf, *cpart;
    int64_t *stat;              // npos, nneg, nzero, first bad key, min |d| bits, max |d| bits
    const uint8_t *bprim;       // [nbd_tot] expected sign of the border pivots
};

hipError_t launch_assemble(const DevArgs &a, const double *z, const double *sig, double rho, hipStream_t st);
hipError_t launch_values(const DevArgs &a, const double *src, double *dst, bool to_internal, hipStream_t st);
hipError_t launch_factor_level(const DevArgs &a, const Work *wa, int na, const Work *wb, int nb, const Work *wc,
                               int nc, hipStream_t st);
hipError_t launch_schur(const DevArgs &a, const Work *ws, int nw, hipStream_t st);
hipError_t launch_factor_border(const DevArgs &a, hipStream_t st);
size_t border_lds_bytes(int nbd);   // dynamic LDS of the dense border factor (largest border)
hipError_t launch_solve_load(const DevArgs &a, const double *b, double *y, hipStream_t st);
hipError_t launch_solve_fwd_level(const DevArgs &a, double *y, const Work *wf, int nf, const Work *wd, int nd,
                                  hipStream_t st);
hipError_t launch_solve_bpart(const DevArgs &a, const double *y, double *cpart, const Work *wp, int np,
                              hipStream_t st);
hipError_t launch_solve_border(const DevArgs &a, const double *b, double *x, double *y, const double *cpart,
                               hipStream_t st);
hipError_t launch_solve_scale(const DevArgs &a, double *y, hipStream_t st);
hipError_t launch_solve_bwd_level(const DevArgs &a, double *y, const Work *wg, int ng, const Work *wd, int nd,
                                  hipStream_t st);
hipError_t launch_solve_store(const DevArgs &a, const double *y, double *x, hipStream_t st);

}  // namespace ncl
