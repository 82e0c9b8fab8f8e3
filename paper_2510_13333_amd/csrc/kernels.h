// Argument structs and launchers of the device kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include "ncl_internal.h"

namespace ncl {

struct AsmArgs {
    const TemplDev *tmpls;
    const BlockDev *blks;
    int nblk, nb, ng, nbd;
    const double *z, *sig;
    double rho;
    double *kval;
    int64_t kbase_border, bstart;
    const double *br_r, *br_x, *gen_c2;
    const int32_t *border_pg, *kbb_pos;
};

struct FactorArgs {
    const TemplDev *tmpls;
    const BlockDev *blks;
    const double *kval;
    double *lpan, *dval, *spart;
    int64_t *stat;            // [nblk][4]: npos, nneg, nzero, first bad key (col*8+code)
    double *dminmax;          // [nblk][2]
    int nbd;
};

struct BorderArgs {
    int nblk, nbd;
    const double *kval;
    int64_t kbase_border;
    const int32_t *kbb_pos;
    const double *spart;
    double *sbb;               // packed lower S, then L_bb (unit lower, strict part) in place
    double *dval;              // border pivots at dval[bcol0 ..]
    int64_t bcol0;
    const uint8_t *bprimal;
    int64_t *stat;             // [nblk+1][4]; border row at nblk
    double *dminmax;
};

struct SolveArgs {
    const TemplDev *tmpls;
    const BlockDev *blks;
    const double *lpan, *dval, *sbb;
    double *ybuf, *cpart;
    const double *b;
    double *x;
    int64_t ld, N, bstart;
    int nblk, nbd, nrhs;
};

hipError_t launch_assemble(const AsmArgs &a, hipStream_t st);
hipError_t launch_factor_blocks(const FactorArgs &fa, int nblk, hipStream_t st);
hipError_t launch_factor_border(const BorderArgs &ba, hipStream_t st);
hipError_t launch_solve(const SolveArgs &a, hipStream_t st);

}  // namespace ncl
