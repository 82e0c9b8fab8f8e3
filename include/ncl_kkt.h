/*
 * ncl_kkt.h -- C ABI of the MI355X (gfx950) library for the Newton step of
 * the NCL augmented-Lagrangian method for security-constrained AC optimal
 * power flow (the regularised KKT system of Section IV-B, eq. (newtonsystem)).
 *
 * Each interior-point iteration of NCL solves
 *
 *        [ A   B^T ] [dw]   [r1]        A = H + Sigma (+ nu0 off-diagonals)
 *        [ B   -C  ] [dy] = [r2],       B = [J; 0 W2 W1],  C = diag(1/rho, 1/rho + s/nu0)
 *
 * whose sparsity pattern never changes (only the objective changes between
 * outer iterations, Section IV-A).  C > 0 makes the matrix quasi-definite,
 * so it has an LDL^T factorisation without pivoting for any symmetric
 * ordering (Section IV-B, last paragraph).  The library computes the
 * ordering and symbolic factorisation once (ncl_kkt_analyze), then per
 * iteration assembles K from the state (ncl_kkt_assemble), factors it
 * (ncl_kkt_factor) and solves (ncl_kkt_solve, ncl_kkt_solve_adjoint).
 *
 * Structure: K is block-arrowhead (Section II-B, eq. (scopf)): one block per
 * scenario k = 0 (base case) .. K (contingencies), coupled only through the
 * first-stage "border" variables u0 (pg, and with PV/PQ switching the PV
 * voltages vm0).  Blocks are factored independently, then the Schur
 * complement on the border.
 *
 * Layout (the order of every vector this library reads or writes):
 *   per block, primal then dual:
 *     primal: vm[nb], va[nb], qg[ng]; a single-block network adds pg[ng];
 *             with NCL_PVPQ the contingency blocks add nu_plus[ng],
 *             nu_minus[ng], s_up[ng], s_lo[ng], and the base block omits vm
 *             at generator buses (those voltages are the border vm0);
 *             with NCL_AGC the contingency blocks then add pgk[ng] (their
 *             own generation, which takes the place of pg in their P rows),
 *             pi_plus[ng], pi_minus[ng], sp_up[ng], sp_lo[ng] and one
 *             adjustment delta;
 *     dual:   P[nb], Q[nb], Ffrom[nl], Fto[nl]; with NCL_PVPQ the
 *             contingency blocks add LIN[ng], DUP[ng], DLO[ng], CUP[ng],
 *             CLO[ng] (eq. (pvpq): linear row, the two slack definitions and
 *             the two complementarity products); with NCL_AGC they then add
 *             ALIN[ng], ADUP[ng], ADLO[ng], ACUP[ng], ACLO[ng], the same five
 *             rows of eq. (droopmpec): pi_plus - pi_minus - pgk + pg +
 *             alpha_g delta, sp_up - (pmax - pgk), sp_lo - (pgk - pmin),
 *             pi_minus sp_up and pi_plus sp_lo;
 *   blocks 0..K in order, then the border pg[ng] (and vm0[ng] with NCL_PVPQ).
 *   With NCL_SCREEN the blocks are the K contingencies alone, each with the
 *   contingency layout (pg and vm0 fixed, so neither a column nor a border).
 *
 * Conventions
 *   - Pointers named d* and the fields of ncl_kkt_point are DEVICE pointers;
 *     everything else is host memory.  The library copies what it needs from
 *     host arrays during the call; the caller keeps ownership of all memory
 *     it passes in, and the library never frees caller memory.
 *   - Device memory: the library performs no device allocation of its own.
 *     ncl_kkt_workspace_bytes reports how much it needs and the caller binds
 *     one buffer with ncl_kkt_bind_workspace (the Python binding uses a torch
 *     tensor).  The buffer must stay valid until destroy or a new bind.
 *   - `stream` is a hipStream_t (0 = the null stream).  Compute calls are
 *     asynchronous on it; argument and state errors return immediately;
 *     numerical failures (zero, non-finite or wrong-sign pivot) are recorded
 *     on the device and reported by ncl_kkt_info.
 *   - A handle must not be used from two host threads at once, and calls on
 *     one handle must be ordered (one stream, or caller-side events).
 *     Distinct handles are independent.
 *   - Results are bitwise reproducible run to run: no floating-point atomics
 *     and fixed summation orders everywhere.
 */
#ifndef NCL_KKT_H
#define NCL_KKT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ncl_kkt ncl_kkt;

enum {
    NCL_OK = 0,
    NCL_ERR_ARG = -1,        /* bad argument (sizes, indices, null pointers, rho <= 0) */
    NCL_ERR_ALLOC = -2,      /* host allocation failed */
    NCL_ERR_HIP = -3,        /* a HIP runtime call failed */
    NCL_ERR_STATE = -4,      /* call out of order (no workspace, not factored, ...) */
    NCL_ERR_ZERO_PIVOT = -5, /* a pivot was exactly zero */
    NCL_ERR_INERTIA = -6,    /* a pivot had the wrong sign (primal must be >0, dual <0) */
    NCL_ERR_NONFINITE = -7,  /* a pivot was NaN or infinite */
    NCL_ERR_NOT_CONVERGED = -8 /* the dispatch map's Newton method ran out of steps */
};

#define NCL_MAX_BORDER 600   /* largest first-stage border (dense factor in local memory) */
#define NCL_PVPQ 1u          /* PV/PQ complementarity rows and the vm0 border (eq. (pvpq)) */
#define NCL_SCREEN 2u        /* contingency screening (eq. (screening)): the first-stage variables are
                                fixed, so the blocks are the K contingencies alone, with no base case
                                and no border; each block's KKT is that of its own feasibility problem */
#define NCL_AGC 4u           /* AGC droop recourse (eq. (agc) as its complementarity form (droopmpec))
                                in every contingency block; needs gen_alpha */

/* Network topology and constants (host arrays, copied during analyze).
 * Branch l joins buses br_from[l] < br_to[l] with series impedance
 * br_r[l] + j br_x[l] (no shunts, no taps); generator g sits at bus
 * gen_bus[g] (distinct buses) with cost gen_c2[g] * pg^2; contingency k+1
 * (k = 0..ncont-1) removes branch outage[k] (a non-bridge branch).
 * Branches must be sorted by (from, to) without duplicates.  gen_alpha[g]
 * is the AGC participation factor of generator g (read only with NCL_AGC,
 * which needs contingencies; finite values; NULL otherwise). */
typedef struct {
    int32_t nbus, nbranch, ngen, ncont;
    const int32_t *br_from, *br_to, *gen_bus, *outage;
    const double *br_r, *br_x, *gen_c2;
    uint32_t flags;
    const double *gen_alpha;
} ncl_network;

/* Options of the symbolic analysis (all zero / NULL: the defaults).
 *
 * Supernode amalgamation: a supernode absorbs its parent supernode when the
 * merged width is <= relax_maxw and explicit zeros * relax_zden <=
 * entries * relax_znum.  Defaults (zero here): 16, 1, 4.
 *
 * Ordering (Section IV-B, last paragraph: the regularisation block C makes
 * K quasi-definite, so every symmetric ordering has an LDL^T factorisation
 * with 1x1 pivots and no pivoting):
 *   NCL_ORDER_MD (0, default): exact minimum degree per block, ties to the
 *     smallest layout index, the border last;
 *   NCL_ORDER_USER: user_perm[N] (host, new -> layout index of the
 *     network, or of the pattern for ncl_kkt_analyze_pattern) gives the
 *     elimination order.  It must respect the block-arrowhead structure:
 *     every block's positions map onto that block's own columns, blocks
 *     that share a pattern template (every contingency block of a network;
 *     the base block too when it has no complementarity rows) use the same
 *     local order, and the border maps to itself in layout order (it is
 *     factored as a dense matrix).  NCL_ERR_ARG otherwise.  Within a block
 *     the library relabels the given order by the DFS postorder of its
 *     elimination forest (children in elimination order): the same
 *     elimination, so the fill and the pivots are those of the given order,
 *     only their positions move (ncl_kkt_symbolic reports the final perm).
 * For ncl_kkt_analyze_batch, user_perm of instance i indexes that
 * instance's own columns. */
enum { NCL_ORDER_MD = 0, NCL_ORDER_USER = 1 };
typedef struct {
    int32_t relax_maxw, relax_znum, relax_zden;
    int32_t ordering;
    const int32_t *user_perm;
} ncl_analyze_opts;

/* One primal-dual state, DEVICE arrays of length N in layout order.
 * z: primal values at primal positions and multipliers at dual positions
 *    (CUP/CLO rows hold the complementarity multiplier nu0).
 * sigma: the barrier diagonal Sigma at primal positions (W0^{-1} Xi etc.,
 *    must be > 0 unless the row's Hessian makes K11 definite); at CUP/CLO
 *    rows the slack s of W1 W2 e <= t; at any other dual row an extra
 *    diagonal omega >= 0 (an eliminated inequality slack, block C), so that
 *    the row's diagonal is -(1/rho + omega).
 * rho: augmented-Lagrangian penalty (> 0).
 * flags: NCL_NO_SHIFT assembles K without the diagonal-dominance shift
 *    delta (the exact Newton matrix, e.g. at a solution whose K11 is known
 *    to be positive definite on the relevant subspace); 0 otherwise. */
#define NCL_NO_SHIFT 1u
typedef struct {
    const double *z;
    const double *sigma;
    double rho;
    uint32_t flags;
} ncl_kkt_point;

/* Factorisation report (ncl_kkt_info).  npos/nneg/nzero count the signs of
 * D and nnonfinite its NaN or infinite pivots; first_bad is the first pivot
 * (factor order) that was zero, non-finite or of the wrong sign (-1 if
 * none); status is NCL_OK or the NCL_ERR_* of that pivot.
 * solvable = 1 when the solves may use the factors: no zero or non-finite
 * pivot and the inertia (npos, nneg) equal to (n, m) (the inertia a
 * quasi-definite K has, Section IV-B).  A factor with the right inertia but
 * individual pivots of the other sign (possible only when K11 is not
 * definite, e.g. the exact Newton matrix at a local minimum, whose reduced
 * Hessian is positive definite) reports NCL_ERR_INERTIA and stays
 * solvable; the inertia-correction loop of Section V-C acts on the counts. */
typedef struct {
    int64_t npos, nneg, nzero, first_bad;
    double min_absd, max_absd;
    int32_t status;
    int32_t solvable;
    int64_t nnonfinite;
} ncl_kkt_report;

/* Symbolic analysis of the KKT of a network (once per pattern: between NCL
 * outer iterations only the objective changes, Section IV-A, and inside an
 * outer iteration only the values, Section IV-B).  The block-arrowhead
 * structure is that of the SCOPF (Section II-B, eq. (scopf)): one block per
 * scenario coupled through the first-stage border.
 * Builds the union pattern of K (an outaged branch keeps explicit zeros,
 * so every contingency block has the same pattern), a minimum-degree
 * ordering per block with the border last (or the caller's, see
 * ncl_analyze_opts), the elimination tree, the column counts, the
 * supernode partition and all schedules.  Host only; no device memory is
 * touched.  opts may be NULL (defaults).
 * Returns NCL_ERR_ARG for out-of-range indices, unsorted or duplicate
 * branches, too many or bridge outages, and for a border of more than
 * NCL_MAX_BORDER variables (the dense border factor works on one compute
 * unit's local memory). */
int ncl_kkt_analyze(const ncl_network *net, const ncl_analyze_opts *opts, ncl_kkt **out);

/* Symbolic analysis of a user-given block-arrowhead pattern (no assembly;
 * values come through ncl_kkt_set_values).  colptr[N+1]/rowind: the lower
 * triangle (row >= column, diagonal included, rows sorted) in the caller's
 * order, blocks [block_off[b], block_off[b+1]) for b < nblk, border
 * [block_off[nblk], N).  No entry may couple two different blocks.
 * is_primal[N] gives the expected pivot sign (1 positive, 0 negative).
 * The border may hold at most NCL_MAX_BORDER columns. */
int ncl_kkt_analyze_pattern(int64_t N, int32_t nblk, const int64_t *block_off, const int64_t *colptr,
                            const int32_t *rowind, const uint8_t *is_primal,
                            const ncl_analyze_opts *opts, ncl_kkt **out);

/* Symbolic analysis of a batch of independent networks in one handle
 * (batched workloads: many scenarios or snapshots factored together).
 * Each network is analysed exactly as by ncl_kkt_analyze; the handle's
 * matrix is block diagonal over the instances, and every vector is the
 * instances' layout-order vectors concatenated in the order given (see
 * ncl_kkt_instance for each instance's first column).  Every launch of
 * assemble, factor and solve covers all instances at once; instance i's
 * results are bitwise equal to those of a handle holding network i alone.
 * opts: NULL with nopts = 0 (defaults), one set for all (nopts = 1), or one
 * per instance (nopts = count), e.g. supernode amalgamation widths chosen
 * per instance shape.  ncl_kkt_point.rho is shared by all instances.
 * Returns NCL_ERR_ARG on a bad network (as ncl_kkt_analyze) or count < 1. */
int ncl_kkt_analyze_batch(const ncl_network *nets, int32_t count, const ncl_analyze_opts *opts, int32_t nopts,
                          ncl_kkt **out);

/* Number of instances of a handle (1 unless made by ncl_kkt_analyze_batch). */
int ncl_kkt_instances(const ncl_kkt *h, int32_t *count);

/* Instance i: first global column col0, its size n (blocks then border),
 * its primal count, its block count and border size.  Any output may be
 * NULL.  NCL_ERR_ARG if i is out of range. */
int ncl_kkt_instance(const ncl_kkt *h, int32_t i, int64_t *col0, int64_t *n, int64_t *nprimal, int32_t *nblk,
                     int32_t *nbd);

/* Sizes: N, primal count, nnz of K's lower triangle, nnz of L's strict
 * lower triangle (exact pattern), number of supernodes, number of panel
 * row indices (length of srowind below). */
int ncl_kkt_dims(const ncl_kkt *h, int64_t *N, int64_t *nprimal, int64_t *nnzK, int64_t *nnzL,
                 int64_t *nsuper, int64_t *npanel);

/* Host copies of the symbolic result in factor order ("new" numbering).
 * perm[N]: new -> layout index.  etree[N]: parent (-1 for roots).
 * colcount[N]: nnz of each column of L including the diagonal.
 * super_ptr[nsuper+1]: first column of each supernode.
 * lcolptr[N+1], lrowind[nnzL]: strict-lower pattern of L, rows sorted.
 * srowptr[nsuper+1], srowind[npanel]: panel rows of each supernode (its
 * columns, then the sorted rows below it).  Any pointer may be NULL. */
int ncl_kkt_symbolic(const ncl_kkt *h, int32_t *perm, int32_t *etree, int64_t *colcount,
                     int64_t *super_ptr, int64_t *lcolptr, int32_t *lrowind, int64_t *srowptr,
                     int32_t *srowind);

/* Lower-triangle pattern of K in layout order (colptr[N+1], rowind[nnzK]),
 * the order of ncl_kkt_set_values' input. */
int ncl_kkt_pattern(const ncl_kkt *h, int64_t *colptr, int32_t *rowind);

/* Device bytes needed for solves of up to nrhs_max right-hand sides. */
int ncl_kkt_workspace_bytes(const ncl_kkt *h, int32_t nrhs_max, size_t *bytes);

/* Bind caller-owned device memory (>= the reported size, 256-byte aligned)
 * and upload the schedules on `stream`. */
int ncl_kkt_bind_workspace(ncl_kkt *h, void *dptr, size_t bytes, int32_t nrhs_max, void *stream);

/* Assemble K from a state (Section IV-B blocks A, B, C with the polar
 * power-flow Jacobian and Lagrangian Hessian; the per-row shift
 * delta_i = max(0, sum_{j!=i}|H_ij| - H_ii) keeps H + delta + Sigma
 * positive definite at non-optimal states).  Writes the lower CSC values
 * of K inside the workspace.  NCL_ERR_STATE if the handle came from
 * ncl_kkt_analyze_pattern. */
int ncl_kkt_assemble(ncl_kkt *h, const ncl_kkt_point *pt, void *stream);

/* Seam that bypasses assembly: dvals[nnzK] are the lower CSC values (in the
 * order of ncl_kkt_pattern), copied device-to-device into the workspace. */
int ncl_kkt_set_values(ncl_kkt *h, const double *dvals, void *stream);

/* Device copy of the current K values (lower CSC order) into dvals[nnzK]. */
int ncl_kkt_get_values(ncl_kkt *h, double *dvals, void *stream);

/* Pivot-free LDL^T of the current values (Section IV-B, last paragraph:
 * the regularisation block C makes K quasi-definite, so the 1x1 pivots of
 * any symmetric ordering exist; the paper's signed Cholesky): blocks in
 * parallel, then the fixed-order sum of their border Schur contributions
 * and the dense LDL^T of the border.  Asynchronous; pivot signs, zeros and
 * non-finite values are recorded on the device (see ncl_kkt_info).
 * NCL_ERR_STATE without a bound workspace or before any assemble /
 * set_values.  From the start of the call until it completes, the previous
 * factors are gone: solves in between return NCL_ERR_STATE. */
int ncl_kkt_factor(ncl_kkt *h, void *stream);

/* The two phases of ncl_kkt_factor, callable separately (same result):
 * factor_blocks factors every block and forms the border Schur products
 * sum_k K_bk K_kk^{-1} K_kb as partial tiles (tile pairs of the border,
 * slices of supernodes, chunks of 16 blocks); factor_border sums the
 * partials in a fixed order, subtracts them from K_bb and factors the
 * dense border.  factor_border returns NCL_ERR_STATE unless factor_blocks
 * ran since the last bind. */
int ncl_kkt_factor_blocks(ncl_kkt *h, void *stream);
int ncl_kkt_factor_border(ncl_kkt *h, void *stream);

/* Synchronises `stream` and reports the last factorisation: the inertia
 * that the inertia correction of Section V-C acts on, and whether the
 * factors may be solved with (ncl_kkt_report.solvable).  After a report
 * with solvable = 0, solve, solve_adjoint and refine return NCL_ERR_STATE
 * until the next factor.  (A solve issued before the report runs on the
 * device, which finds the same failure and fills x with NaN.) */
int ncl_kkt_info(ncl_kkt *h, ncl_kkt_report *rep, void *stream);

/* Device copies of the factors: lx[nnzL] on the exact pattern of
 * ncl_kkt_symbolic (strict lower part of unit-lower L) and d[N], both in
 * factor order. */
int ncl_kkt_get_factors(ncl_kkt *h, double *dlx, double *dd, void *stream);

/* Factor and solve in one call.  The blocks couple only through the
 * border (Section II-B, eq. (scopf)), so the forward substitution of the
 * blocks does not need the border's factor: the blocks are factored on
 * `stream`, then the border's Schur products, their sum and the dense
 * border factor run on a second stream that the library creates on first
 * use (default priority, on the device current then) while `stream` runs
 * the forward substitution of the blocks; `stream` then waits for the border
 * and finishes the solve (a border of fewer than 128 rows is factored in
 * line on `stream`).  Results equal those of ncl_kkt_factor followed
 * by ncl_kkt_solve bit for bit, ncl_kkt_info reports the same, and a
 * factorisation that may not be solved with gives NaN in dx.  Arguments and
 * errors as ncl_kkt_solve, except that the handle needs values, not factors
 * (NCL_ERR_STATE without them).  The second stream is joined back to
 * `stream` within the call, so a stream capture of the call is complete. */
int ncl_kkt_factor_solve(ncl_kkt *h, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream);

/* X = K^{-1} B for nrhs columns of length N in layout order, leading
 * dimension ld >= N (device): the Newton step of eq. (newtonsystem),
 * [dw; dy] for the right-hand side (r1, r2) the interior-point method sets
 * (Section IV-B).  Forward substitution by blocks, the border, D^{-1},
 * backward substitution.  dx may equal db.  nrhs <= the workspace's
 * nrhs_max.  NCL_ERR_STATE before the first factor, during one, or after a
 * factor that ncl_kkt_info reported not solvable; NCL_ERR_ARG for nrhs or
 * ld out of range. */
int ncl_kkt_solve(ncl_kkt *h, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream);

/* X = K^{-T} B on the stored factors (K is symmetric, so the same
 * triangular solves; bitwise equal to ncl_kkt_solve).  The entry used by
 * reverse-mode differentiation; it never refactors. */
int ncl_kkt_solve_adjoint(ncl_kkt *h, const double *db, double *dx, int32_t nrhs, int64_t ld,
                          void *stream);

/* Accuracy gate (the residual of eq. (newtonsystem)): for each of nrhs
 * columns (layout order, leading dimension ld, device) the normwise
 * backward error eta = ||b - Kx||_inf / (||K||_inf ||x||_inf + ||b||_inf)
 * and the componentwise one omega = max_i |b - Kx|_i / (|K||x| + |b|)_i
 * (0/0 counts 0), with K the current values (assembled or set), written to
 * derr[2 rhs] and derr[2 rhs + 1] (device doubles).  No host
 * synchronisation: the caller reads derr when it needs it.  A NaN in x or b
 * makes both NaN.  NCL_ERR_STATE without values; NCL_ERR_ARG for
 * ld < N or null pointers.  Uses the workspace's residual buffers, so calls
 * on one handle must not overlap. */
int ncl_kkt_backward_error(ncl_kkt *h, const double *db, const double *dx, int32_t nrhs, int64_t ld, double *derr,
                           void *stream);

/* One step of iterative refinement on the stored factors:
 * x += K^{-1} (b - K x) for each of nrhs columns (device, in place), with K
 * the current values (they must be the ones factored).  Errors as
 * ncl_kkt_solve. */
int ncl_kkt_refine(ncl_kkt *h, const double *db, double *dx, int32_t nrhs, int64_t ld, void *stream);

/* For callers that cannot allocate device memory or use a workspace's
 * staging (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): ncl_kkt_backward_error with its residual staging
 * (x, b and r transposed to the blocks' interleaved order, r in layout
 * order, per-workgroup partial maxima) in a device array the library holds
 * on each GPU it runs on, from module load until the process ends, instead
 * of in the bound workspace.  Same kernels, same results bit for bit.
 * Allocates nothing (no hipMalloc, hipFree or allocating library call).
 * The staging needs 3 * (N + 32) + N + 8 * (row wavefronts / 4 + border
 * rows / 4) doubles, about 4 N; above NCL_NOALLOC_MAX_DOUBLES (48 MiB, so N
 * up to about 1.5 million) the call returns NCL_ERR_ARG.  Every call on one
 * GPU shares that GPU's array and leaves its contents behind (nothing in it
 * needs to start at zero): calls that overlap on one GPU, from any handle
 * or stream, race.  Other errors as ncl_kkt_backward_error. */
#define NCL_NOALLOC_MAX_DOUBLES (6 * 1048576)
int ncl_kkt_backward_error_noalloc(ncl_kkt *h, const double *db, const double *dx, int32_t nrhs, int64_t ld,
                                   double *derr, void *stream);

void ncl_kkt_destroy(ncl_kkt *h);
const char *ncl_status_string(int status);

/* ---------------------------------------------------------------- dispatch map
 * The stationarity F(z; pd) = 0 of the NCL subproblem (Section III, fixed
 * rho, multiplier estimate 0, barrier parameter mu) of the corrective SCOPF
 * without PV/PQ rows: objective sum_g c2 pg^2 + log barriers of vm in
 * [vmin, vmax], qg in [-qmax, qmax], pg in [0, pmax] + (eps/2) va_ref^2 per
 * block (bus 0's angle), balance rows c(w; pd) with loads pd (P) and
 * qd_ratio * pd (Q) in every block, flow rows h <= smax2 with an eliminated
 * slack t = mu / y.  Its Jacobian is the KKT matrix assembled with
 * NCL_NO_SHIFT and the sigma this call returns.  Networks with NCL_PVPQ or
 * NCL_AGC are rejected. */
typedef struct {
    const double *pd;      /* DEVICE [nbus of the network] active loads */
    double qd_ratio;
    double mu, rho;
    double vmin, vmax, qmax, pmax, smax2, eps;
} ncl_nlp;

/* Layout kinds (HOST out, [N]): for each global column, 1 vm, 2 va, 3 qg,
 * 4 pg, 5 P balance row, 6 Q balance row, 7 flow row, 8..11 the
 * complementarity variables nu_plus, nu_minus, s_up, s_lo, 12..16 the rows
 * LIN, DUP, DLO, CUP, CLO, 17 the border vm0, and with NCL_AGC 18 pgk,
 * 19..22 pi_plus, pi_minus, sp_up, sp_lo, 23 delta, 24..28 the rows ALIN,
 * ADUP, ADLO, ACUP, ACLO. */
enum { NCL_L_OTHER = 0, NCL_L_VM, NCL_L_VA, NCL_L_QG, NCL_L_PG, NCL_L_ROWP, NCL_L_ROWQ, NCL_L_FLOW,
       NCL_L_NUP, NCL_L_NUM, NCL_L_SUP, NCL_L_SLO, NCL_L_LIN, NCL_L_DUP, NCL_L_DLO, NCL_L_CUP, NCL_L_CLO,
       NCL_L_VM0, NCL_L_PGK, NCL_L_PIP, NCL_L_PIM, NCL_L_SPU, NCL_L_SPL, NCL_L_DELTA, NCL_L_ALIN,
       NCL_L_ADUP, NCL_L_ADLO, NCL_L_ACUP, NCL_L_ACLO };
int ncl_kkt_layout_kinds(const ncl_kkt *h, uint8_t *kinds);

/* F (DEVICE [N]) = F(z; pd) and sigma (DEVICE [N]) = the barrier Hessian
 * (+ eps on reference angles) at primal rows, mu / y^2 at flow rows, 0 at
 * balance rows.  z, F and sigma in layout order; F and sigma must not
 * alias z.  Asynchronous on stream.  NCL_ERR_ARG for a pattern handle, a
 * batch of several networks or a network with PV/PQ rows; NCL_ERR_STATE if
 * no workspace is bound. */
int ncl_kkt_residual(ncl_kkt *h, const ncl_nlp *p, const double *z, double *F, double *sigma, void *stream);

/* Fraction-to-boundary step: *alpha (DEVICE, one double) = the largest
 * a <= 1 such that z + a dz keeps every barrier argument of the dispatch
 * map at least (1 - tau) of its current value (vm, qg, pg inside their
 * bounds, flow-row multipliers positive).  Asynchronous on stream. */
int ncl_kkt_max_step(ncl_kkt *h, const ncl_nlp *p, const double *z, const double *dz, double tau, double *alpha,
                     void *stream);

/* Newton solve of F(z; pd) = 0 for the dispatch map, every step of it in
 * the library's kernels (the host only orders them and reads scalars back):
 * per step the exact K at z (NCL_NO_SHIFT, sigma from ncl_kkt_residual),
 * factored; if its inertia is not (n, m) (zero or non-finite pivots, or the
 * wrong counts), dw is added on the primal diagonal, from a third of the
 * last accepted dw (or 1e-4) growing x8 until it is (the inertia correction
 * of Section V-C, as a primal shift); dz = -K^{-1} F; the fraction-to-
 * boundary step (tau 0.995) and backtracking on |F|_2 (sufficient decrease
 * 1e-4 alpha, halving down to 1e-10).  Converged when every |dz_i| <=
 * step_tol (1 + |z_i|) (1e-6 at the continuation's intermediate barrier
 * values), the last step then taken when feasible; also when backtracking
 * stalls below 1e-10 with every |dz_i| <= floor_tol (1 + |z_i|) (|F| at its
 * rounding floor).  With from_default the start is vm = 1, pg = pmax / 2,
 * flow-row multipliers mu / smax2, and the barrier is continued through 10,
 * 3, 1, 0.3, 0.1, 0.03 (those above mu) down to mu; else the solve starts
 * from dz_state at mu.  On return the exact K at the solution is factored
 * (for ncl_kkt_dispatch_vjp).  dz_state: DEVICE [N] state (in: start
 * unless from_default; out: solution).  dwork: DEVICE, 7 N + 8 doubles.
 * Synchronises the stream at every step.  NCL_ERR_NOT_CONVERGED after
 * maxit steps at one barrier value; NCL_ERR_INERTIA if no shift up to 1e12
 * gives the inertia, or the exact K at the solution lacks it. */
typedef struct {
    double step_tol;         /* e.g. 1e-10 */
    double floor_tol;        /* e.g. 1e-6 */
    int32_t maxit;           /* Newton steps per barrier value */
    int32_t from_default;    /* 1: default start and barrier continuation */
    int32_t iterations;      /* out: Newton steps taken */
    int32_t pad;
    double dw_last;          /* in/out: the last accepted inertia shift (0 at first) */
} ncl_newton_opts;
int ncl_kkt_dispatch_newton(ncl_kkt *h, const ncl_nlp *p, double *dz_state, double *dwork, ncl_newton_opts *opts,
                            void *stream);

/* Outputs of the map at state dz: *dphi (DEVICE, one double) = sum_g c2_g
 * pg_g^2 (generators in order) and dpg (DEVICE [ng], may be NULL) = pg. */
int ncl_kkt_dispatch_outputs(ncl_kkt *h, const double *dz, double *dphi, double *dpg, void *stream);

/* Vector-Jacobian product of the map at its solution dz: with g the
 * gradient of gphi phi + gpg . pg in z, a = K^{-T} g by one
 * ncl_kkt_solve_adjoint on the stored factors (those ncl_kkt_dispatch_newton
 * left), and dgpd[i] = -(sum over blocks of a at bus i's P row + qd_ratio
 * times the same sum at its Q row) (implicit function theorem: loads enter
 * F only through the balance rows).  dgphi: DEVICE one double; dgpg: DEVICE
 * [ng] or NULL (zero); dgpd: DEVICE [nbus]; dwork: DEVICE 2 N doubles.
 * NCL_ERR_STATE without usable factors. */
int ncl_kkt_dispatch_vjp(ncl_kkt *h, const ncl_nlp *p, const double *dz, const double *dgphi, const double *dgpg,
                         double *dgpd, double *dwork, void *stream);

/* ---------------------------------------------------------------- IPM step
 * One Newton direction of the primal-dual interior-point method that
 * solves the NCL subproblem (Section IV-A, eq. (nclsubpb); its KKT
 * conditions eq. (kktncl) with the complementarity products perturbed to
 * mu, Section IV-B) of the corrective SCOPF, PV/PQ rows included:
 *
 *   min  phi(w) + lam_n' r + nu0_n' t + rho/2 (|r|^2 + |t|^2)
 *   s.t. c_E(w) - r = 0            balance, LIN, DUP, DLO rows
 *        c_I(w) + s - r = 0, s >= 0  flow rows (h <= smax2) and CUP/CLO rows
 *        lo <= w <= hi             (finite bounds only)
 *
 * phi = sum_g c2_g pg_g^2 + (eps/2) sum over blocks of bus 0's angle^2.
 * c: P_i = sum of branch-end P leaving bus i - pg at i + pd_i; Q_i likewise
 * with qg and qd_ratio pd_i; flow rows P^2 + Q^2 - smax2 at both ends;
 * LIN = nu_plus - nu_minus - vm_i + vm0_g, DUP = s_up - (qmax - qg),
 * DLO = s_lo - (qg + qmax), CUP = nu_minus s_up, CLO = nu_plus s_lo; with
 * NCL_AGC the contingency blocks' P rows take their own pgk, and
 * ALIN = pi_plus - pi_minus - pgk + pg + alpha_g delta,
 * ADUP = sp_up - (pmax - pgk), ADLO = sp_lo - pgk (pmin = 0),
 * ACUP = pi_minus sp_up, ACLO = pi_plus sp_lo, ACUP/ACLO inequality rows
 * like CUP/CLO.  The
 * slack of an inequality row has the row multiplier as its bound
 * multiplier (S V0 = mu e for the complementarity rows; the flow rows take
 * the same form).  Unknowns: w and y (the state vector z), the
 * regularisation rt (r on the rows of c, t on CUP/CLO), the slacks s and
 * the bound multipliers zl, zu.  Eliminating rt, s, zl, zu from the Newton
 * equations leaves eq. (newtonsystem), K [dw; dy] = [r1; r2], where K is
 * the assembled matrix (NCL_NO_SHIFT) at
 *   sigma = zl/(w - lo) + zu/(hi - w) (+ eps at the reference angles) on
 *   primal positions, s on CUP/CLO (ACUP/ACLO) rows, s/y on flow rows, 0
 *   elsewhere,
 * and
 *   r1 = -(grad phi + J' y) + mu/(w - lo) - mu/(hi - w)
 *   r2 = -c(w) + (y - y_n)/rho - [inequality row] mu/y.
 * The eliminated directions follow from (dw, dy); their signs are those of
 * the linearisation (the printed recovery formulas of Section IV-B carry
 * the opposite sign on the mu terms and on d lam):
 *   d rt = (dy + y - y_n - rho rt)/rho                (dual rows)
 *   d s  = mu/y - s - (s/y) dy                         (inequality rows)
 *   d zl = (mu - (w - lo) zl - zl dw)/(w - lo)         (finite lo)
 *   d zu = (mu - (hi - w) zu + zu dw)/(hi - w)         (finite hi).
 * An NCL_SCREEN network (eq. (screening)) takes pg0 and vm0 as data: its
 * blocks are the contingencies' problems at that first stage, and phi
 * keeps only the angle term.  Handles of one network only: batches of
 * several networks and pattern handles are rejected (NCL_ERR_ARG), and so
 * are qmax, pmax or smax2 <= 0 and a screening network without pg0 (or,
 * with NCL_PVPQ, vm0). */
typedef struct {
    const double *pd;        /* DEVICE [nbus] active loads */
    const double *lo, *hi;   /* DEVICE [N] bounds at primal positions (-inf/+inf: none; dual rows ignored) */
    const double *y_n;       /* DEVICE [N] multiplier estimates lam_n, nu0_n at dual rows */
    double qd_ratio, qmax, pmax, smax2, eps;
    double mu, rho;
    const double *pg0;       /* DEVICE [ngen] fixed first-stage pg (NCL_SCREEN networks; NULL otherwise) */
    const double *vm0;       /* DEVICE [ngen] fixed first-stage PV voltages (NCL_SCREEN with NCL_PVPQ) */
} ncl_ipm_problem;

/* A primal-dual point, DEVICE [N] each, layout order (entries outside the
 * positions named are not read). */
typedef struct {
    const double *z;         /* w at primal positions, y at dual rows (inequality rows: y > 0) */
    const double *rt;        /* dual rows */
    const double *s;         /* inequality rows (s > 0) */
    const double *zl, *zu;   /* primal positions with a finite lo, resp. hi */
} ncl_ipm_state;

/* A direction, DEVICE [N] each, written at every position (zero where the
 * unknown does not exist). */
typedef struct {
    double *dz;              /* (dw, dy) */
    double *drt, *ds, *dzl, *dzu;
} ncl_ipm_direction;

/* sigma (DEVICE out [N]) of the Newton matrix at the point (see above).
 * Asynchronous. */
int ncl_kkt_ipm_sigma(ncl_kkt *h, const ncl_ipm_problem *p, const ncl_ipm_state *s, double *dsigma, void *stream);

/* The reduced right-hand side (r1, r2) (DEVICE out [N]).  J' y is taken
 * from the K values the handle holds, which must have been assembled at
 * the same z (any sigma, any diagonal shift: only the Jacobian blocks are
 * read).  dwork: DEVICE 2 N doubles.  NCL_ERR_STATE without values.
 * Asynchronous. */
int ncl_kkt_ipm_rhs(ncl_kkt *h, const ncl_ipm_problem *p, const ncl_ipm_state *s, double *drhs, double *dwork,
                    void *stream);

/* The eliminated directions from ddz = (dw, dy): writes d->drt, d->ds,
 * d->dzl, d->dzu (d->dz is not touched).  Asynchronous. */
int ncl_kkt_ipm_recover(ncl_kkt *h, const ncl_ipm_problem *p, const ncl_ipm_state *s, const double *ddz,
                        const ncl_ipm_direction *d, void *stream);

/* Inertia correction (Section V-C: the Newton matrix must have n positive
 * and m negative eigenvalues; when it does not, a primal shift is added and
 * the matrix factored again): assembles K at (dz, dsigma) with
 * NCL_NO_SHIFT and factors it; while its inertia is not (n, m) (or a pivot
 * is zero or not finite) it adds dw to sigma on the primal positions and
 * assembles and factors again, dw taking 0, then dw_last/3 (1e-4 if
 * dw_last is 0), growing x8 below 1e12.  On success the factors of the
 * accepted matrix are held (solvable), o->dw_last is the accepted shift
 * (0 when the exact matrix had the inertia) and o->nfactor the number of
 * factorisations.  dwork: DEVICE N doubles (the shifted sigma).
 * Synchronises the stream after every factorisation.  NCL_ERR_INERTIA when
 * no shift below 1e12 gives the inertia. */
typedef struct {
    double dw_last;          /* in: the last accepted shift (0 at the first step); out: this one */
    int32_t nfactor;         /* out: factorisations made */
    int32_t pad;
} ncl_inertia_opts;
int ncl_kkt_factor_inertia(ncl_kkt *h, const double *dz, const double *dsigma, double rho, ncl_inertia_opts *o,
                           double *dwork, void *stream);

/* The whole Newton direction: sigma, the inertia-corrected factorisation,
 * the right-hand side, one solve and the recovery, all on the device (the
 * host reads the inertia reports).  rho is p->rho.  dwork: DEVICE 3 N
 * doubles.  Errors as ncl_kkt_factor_inertia. */
int ncl_kkt_ipm_step(ncl_kkt *h, const ncl_ipm_problem *p, const ncl_ipm_state *s, const ncl_ipm_direction *d,
                     ncl_inertia_opts *o, double *dwork, void *stream);

/* ---------------------------------------------------------------- NCL solve
 * The NCL method end to end (Section IV-A): outer iterations update the
 * penalty rho and the multiplier estimates y_n from the solution of the
 * subproblem eq. (nclsubpb), which inner iterations solve with the
 * primal-dual IPM above, warm-started from the previous point.  Section V
 * fixes tol = 1e-6 and the smallest barrier parameter 1e-7; the paper
 * defers the update rules, and these are the library's:
 *   outer: solve the subproblem; r_inf = max |rt| over the dual rows;
 *     r_inf <= tol: converged; r_inf <= eta: y_n = y at the dual rows (the
 *     first-order update y_n + rho r) and eta = max(eta / eta_shrink, tol);
 *     otherwise rho = min(rho_grow rho, rho_max); the next subproblem
 *     starts at mu_warm (the first at mu0);
 *   inner: E0 = max |G| at mu = 0 (G the barrier KKT residual of
 *     ncl_kkt_ipm_step's unknowns, largest component magnitude); stop at
 *     E0 <= tol; while max |G| at mu <= kappa_eps mu and mu > mu_min, mu =
 *     max(mu_min, min(kappa_mu mu, mu^theta_mu)); an inertia-corrected
 *     Newton direction (ncl_kkt_ipm_step); fraction to the boundary with
 *     tau = max(tau_min, 1 - mu): alpha_p keeps w within its bounds and the
 *     slacks s, alpha_d keeps zl, zu and y at inequality rows, each above
 *     (1 - tau) of its value; w, y at equality rows, rt and s move by
 *     alpha_p, zl, zu and y at inequality rows by alpha_d.
 * p: the subproblem data as for ncl_kkt_ipm_step; p->rho is the first
 * penalty; p->y_n and p->mu are not read.  s: DEVICE [N] arrays, in: a
 * strictly interior start (w strictly within its finite bounds with
 * positive zl, zu there; s and y positive at inequality rows; everything
 * finite; else NCL_ERR_ARG before any iteration) and the first y_n; out:
 * the last iterate and y_n.  dwork: DEVICE 17 N + 64 doubles.  Synchronises the stream several
 * times per inner iteration (it reads the inertia, the error norms and the
 * step lengths).  Returns NCL_OK with rep->status 0 (converged), 1 (outer
 * limit) or 2 (inner limit); numerical failures of a step as
 * ncl_kkt_ipm_step, with rep->status 3 and the counts so far. */
typedef struct {
    double tol, mu_min;                 /* 1e-6, 1e-7 */
    double mu0, mu_warm;                /* 0.1, 1e-5 */
    double kappa_eps, kappa_mu, theta_mu, tau_min;   /* 10, 0.2, 1.5, 0.99 */
    double eta0, eta_shrink;            /* 1e-2, 10 */
    double rho_grow, rho_max;           /* 10, 1e12 */
    int32_t max_inner, max_outer;       /* per subproblem 300, 30 */
    /* optional iteration log (HOST, may be NULL): record t < trace_len of
     * inner iteration t (counted over all subproblems) holds NCL_TRACE_W
     * doubles: outer index, mu, E0 and max |G| at mu before the step, the
     * accepted shift, the factorisations, alpha_p, alpha_d, rho. */
    double *trace;
    int32_t trace_len, pad;
} ncl_solve_opts;
#define NCL_TRACE_W 9
typedef struct {
    int32_t status, outer, inner, factorizations;
    double rho, mu, r_inf, kkt_err;     /* at the last iterate (kkt_err = E0) */
} ncl_solve_report;
typedef struct {
    double *z, *rt, *s, *zl, *zu, *y_n;
} ncl_solve_state;
int ncl_kkt_ncl_solve(ncl_kkt *h, const ncl_ipm_problem *p, const ncl_solve_state *s, const ncl_solve_opts *o,
                      ncl_solve_report *rep, double *dwork, void *stream);

/* ---------------------------------------------------------------- measurement
 * Kernel kinds: every launch of the library runs exactly one kernel of one
 * of these kinds.  A "step" below is one assemble, one factor and one solve
 * with one right-hand side. */
enum {
    NCL_K_ASSEMBLE = 0,     /* k_assemble */
    NCL_K_VALUES,           /* k_values (set/get values; not part of a step) */
    NCL_K_FAC_GATHER,       /* k_fac_gather: panel entries minus descendant updates, one launch per level */
    NCL_K_FAC_DIAG,         /* k_fac_diag: LDL^T of diagonal blocks, and the pivots of width-1 supernodes, per level */
    NCL_K_FAC_ROWS,         /* k_fac_rows: off-diagonal rows of supernodes 2 or more wide, per level */
    NCL_K_BORDER_SCHUR,     /* k_border_schur: border Schur products on FP64 MFMA, partial tiles */
    NCL_K_BORDER_SUM,       /* k_border_sum: fixed-order sum of the partial tiles into the border matrix */
    NCL_K_BORDER_FACTOR,    /* k_border_factor (borders up to 216 rows, in registers) and k_border_step (larger, one launch per 32-column block): dense border LDL^T */
    NCL_K_STATUS_INIT,      /* k_status_init */
    NCL_K_STATUS,           /* k_status: pivot signs and magnitudes */
    NCL_K_SOL_LOAD,         /* k_sol_load */
    NCL_K_SOL_FWD_GATHER,   /* k_sol_fwd_gather: forward gathers of one level's diagonal rows */
    NCL_K_SOL_FWD_DIAG,     /* k_sol_fwd_diag: unit lower diagonal blocks of one level's wide supernodes */
    NCL_K_SOL_BPART,        /* k_sol_bpart */
    NCL_K_SOL_BORDER,       /* k_sol_border */
    NCL_K_SOL_BWD_BORDER,   /* k_sol_bwd_border: D^-1 and the border rows' part of the backward sums, every column */
    NCL_K_SOL_BWD,          /* k_sol_bwd: backward substitution of one level's supernodes (block rows, diagonal block) */
    NCL_K_SOL_STORE,        /* k_sol_store */
    NCL_K_RESIDUAL,         /* k_residual (dispatch map; not part of a step) */
    NCL_K_MAX_STEP,         /* k_max_step (dispatch map; not part of a step) */
    NCL_K_INTERLEAVE,       /* k_interleave: the state transposed to the blocks' interleaved order (assembly) */
    NCL_K_BERR_ROWS,        /* k_berr_rows: residual of the block rows (backward error, refinement) */
    NCL_K_BERR_BORDER,      /* k_berr_border: residual of the border rows */
    NCL_K_BERR_FINAL,       /* k_berr_final: eta and omega from the partial maxima */
    NCL_K_COUNT
};

/* Device kernel name of a kind ("k_fac_gather", ...), or NULL. */
const char *ncl_kernel_name(int kind);

/* Launches per step and algorithmic HBM bytes per step of a kernel kind:
 * every distinct array element a launch must read or write counted once
 * per launch (8 bytes per double; schedule tables not counted), summed over
 * the step's launches.  Host only. */
int ncl_kkt_kernel_model(const ncl_kkt *h, int32_t kind, int64_t *launches, int64_t *bytes);

/* Bracket every later launch of one kernel kind with a pair of HIP events
 * on the launch stream (kind = -1: stop).  Resets the accumulated record and
 * the stride to 1.  Launches of other kinds are not touched. */
int ncl_kkt_profile(ncl_kkt *h, int32_t kind);

/* Bracket only every stride-th launch of the profiled kind (counted from
 * the next launch; stride >= 1, else NCL_ERR_ARG).  A stride coprime with
 * the kind's launches per step samples every level evenly over that many
 * steps while adding fewer event records to the stream. */
int ncl_kkt_profile_stride(ncl_kkt *h, int32_t stride);

/* Streaming copy ddst[i] = dsrc[i], i < n, on the device (measurement: the
 * bandwidth a plain streaming kernel reaches, against which the path's
 * kernels are compared).  n even, both pointers 16-byte aligned, ranges
 * not overlapping; else NCL_ERR_ARG.  Asynchronous on `stream`. */
int ncl_stream_copy(const double *dsrc, double *ddst, int64_t n, void *stream);

/* Number of bracketed launches since ncl_kkt_profile and the sum of their
 * event-measured durations in milliseconds (waits for the last event). */
int ncl_kkt_profile_read(ncl_kkt *h, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* NCL_KKT_H */
