// Internal structures of libnclkkt: host-side symbolic data, schedules and
// the plain structs that carry device tables into the kernels.
//
// Storage: blocks that share a template (all contingency blocks of a
// network do) are processed together, one block per lane of a wavefront.
// Every per-block numeric array of a template is therefore stored
// interleaved: element e of the template's block number bl (its position in
// the template's block list) lives at base + e * nb + bl, so that the 64
// lanes of a wavefront touch 64 consecutive doubles.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ncl_kkt.h"

namespace ncl {

constexpr int kMaxW = 32;            // widest supernode
constexpr int kNarrowW = 8;          // diagonal blocks up to this width are factored one block per lane
constexpr int32_t kNarrowFlag = 0x40000000;   // marks such a supernode in the diagonal-block work list
constexpr int32_t kPivotFlag = 0x20000000;    // marks a width-1 supernode there (its pivot and column)
constexpr int32_t kBorderFlag = int32_t(1u << 30);   // slot refers to the border K_bb pattern
// A supernode of a solve level is "wide" (a workgroup of four wavefronts
// shares it) when it is wider than kNarrowW or has more than kSolWideRows
// rows below its diagonal block; otherwise one wavefront takes it.
constexpr int kSolWideRows = 24;
constexpr int32_t kWideFlag = 0x40000000;     // marks a wide supernode in the solve work lists
constexpr int kSolBorderWideRows = 32;        // a border column this long takes a workgroup

// ---------------------------------------------------------------- device tables

// One descendant supernode d's contribution to one entry (row, column c) of a
// panel: sum_k L_d[row, k] d_k L_d[c, k] (host-side; flattened into Terms).
struct CItem {
    int32_t ioff;    // panel element of L_d[row, 0] (template-relative)
    int32_t coff;    // panel element of L_d[c, 0]
    int32_t dcol;    // first column of d (block-local factor numbering)
    int32_t meta;    // ld (16 bits) | wd << 16
};

// Border Schur products on the matrix cores: the border matrix is cut into
// tiles of kMT rows; for a pair of tiles (I >= J) the products U[i, k] L[j, k]
// over every supernode holding rows of both tiles, its columns k and the
// blocks are summed with FP64 MFMA (16 x 16 outputs, 4 products a lane
// group per instruction).  An item is one supernode of one template: its
// panel (first element, rows, columns) and the panel row of each tile row
// it holds (-1 where it holds none).  A wavefront takes a slice of one
// pair's items (of one template) for one chunk of kMC blocks, about
// kMSlice instructions, and writes its own partial tile.
constexpr int kMT = 16;
constexpr int kMC = 16;
constexpr int kMSlice = 128;
constexpr int kMItemCost = 8;      // slicing cost of an item beyond its instructions (its dependent loads)
struct MItem {
    int32_t tmpl, poff, r, w;
    int16_t ri[kMT], rj[kMT];
};
struct MDesc {
    int32_t pair, chunk, ib, ie;   // tile pair, block chunk, item range
};
// transposes between layout order and the interleaved order move tiles of
// kTileJ columns x kTileB blocks
constexpr int kTileJ = 16;
constexpr int kTileB = 64;

// One product of an update sum: L[a] * d[k] * L[c] (factor, border Schur) or
// L[a] * y[k] (solves), with a, c panel elements and k a column, all
// template-relative.  Each entry's terms are contiguous, so that a kernel can
// keep many independent loads in flight.
struct Term {
    int32_t a, c, k, pad;
};

// A unit of work of one launch: template (high 16 bits) and block group
// (low 16 bits), and the task / supernode / entry index within the template.
struct Work {
    int32_t tg;
    int32_t k;
};

// Assembly slot indices (positions in the template CSC, or kBorderFlag|pos in K_bb, or -1).
enum BusSlot { BS_VMVM, BS_VAVA, BS_VMVA, BS_PVM, BS_PVA, BS_QVM, BS_QVA, BS_PP, BS_QQ, BS_N };
enum BranchSlot {
    LS_VMVM, LS_VMVA, LS_VAVM, LS_VAVA,                     // (from var, to var) Hessian couplings
    LS_PF_VMT, LS_PF_VAT, LS_QF_VMT, LS_QF_VAT,             // from-bus rows x to-bus vars
    LS_PT_VMF, LS_PT_VAF, LS_QT_VMF, LS_QT_VAF,             // to-bus rows x from-bus vars
    LS_FF_VMF, LS_FF_VMT, LS_FF_VAF, LS_FF_VAT,             // flow row at the from end
    LS_FT_VMF, LS_FT_VMT, LS_FT_VAF, LS_FT_VAT,             // flow row at the to end
    LS_FFFF, LS_FTFT, LS_N
};
enum GenSlot {
    GS_PPG, GS_QQG, GS_QGQG, GS_PGPG,
    GS_LIN_NUP, GS_LIN_NUM, GS_LIN_VM, GS_LIN_VM0, GS_DUP_SUP, GS_DUP_QG, GS_DLO_SLO, GS_DLO_QG,
    GS_CUP_NUM, GS_CUP_SUP, GS_CLO_NUP, GS_CLO_SLO, GS_H_NUM_SUP, GS_H_NUP_SLO,
    GS_NUPNUP, GS_NUMNUM, GS_SUPSUP, GS_SLOSLO, GS_LL, GS_UU, GS_DD, GS_CUCU, GS_CLCL,
    // AGC droop rows (eq. droopmpec): ALIN x (pi+, pi-, pgk, pg0, delta), the
    // slack rows, the complementarity products and their nu0 pairs, diagonals
    GS_ALIN_PIP, GS_ALIN_PIM, GS_ALIN_PGK, GS_ALIN_PG0, GS_ALIN_DEL, GS_ADUP_SPU, GS_ADUP_PGK,
    GS_ADLO_SPL, GS_ADLO_PGK, GS_ACUP_PIM, GS_ACUP_SPU, GS_ACLO_PIP, GS_ACLO_SPL, GS_H_PIM_SPU, GS_H_PIP_SPL,
    GS_PIPPIP, GS_PIMPIM, GS_SPUSPU, GS_SPLSPL, GS_PGKPGK, GS_AL, GS_AU, GS_AD, GS_ACUACU, GS_ACLACL,
    GS_DELDEL,                     // the block's delta diagonal (generator 0 only)
    GS_N
};
// State index tables per bus / generator: layout-local positions (n + b for border refs).
enum BusIdx { BI_VM, BI_VA, BI_P, BI_Q, BI_N };
// With AGC rows GI_PG is the block's own generation pgk and GI_PG0 the
// first-stage pg (or -1 when it is fixed).
enum GenIdx { GI_BUS, GI_QG, GI_PG, GI_NUP, GI_NUM, GI_SUP, GI_SLO, GI_LIN, GI_DUP, GI_DLO, GI_CUP, GI_CLO, GI_VM0,
              GI_PIP, GI_PIM, GI_SPU, GI_SPL, GI_ALIN, GI_ADUP, GI_ADLO, GI_ACUP, GI_ACLO, GI_DELTA, GI_PG0, GI_N };

struct TemplDev {
    int32_t n, nsup, nblk, nbd;     // columns, supernodes, blocks using the template, its instance's border size
    int64_t kbase;                 // interleaved K values (nnz * nblk)
    int64_t lbase;                 // interleaved panels (panel_size * nblk)
    int64_t dbase;                 // interleaved pivots and solve vectors (n * nblk)
    int32_t nnz;                   // K entries of one block
    int32_t pvpq_rows;             // this template has the complementarity rows
    int32_t has_pg_local;          // single-block network: pg inside the block
    int32_t agc_rows;              // this template has the AGC droop rows
    int32_t inst;                  // instance (network) the template belongs to
    int32_t nbus, ngen;            // network sizes (assembly threads per block)
    int64_t abase;                 // first residual thread of the template
    int64_t awbase;                // first assembly thread of the template (wavefront-aligned)
    int64_t tile0;                 // first transpose tile of the template (kTileJ columns x kTileB blocks)
    int64_t bd0;                   // the instance's border pivots / solution at dint + bd0
    const double *br_r, *br_x;     // the instance's branch data
    const double *gen_c2;
    const double *gen_alpha;       // AGC participation factors (zeros without AGC rows)
    const int32_t *blocks;         // [nblk] global block ids
    // supernodes (block-local factor numbering; border rows are n + b)
    const int32_t *sup_first;      // [nsup+1]
    const int32_t *sup_rowptr;     // [nsup+1]
    const int32_t *sup_rows;
    const int32_t *panel_off;      // [nsup+1]
    // row tasks: (supernode, panel row); entries of a task are its w columns
    const int32_t *task_s;
    const int32_t *task_p;
    const int32_t *task_cbase;     // [ntask+1] first entry of each task
    const int32_t *ent_kpos;       // [nent] K value of the entry or -1
    const int32_t *ent_out;        // [nent] panel element of the entry
    const int32_t *ent_tptr;       // [nent+1] update terms of each entry
    const Term *terms;
    // border rows: terms L[b, k] y_k of the border right-hand side
    const int32_t *bterm_ptr;      // [nbd+1]
    const Term *bterms;
    // backward solve: a panel's block rows are its first sup_rnb[s] rows,
    // its border rows the rest
    const int32_t *sup_rnb;        // [nsup]
    const int32_t *col_sup;        // [n] supernode of each column
    // assembly
    const int32_t *bus_idx;        // [nb][BI_N]
    const int32_t *bus_slot;       // [nb][BS_N]
    const int32_t *bus_adj_ptr;    // [nb+1]
    const int32_t *bus_adj;        // branch l (to-end if negative: ~l)
    const int32_t *br_slot;        // [nl][LS_N]
    const int32_t *br_idx;         // [nl][4]: row Ff, row Ft, from bus, to bus
    const int32_t *gen_idx;        // [ng][GI_N]
    const int32_t *gen_slot;       // [ng][GS_N]
    const int32_t *perm;           // [n] factor order -> layout-local
    const int32_t *iperm;          // [n] layout-local -> factor order
    const uint8_t *col_primal;     // [n] expected pivot sign (1: positive) in factor order
    const int32_t *bus_gen;        // [nb] generator at the bus or -1
    const uint8_t *lkind;          // [n] layout-local kind (LK_*), for the dispatch map
    // residual rows (backward error and refinement)
    const int32_t *rr_ptr;         // [n+1]
    const int32_t *rr_ent;         // pairs (K value, column; n + b for border columns)
    const int32_t *rb_ptr;         // [nbd+1]
    const int32_t *rb_ent;         // pairs (K value, block column) of border row b
    int64_t rwbase;                // first residual-row wavefront of the template
};

// Layout-local kinds used by the dispatch-map and IPM kernels (bounds and
// rows); the codes are those of NCL_L_* in the public header.
enum LocalKind : uint8_t {
    LK_OTHER = 0, LK_VM, LK_VA, LK_QG, LK_PG, LK_ROWP, LK_ROWQ, LK_FLOW,
    LK_NUP, LK_NUM, LK_SUP, LK_SLO, LK_LIN, LK_DUP, LK_DLO, LK_CUP, LK_CLO, LK_VM0,
    LK_PGK, LK_PIP, LK_PIM, LK_SPU, LK_SPL, LK_DELTA, LK_ALIN, LK_ADUP, LK_ADLO, LK_ACUP, LK_ACLO
};
inline constexpr bool lk_primal(int k) {
    return (k >= LK_VM && k <= LK_PG) || (k >= LK_NUP && k <= LK_SLO) || (k >= LK_VM0 && k <= LK_DELTA);
}

// Per-instance (per-network) border data of a batch.
struct InstDev {
    int32_t nbd, nblk, blk0, ng;   // border size, blocks, first block, generators
    int64_t bstart;                // first global column of the border
    int64_t kbb0;                  // K_bb values at kval[kint + kbb0 ...]
    int64_t sbb0;                  // packed border matrix / factor at sbb[sbb0 ...]
    int64_t bd0;                   // border pivots at dval[dint + bd0 ...]
    int64_t sp0;                   // border Schur partial tiles at spart[sp0 + slice * kMT * kMT]
    int64_t mw0;                   // first border Schur wavefront (one per slice)
    int64_t pe0;                   // first thread of the partial-tile sum (one per tile-pair entry)
    int32_t npair, pad_m;
    const int32_t *mdesc_ptr;      // [npair + 1] slices of each tile pair
    const int32_t *bperm;          // [nbd] border row at each tile position
    const MDesc *mdesc;            // the slices, pair-major
    const MItem *mitems;
    int64_t cp0;                   // border right-hand-side partials at cpart[cp0 + b * nblk + block]
    int64_t npk0;                  // first packed border entry (all instances together)
    int64_t gp0;                   // first border-pg assembly thread
    int64_t kcsc_border;           // first public CSC value of the border
    int64_t nbb;                   // K_bb values
    const int32_t *kbb_pos;        // [nbd*nbd]
    const int32_t *border_pg;      // [ng]
    const double *gen_c2;          // [ng]
    const int32_t *kbr_ptr;        // [nbd+1] full symmetric rows of K_bb
    const int32_t *kbr_ent;        // pairs (K_bb value, border column)
    int32_t t0, nt;                // the instance's templates
};

struct BlockDev {
    int32_t tmpl;
    int32_t bl;                    // position in the template's block list
    int32_t outage;                // outaged branch or -1
    int32_t pad;
    int64_t col0;                  // first global column (layout order)
    int64_t kcsc;                  // first K value of the block in the public CSC order
};

// ---------------------------------------------------------------- host symbolic

struct Template {
    int inst = 0;                  // instance (network) of the template
    int n = 0;                     // block columns
    int nprim = 0;
    bool pvpq_rows = false;
    bool pg_local = false;
    bool agc_rows = false;
    std::vector<int32_t> blocks;   // global ids of the blocks using this template
    // model tables (layout-local; border refs n + b)
    std::vector<int32_t> bus_idx, bus_slot, bus_adj_ptr, bus_adj, br_slot, br_idx, gen_idx, gen_slot, bus_gen;
    std::vector<uint8_t> lkind;
    // lower CSC pattern in layout-local numbering (rows may be n + b)
    std::vector<int64_t> colptr;
    std::vector<int32_t> rowind;
    std::vector<uint8_t> is_primal;     // [n]
    // ordering and symbolic (factor numbering, rows n + b for border)
    std::vector<int32_t> perm, iperm;
    std::vector<int32_t> parent;        // in-block parent or -1
    std::vector<int64_t> colcount;
    std::vector<int32_t> lp, li;        // exact structure
    std::vector<int32_t> sup, srp, sri; // supernodes and panel rows
    // schedule
    int nlev = 0;
    std::vector<int32_t> level;         // [nsup]
    std::vector<int32_t> panel_off, task_s, task_p, task_cbase, ent_kpos, ent_out, ent_tptr;
    std::vector<int32_t> bterm_ptr, sup_rnb, col_sup;   // solves: border terms, block rows per panel, column -> supernode
    std::vector<std::vector<int32_t>> lev_tasks;   // row tasks of each level
    std::vector<Term> terms, bterms;
    // border rows held by each supernode: (border row, panel row), ascending
    std::vector<std::vector<std::pair<int32_t, int32_t>>> brow;
    // residual rows: the full symmetric row j of the block (both triangles),
    // as (K value, column) pairs; columns n + b are border columns; and per
    // border row b the block's entries (K value, block column) of that row
    std::vector<int32_t> rr_ptr, rr_ent, rb_ptr, rb_ent;
};

// Work lists of every launch (all templates together), per level.
struct Schedule {
    int nlev = 0;
    // factor: A gathers every lower panel entry (k = entry); B factors the
    // diagonal blocks (narrow ones a block per lane, wide ones two blocks
    // per wavefront) and the pivot and column of width-1 supernodes
    // (k = supernode, flagged); C the off-diagonal rows of supernodes 2 or
    // more wide (k = row task)
    std::vector<int32_t> a_ptr, b_ptr, c_ptr;           // [nlev+1]
    std::vector<Work> a, b, c;
    // solve, forward: gathers of the diagonal rows (k = row task), diagonal
    // solves of wide supernodes (k = supernode)
    std::vector<int32_t> f_ptr, d_ptr;                  // [nlev+1]
    std::vector<Work> f, d;
    // solve, backward: the supernodes of each level (k = supernode,
    // kWideFlag on the wide ones), per level the narrow ones first
    std::vector<int32_t> sn_ptr, sn_nar, sn_wmax;       // [nlev+1], [nlev] narrow items, widest supernode
    std::vector<Work> sn;
    // the backward border step: every block column (k = column, kWideFlag
    // on long border columns; narrow first), its border rows' part of the
    // backward sums and D^-1
    std::vector<Work> sb;
    int sb_nar = 0;
    std::vector<Work> bpart;                            // border rows x block groups (forward partials)
    std::vector<Work> schur;                            // border entries x block groups
};

// One network (or one user pattern) of a handle: its blocks, its dense
// first-stage border and the border's symbolic structure.
struct Inst {
    int nb = 0, nl = 0, ng = 0;
    uint32_t flags = 0;
    std::vector<double> gen_c2, br_r, br_x;
    std::vector<double> gen_alpha;       // [ng] AGC participation factors (zeros without AGC)
    std::vector<int32_t> border_pg;      // [ng] border index of pg_g (or -1)
    int blk0 = 0, nblk = 0;              // global block range
    int t0 = 0, nt = 0;                  // template range
    int nbd = 0;
    int64_t col0 = 0, N = 0;             // first global column, columns of the instance
    int64_t bstart = 0;                  // first global column of the border
    int64_t kcsc_border = 0;             // first public CSC value of the border
    int64_t nprimal = 0;
    // border K_bb pattern (lower CSC, border-local) and pivot signs
    std::vector<int64_t> bcolptr;
    std::vector<int32_t> browind;
    std::vector<int32_t> kbb_pos;        // [nbd*nbd]
    std::vector<uint8_t> border_primal;
    // border symbolic (border-local numbering)
    std::vector<int32_t> bparent;
    std::vector<int64_t> bcolcount;
    std::vector<int32_t> blp, bli;
    std::vector<int32_t> bsup;
    // full symmetric rows of K_bb: (value position, border column) pairs
    std::vector<int32_t> kbr_ptr, kbr_ent;
    // offsets in the concatenated device border arrays
    int64_t kbb0 = 0, sbb0 = 0, bd0 = 0, sp0 = 0, cp0 = 0, npk0 = 0, gp0 = 0;
    // border Schur items of every tile pair (all templates, in order) and
    // the wavefront slices over them
    std::vector<MItem> mitems;
    std::vector<int32_t> mdesc_ptr;
    std::vector<int32_t> bperm;          // tile position -> border row
    std::vector<MDesc> mdesc;
    int32_t npair = 0;
    int64_t mw0 = 0, pe0 = 0;
    int64_t nbb() const { return nbd ? bcolptr[nbd] : 0; }
    int64_t npk() const { return int64_t(nbd) * (nbd + 1) / 2; }
};

struct Handle {
    bool from_network = false;
    int64_t N = 0, nprimal = 0;
    int nblk = 0;
    std::vector<Inst> inst;
    std::vector<int64_t> block_col0;     // [nblk] first global column of each block
    std::vector<int32_t> block_tmpl, block_outage, block_bl, block_inst;
    std::vector<Template> tmpl;
    std::vector<int64_t> kbase;          // [nblk] first public CSC value of each block
    int64_t nnzK = 0;
    // totals over instances
    int64_t nbd_tot = 0, nbb_tot = 0, npk_tot = 0, sp_tot = 0, cp_tot = 0, gp_tot = 0, mw_tot = 0, pe_tot = 0;
    int max_nbd = 0;
    // sizes
    int64_t nnzL = 0, nsuper = 0, npanel = 0;
    int64_t kint = 0, lint = 0, dint = 0;   // interleaved K values, panels, pivots (all templates)
    int64_t asm_threads = 0;                // template residual threads (border pg threads follow)
    int64_t asm_wthreads = 0;               // template assembly threads, wavefront-aligned (border pg threads follow)
    int64_t tiles = 0;                      // transpose tiles of all templates
    int64_t rows_waves = 0;                 // residual-row wavefronts of all templates
    int ng_disp = 0, nbus_disp = 0;         // dispatch map: generators and buses (0: not a dispatch network)
    std::vector<int64_t> t_kbase, t_lbase, t_dbase, t_abase, t_awbase, t_tile0, t_rwbase;
    Schedule sched;
    // numeric state
    int64_t nrhs_max = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool factored = false;
    bool blocks_done = false;
    bool bound = false;
    bool values_set = false;                // K values assembled or set since the bind
    bool factor_failed = false;             // ncl_kkt_info saw a factor the solves may not use
    struct Dev {
        double *kval = nullptr;          // interleaved K, then the border K_bb values of every instance
        double *lpan = nullptr, *upan = nullptr, *dval = nullptr, *spart = nullptr, *sbb = nullptr, *lbb = nullptr,
               *ybuf = nullptr,
               *cpart = nullptr;
        double *zint = nullptr, *sint = nullptr;   // state and Sigma in the blocks' interleaved layout order
        double *xint = nullptr, *bint = nullptr, *rint = nullptr;   // residual: x, b, r interleaved (one column)
        double *rbuf = nullptr;          // residual in layout order (its border part feeds the border solve)
        double *epart = nullptr;         // per-workgroup partial maxima of the backward error
        int64_t *stat = nullptr;
        TemplDev *tmpl = nullptr;
        BlockDev *blk = nullptr;
        InstDev *inst = nullptr;
        Work *work = nullptr;            // all work lists
        const uint8_t *bprim = nullptr;
        const int64_t *pg_col = nullptr, *row_pq = nullptr;   // dispatch-map tables
    } d;
    // offsets of each work list inside d.work
    size_t w_a = 0, w_b = 0, w_c = 0, w_f = 0, w_d = 0, w_sn = 0, w_sb = 0, w_bpart = 0;
    // per kernel kind: launches and algorithmic bytes of one step
    std::vector<int64_t> km_launch, km_bytes;
    // event profiling of one kernel kind (events are hipEvent_t, in pairs)
    int prof_kind = -1;
    int64_t prof_stride = 1, prof_seen = 0;   // bracket every prof_stride-th launch of prof_kind
    std::vector<void *> ev;
    size_t ev_used = 0;
    // the second stream of the combined factor and solve, and its fork and
    // join events (hipStream_t, hipEvent_t; created on first use)
    void *side = nullptr, *ev_fork = nullptr, *ev_join = nullptr;
    std::vector<void *> ev_lev;          // one per factor level: the combined call's pipeline
};

// model.cpp
int build_network_model(const ncl_network *net, Handle &h, std::string &err);
int build_pattern_model(int64_t N, int nblk, const int64_t *block_off, const int64_t *colptr, const int32_t *rowind,
                        const uint8_t *is_primal, Handle &h, std::string &err);
// symbolic.cpp
int analyze_template(Template &t, int nbd, int maxw, int znum, int zden, const int32_t *order);
int analyze_border(Handle &h, Inst &I, int maxw, int znum, int zden);
// schedule.cpp
int build_template_schedule(Template &t, int nbd);
int build_schedule(Handle &h);

}  // namespace ncl

struct ncl_kkt {
    ncl::Handle h;
    ~ncl_kkt();
};
