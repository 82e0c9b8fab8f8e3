// Internal structures of libnclkkt: host-side symbolic data and the plain
// structs that carry device tables into the kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ncl_kkt.h"

namespace ncl {

constexpr int kMaxW = 32;            // widest supernode (panel rows fit one thread's accumulator)
constexpr int32_t kBorderFlag = int32_t(1u << 30);   // slot refers to the border K_bb pattern

// ---------------------------------------------------------------- device tables

// One descendant supernode d's contribution to one panel row of a target
// supernode s (factor), or to one column of s (forward solve).
struct GItem {
    int32_t ioff;    // offset (doubles, within the block's panel storage) of L_d[row, 0]
    int32_t coff;    // offset of L_d[first row that is a column of s, 0]
    int32_t dcol;    // first column of d (block-local factor numbering)
    int32_t crel;    // index of the first entry of d's target-column list in crel[]
    int32_t meta;    // ld (16 bits) | wd << 16 | nc << 24
};

struct AEnt {        // one K entry of a panel row
    int32_t kpos;    // position in the block's K values (template-relative CSC position)
    int32_t crel;    // target column within the supernode
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
    GS_NUPNUP, GS_NUMNUM, GS_SUPSUP, GS_SLOSLO, GS_LL, GS_UU, GS_DD, GS_CUCU, GS_CLCL, GS_N
};
// State index tables per bus / generator: layout-local positions (n + b for border refs).
enum BusIdx { BI_VM, BI_VA, BI_P, BI_Q, BI_N };
enum GenIdx { GI_BUS, GI_QG, GI_PG, GI_NUP, GI_NUM, GI_SUP, GI_SLO, GI_LIN, GI_DUP, GI_DLO, GI_CUP, GI_CLO, GI_VM0, GI_N };

struct TemplDev {
    int32_t n, nsup, nlev, ntask;
    int32_t nbd, nb, nl, ng;
    int64_t panel_size;            // doubles of panel storage per block
    int32_t pvpq_rows;             // this template has the complementarity rows
    int32_t has_pg_local;          // single-block network: pg inside the block
    // supernodes (block-local factor numbering; border rows are n + b)
    const int32_t *sup_first;      // [nsup+1]
    const int32_t *sup_rowptr;     // [nsup+1]
    const int32_t *sup_rows;
    const int32_t *panel_off;      // [nsup+1]
    // level schedule
    const int32_t *lev_sup_ptr;    // [nlev+1]
    const int32_t *lev_sup;
    const int32_t *lev_task_ptr;   // [nlev+1]
    const int32_t *task_s;         // [ntask]
    const int32_t *task_p;
    const int32_t *task_gptr;      // [ntask+1]
    const GItem *gitems;
    const uint8_t *crel;
    const int32_t *task_aptr;      // [ntask+1]
    const AEnt *aents;
    const int32_t *lev_dtask_ptr;  // [nlev+1] tasks whose row is a column of its supernode
    const int32_t *dtask;
    // border rows: supernodes whose panel holds border row b, ascending
    const int32_t *bpath_ptr;      // [nbd+1]
    const int32_t *bpath_s;
    const int32_t *bpath_pos;
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
    const uint8_t *col_primal;     // [n] expected pivot sign (1: positive) in factor order
};

struct BlockDev {
    int32_t tmpl;
    int32_t outage;                // outaged branch or -1
    int64_t col0;                  // first global column (layout and factor numbering agree per block)
    int64_t kbase;                 // K values base
    int64_t lbase;                 // panel storage base
};

struct BorderDev {
    int32_t nbd;
    int64_t kbase;                 // K values base of the border columns
    const int32_t *kbb_pos;        // [nbd*nbd] position (relative to kbase) of (i, j), i >= j, or -1
    const int32_t *pg_idx;         // [ng] border index of pg_g (or -1)
    const double *gen_c2;          // [ng]
    int32_t ng;
    int32_t has_border;
};

// ---------------------------------------------------------------- host symbolic

struct Template {
    int n = 0;                     // block columns
    int nprim = 0;
    bool pvpq_rows = false;
    bool pg_local = false;
    // model tables (layout-local; border refs n + b)
    std::vector<int32_t> bus_idx, bus_slot, bus_adj_ptr, bus_adj, br_slot, br_idx, gen_idx, gen_slot;
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
    std::vector<int32_t> panel_off, lev_sup_ptr, lev_sup, lev_task_ptr, task_s, task_p, task_gptr,
        task_aptr, lev_dtask_ptr, dtask, bpath_ptr, bpath_s, bpath_pos;
    std::vector<GItem> gitems;
    std::vector<uint8_t> crel;
    std::vector<AEnt> aents;
    int nlev = 0;
};

struct Handle {
    bool from_network = false;
    int64_t N = 0, nprimal = 0;
    int nblk = 0, nbd = 0;
    int nb = 0, nl = 0, ng = 0;
    uint32_t flags = 0;
    std::vector<int64_t> block_off;      // [nblk+1]
    std::vector<int32_t> block_tmpl, block_outage;
    std::vector<Template> tmpl;
    std::vector<double> gen_c2, br_r, br_x;
    std::vector<int32_t> border_pg;      // [ng] border index of pg_g
    // K pattern
    std::vector<int64_t> kbase;          // [nblk] + border base at the end
    int64_t nnzK = 0;
    std::vector<int64_t> bcolptr;        // border K_bb lower CSC (border-local)
    std::vector<int32_t> browind;
    std::vector<int32_t> kbb_pos;        // [nbd*nbd]
    std::vector<uint8_t> border_primal;
    // border symbolic (border-local numbering)
    std::vector<int32_t> bparent;        // border parent (border-local) or -1
    std::vector<int64_t> bcolcount;
    std::vector<int32_t> blp, bli;       // exact structure
    std::vector<int32_t> bsup;           // border supernodes
    // sizes
    int64_t nnzL = 0, nsuper = 0, npanel = 0;
    std::vector<int64_t> lbase;          // [nblk+1]
    // numeric state
    int64_t nrhs_max = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool factored = false;
    bool blocks_done = false;
    bool bound = false;
    // device pointers (inside the workspace)
    struct Dev {
        double *kval = nullptr, *lpan = nullptr, *dval = nullptr, *spart = nullptr, *sbb = nullptr,
               *ybuf = nullptr, *cpart = nullptr, *xb = nullptr;
        int64_t *stat = nullptr;         // per-block status words + border row
        double *dmm = nullptr;           // per-block min/max |d|
        TemplDev *tmpl = nullptr;
        BlockDev *blk = nullptr;
        int32_t *kbb_pos = nullptr, *border_pg = nullptr;
        double *gen_c2 = nullptr, *br_g = nullptr, *br_b = nullptr;
    } d;
    const uint8_t *bprim_dev = nullptr;  // border pivot signs (device)
};

// model.cpp
int build_network_model(const ncl_network *net, Handle &h, std::string &err);
int build_pattern_model(int64_t N, int nblk, const int64_t *block_off, const int64_t *colptr, const int32_t *rowind,
                        const uint8_t *is_primal, Handle &h, std::string &err);
// symbolic.cpp
int analyze_template(Template &t, int nbd, int maxw, int znum, int zden);
int analyze_border(Handle &h, int maxw, int znum, int zden);
// schedule.cpp
int build_schedule(Template &t, int nbd);
// api helpers
int64_t panel_entries(const Template &t);

}  // namespace ncl

struct ncl_kkt {
    ncl::Handle h;
};
