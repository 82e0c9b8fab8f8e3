/* Oracle: symbolic analysis and pivot-free LDL^T of the regularised KKT
 * matrix, plain C, FP64.  TEST INFRASTRUCTURE ONLY: only the tests, the
 * smoke check and the benchmark's CPU-baseline leg load this library.
 *
 * Why a pivot-free LDL^T exists: the (2,2) block C of the Newton system is
 * positive definite (augmented-Lagrangian regularisation, Section IV-B), so
 * with a positive definite (1,1) block the matrix is quasi-definite and
 * every symmetric permutation has an LDL^T factorisation with 1x1 pivots
 * (the paper's "pivoting-free factorization", signed Cholesky).  The
 * factor is unique for a given ordering, so this file computes it by the
 * most direct route: a column-by-column left-looking elimination on the
 * exact fill pattern.
 *
 * Ordering rules (the paper leaves ordering to the solver library; these
 * are the rules this project fixes, applied per block of the
 * block-arrowhead structure, with the first-stage border last):
 *  1. exact minimum degree on the block's graph (its vertices plus the
 *     border vertices it touches), with an explicit elimination graph: pick
 *     the non-border vertex of smallest current degree (border neighbours
 *     count), ties to the smallest layout index; its neighbours become a
 *     clique; border vertices are never picked.  A caller may give the
 *     elimination sequence of each block instead (block-respecting, the
 *     border in layout order); rules 2-6 then apply to it unchanged;
 *  2. parent(v) = the neighbour of v at its elimination that is eliminated
 *     first (border vertices come after all block vertices, in layout
 *     order); the block order is the DFS postorder of this forest, children
 *     and roots taken in increasing elimination position;
 *  3. global order: block 0, block 1, ..., block K, then the border in
 *     layout order;
 *  4. symbolic factorisation struct(j) = adj(j) U struct(children) \ {<= j};
 *  5. fundamental supernodes: j, j+1 join iff parent(j) = j+1,
 *     colcount(j) = colcount(j+1) + 1 and j+1 has one child, never across
 *     a block or block/border boundary, and never beyond 32 columns (a
 *     longer chain starts a new supernode every 32 columns);
 *  6. relaxed amalgamation: going left to right, the current supernode s
 *     absorbs the next one p iff parent(last(s)) = first(p), both lie in the
 *     same block (or both in the border), width(s)+width(p) <= maxw and
 *     zden * (explicit zeros of the merged panel) <= znum * (its entries);
 *     the merged supernode stays current.
 * This file's code shares nothing with the GPU library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* no supernode is wider than this many columns (rule 5) */
#define ORACLE_MAXW_HARD 32

typedef struct {
    int64_t N;
    int32_t nblk;
    int64_t *block_off;  /* nblk+1 (+ border end = N) */
    int32_t *perm;       /* new -> old (layout index) */
    int32_t *iperm;      /* old -> new */
    int32_t *parent;     /* etree in new numbering, -1 = root */
    int64_t *colcount;   /* including the diagonal */
    int64_t *lp;         /* exact L pattern, CSC of strictly-lower rows, N+1 */
    int32_t *li;
    int64_t nsuper;
    int64_t *sup;        /* supernode column pointer, nsuper+1 */
    int64_t *srp;        /* panel row pointer, nsuper+1 */
    int32_t *sri;        /* panel rows (columns first, then off-diagonal rows) */
    /* numeric */
    double *lx;          /* values on lp/li */
    double *d;
    int64_t npos, nneg, nzero, first_bad;
    /* row structure of L (transpose of lp/li) */
    int64_t *rp;
    int32_t *rk;         /* column k of entry */
    int64_t *rpos;       /* position of the entry in li/lx */
} oracle_sym;

/* ------------------------------------------------------------ ordering */

/* dense bit-matrix elimination on one block graph: exact minimum degree,
 * or (given != NULL) the elimination sequence given[0..nv-1] (a caller's
 * ordering, rule 1 replaced, rules 2-6 unchanged).
 * nloc = block vertices (0..nv-1) followed by nbd border vertices.
 * adjacency given as a list of undirected edges (a, b) in local indices.
 * Writes order[0..nv-1] = block vertices in the final (postordered) order. */
static int block_order(int nv, int nbd, int64_t ne, const int32_t *ea, const int32_t *eb,
                       const int32_t *given, int32_t *order) {
    int n = nv + nbd;
    if (nv == 0) return 0;
    int64_t W = (n + 63) / 64;
    uint64_t *bits = (uint64_t *)calloc((size_t)n * (size_t)W, sizeof(uint64_t));
    int32_t *deg = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    char *gone = (char *)calloc((size_t)n, 1);
    int32_t *elim = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);    /* elimination sequence */
    int32_t *epos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);     /* vertex -> position */
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);     /* parent vertex or -1 */
    int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t **nbl = (int32_t **)calloc((size_t)nv, sizeof(int32_t *)); /* neighbours at elimination */
    if (!bits || !deg || !gone || !elim || !epos || !par || !nbr || !nbl) return -2;
    for (int64_t e = 0; e < ne; e++) {
        int a = ea[e], b = eb[e];
        if (a == b) continue;
        bits[(int64_t)a * W + (b >> 6)] |= 1ULL << (b & 63);
        bits[(int64_t)b * W + (a >> 6)] |= 1ULL << (a & 63);
    }
    for (int u = 0; u < n; u++) {
        int c = 0;
        for (int64_t w = 0; w < W; w++) c += __builtin_popcountll(bits[(int64_t)u * W + w]);
        deg[u] = c;
        epos[u] = -1;
    }
    for (int step = 0; step < nv; step++) {
        /* smallest current degree among remaining block vertices, ties to the smallest index */
        int v = -1;
        if (given) {
            v = given[step];
            if (v < 0 || v >= nv || gone[v]) return -1;
        } else {
            for (int u = 0; u < nv; u++)
                if (!gone[u] && (v < 0 || deg[u] < deg[v])) v = u;
        }
        elim[step] = v;
        epos[v] = step;
        gone[v] = 1;
        int nn = 0;
        const uint64_t *rv = bits + (int64_t)v * W;
        for (int64_t w = 0; w < W; w++) {
            uint64_t x = rv[w];
            while (x) {
                int b = __builtin_ctzll(x);
                x &= x - 1;
                nbr[nn++] = (int)(w * 64 + b);   /* rows hold remaining vertices only */
            }
        }
        nbl[v] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nn + 1));
        memcpy(nbl[v], nbr, sizeof(int32_t) * (size_t)nn);
        nbl[v][nn] = -1;
        /* neighbours become a clique; v leaves every row */
        for (int a = 0; a < nn; a++) {
            int u = nbr[a];
            uint64_t *ru = bits + (int64_t)u * W;
            for (int64_t w = 0; w < W; w++) ru[w] |= rv[w];
            ru[u >> 6] &= ~(1ULL << (u & 63));
            ru[v >> 6] &= ~(1ULL << (v & 63));
        }
        for (int a = 0; a < nn; a++) {
            int u = nbr[a];
            int c = 0;
            const uint64_t *ru = bits + (int64_t)u * W;
            for (int64_t w = 0; w < W; w++) c += __builtin_popcountll(ru[w]);
            deg[u] = c;
        }
    }
    /* parent = block neighbour at elimination with the smallest position */
    for (int u = 0; u < nv; u++) {
        int bp = -1;
        for (int a = 0; nbl[u][a] >= 0; a++) {
            int w2 = nbl[u][a];
            if (w2 < nv && (bp < 0 || epos[w2] < epos[bp])) bp = w2;
        }
        par[u] = bp;
        free(nbl[u]);
    }
    free(nbl);
    /* DFS postorder, children and roots in increasing elimination position */
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);
    int32_t *stk = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);
    int32_t *it = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);
    for (int u = 0; u < nv; u++) head[u] = -1;
    for (int s = nv - 1; s >= 0; s--) {      /* push in decreasing position: lists increase */
        int u = elim[s];
        if (par[u] >= 0) {
            next[u] = head[par[u]];
            head[par[u]] = u;
        }
    }
    int cnt = 0;
    for (int s = 0; s < nv; s++) {
        int r = elim[s];
        if (par[r] >= 0) continue;
        int top = 0;
        stk[0] = r;
        it[0] = head[r];
        while (top >= 0) {
            int c = it[top];
            if (c >= 0) {
                it[top] = next[c];
                top++;
                stk[top] = c;
                it[top] = head[c];
            } else {
                order[cnt++] = stk[top];
                top--;
            }
        }
    }
    free(head); free(next); free(stk); free(it);
    free(bits); free(deg); free(gone); free(elim); free(epos); free(par); free(nbr);
    return cnt == nv ? 0 : -3;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------ symbolic */

void oracle_free(oracle_sym *s) {
    if (!s) return;
    free(s->block_off); free(s->perm); free(s->iperm); free(s->parent); free(s->colcount);
    free(s->lp); free(s->li); free(s->sup); free(s->srp); free(s->sri);
    free(s->lx); free(s->d); free(s->rp); free(s->rk); free(s->rpos);
    free(s);
}

/* A: lower triangle (incl. diagonal) in layout order, CSC: colptr[N+1], rowind.
 * block_off[nblk+1]: block b occupies [block_off[b], block_off[b+1]); the
 * border is [block_off[nblk], N). */
int oracle_symbolic(int64_t N, const int64_t *colptr, const int32_t *rowind, int32_t nblk,
                    const int64_t *block_off, int32_t maxw, int32_t znum, int32_t zden,
                    const int32_t *user_perm, oracle_sym **out) {
    if (N <= 0 || nblk <= 0 || maxw < 1 || zden <= 0 || znum < 0) return -1;
    oracle_sym *s = (oracle_sym *)calloc(1, sizeof(oracle_sym));
    s->N = N;
    s->nblk = nblk;
    s->block_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nblk + 2));
    for (int b = 0; b <= nblk; b++) s->block_off[b] = block_off[b];
    s->block_off[nblk + 1] = N;
    int64_t bstart = block_off[nblk];
    int nbd = (int)(N - bstart);
    /* full symmetric adjacency lists (off-diagonal) in layout numbering */
    int64_t *deg = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    for (int64_t j = 0; j < N; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int64_t i = rowind[p];
            if (i == j) continue;
            deg[i]++;
            deg[j]++;
        }
    int64_t *ap = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    ap[0] = 0;
    for (int64_t j = 0; j < N; j++) ap[j + 1] = ap[j] + deg[j];
    int32_t *ai = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ap[N] > 0 ? ap[N] : 1));
    for (int64_t j = 0; j < N; j++) deg[j] = ap[j];
    for (int64_t j = 0; j < N; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int64_t i = rowind[p];
            if (i == j) continue;
            ai[deg[i]++] = (int32_t)j;
            ai[deg[j]++] = (int32_t)i;
        }
    for (int64_t j = 0; j < N; j++) qsort(ai + ap[j], (size_t)(ap[j + 1] - ap[j]), sizeof(int32_t), cmp_i32);
    free(deg);

    /* block orders; reuse the order of an earlier block whose local graph is identical */
    s->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int rc = 0;
    for (int b = 0; b < nblk && rc == 0; b++) {
        int64_t o = block_off[b];
        int nv = (int)(block_off[b + 1] - o);
        int reuse = -1;
        for (int c = 0; c < b && reuse < 0 && !user_perm; c++) {
            int64_t oc = block_off[c];
            if (block_off[c + 1] - oc != nv) continue;
            int same = 1;
            for (int v = 0; v < nv && same; v++) {
                int64_t p1 = ap[o + v], q1 = ap[o + v + 1], p2 = ap[oc + v], q2 = ap[oc + v + 1];
                if (q1 - p1 != q2 - p2) { same = 0; break; }
                for (int64_t a = 0; a < q1 - p1; a++) {
                    int64_t x1 = ai[p1 + a], x2 = ai[p2 + a];
                    int64_t l1 = x1 >= bstart ? x1 - bstart + (1LL << 40) : x1 - o;
                    int64_t l2 = x2 >= bstart ? x2 - bstart + (1LL << 40) : x2 - oc;
                    if (l1 != l2) { same = 0; break; }
                }
            }
            if (same) reuse = c;
        }
        if (reuse >= 0) {
            int64_t oc = block_off[reuse];
            for (int v = 0; v < nv; v++) s->perm[o + v] = (int32_t)(s->perm[oc + v] - oc + o);
            continue;
        }
        /* local edge list: block vertices 0..nv-1, border vertex bstart+t -> nv+t */
        int64_t ne = 0;
        for (int v = 0; v < nv; v++) ne += ap[o + v + 1] - ap[o + v];
        int32_t *ea = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne + 1));
        int32_t *eb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne + 1));
        int64_t k = 0;
        for (int v = 0; v < nv; v++)
            for (int64_t p = ap[o + v]; p < ap[o + v + 1]; p++) {
                int64_t x = ai[p];
                int loc;
                if (x >= o && x < o + nv) loc = (int)(x - o);
                else if (x >= bstart) loc = nv + (int)(x - bstart);
                else { rc = -4; continue; }      /* edge to another block: not block-arrowhead */
                ea[k] = v;
                eb[k] = loc;
                k++;
            }
        int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv + 1));
        int32_t *given = NULL;
        if (user_perm) {
            /* the caller's order of this block, in block-local indices */
            given = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv + 1));
            for (int v = 0; v < nv; v++) {
                int64_t x = (int64_t)user_perm[o + v] - o;
                if (x < 0 || x >= nv) rc = -1;
                given[v] = (int32_t)x;
            }
        }
        if (rc == 0) rc = block_order(nv, nbd, k, ea, eb, given, ord);
        free(given);
        for (int v = 0; v < nv && rc == 0; v++) s->perm[o + v] = (int32_t)(o + ord[v]);
        free(ea); free(eb); free(ord);
    }
    if (rc) { free(ap); free(ai); oracle_free(s); return rc; }
    for (int64_t j = bstart; j < N; j++) {
        s->perm[j] = (int32_t)j;
        if (user_perm && user_perm[j] != j) rc = -1;    /* the border keeps its layout order */
    }
    if (rc) { free(ap); free(ai); oracle_free(s); return rc; }
    s->iperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int64_t j = 0; j < N; j++) s->iperm[s->perm[j]] = (int32_t)j;

    /* symbolic factorisation in the new numbering:
     * struct(j) = {i > j : A_ij != 0} U struct(children) \ {j} */
    int64_t cap = 1 << 20;
    int32_t *li = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int64_t *lp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *chead = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *cnext = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int64_t j = 0; j < N; j++) { chead[j] = -1; mark[j] = -1; }
    lp[0] = 0;
    for (int64_t j = 0; j < N; j++) {
        int64_t old = s->perm[j];
        int64_t nt = 0;
        mark[j] = (int32_t)j;
        for (int64_t p = ap[old]; p < ap[old + 1]; p++) {
            int32_t i = s->iperm[ai[p]];
            if (i > j && mark[i] != j) { mark[i] = (int32_t)j; tmp[nt++] = i; }
        }
        for (int32_t c = chead[j]; c >= 0; c = cnext[c])
            for (int64_t p = lp[c]; p < lp[c + 1]; p++) {
                int32_t i = li[p];
                if (i > j && mark[i] != j) { mark[i] = (int32_t)j; tmp[nt++] = i; }
            }
        qsort(tmp, (size_t)nt, sizeof(int32_t), cmp_i32);
        if (lp[j] + nt > cap) {
            while (lp[j] + nt > cap) cap *= 2;
            li = (int32_t *)realloc(li, sizeof(int32_t) * (size_t)cap);
        }
        memcpy(li + lp[j], tmp, sizeof(int32_t) * (size_t)nt);
        lp[j + 1] = lp[j] + nt;
        parent[j] = nt ? tmp[0] : -1;
        if (nt) { cnext[j] = chead[tmp[0]]; chead[tmp[0]] = (int32_t)j; }
    }
    free(ap); free(ai); free(mark); free(tmp);
    s->lp = lp;
    s->li = li;
    s->parent = parent;
    s->colcount = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int32_t *nchild = (int32_t *)calloc((size_t)N, sizeof(int32_t));
    for (int64_t j = 0; j < N; j++) {
        s->colcount[j] = lp[j + 1] - lp[j] + 1;
        if (parent[j] >= 0) nchild[parent[j]]++;
    }
    free(chead); free(cnext);
    /* region id of a column: block number, or nblk for the border */
    int32_t *region = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int b = 0; b <= nblk; b++)
        for (int64_t j = s->block_off[b]; j < s->block_off[b + 1]; j++) region[j] = b;

    /* fundamental supernodes */
    int64_t *fs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    int64_t nf = 0;
    fs[nf++] = 0;
    int64_t run = 1;                         /* width of the supernode being grown */
    for (int64_t j = 0; j + 1 < N; j++) {
        int join = parent[j] == j + 1 && s->colcount[j] == s->colcount[j + 1] + 1 &&
                   nchild[j + 1] == 1 && region[j] == region[j + 1] && run < ORACLE_MAXW_HARD;
        if (join) run++;
        else { fs[nf++] = j + 1; run = 1; }
    }
    fs[nf] = N;
    /* relaxed amalgamation */
    int64_t *sp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nf + 1));
    int64_t ns = 0;
    int64_t cf = fs[0], cl = fs[1] - 1;        /* current supernode [cf, cl] */
    for (int64_t q = 1; q < nf; q++) {
        int64_t pf = fs[q], pl = fs[q + 1] - 1;
        int ok = parent[cl] == pf && region[cl] == region[pf] && (pl - cf + 1) <= maxw &&
                 (pl - cf + 1) <= ORACLE_MAXW_HARD;
        if (ok) {
            /* merged panel rows = columns [cf, pl] U (union of structs) \ columns */
            int64_t w = pl - cf + 1;
            int64_t nrow_off = 0;
            /* union of struct(j) for j in [cf, pl] restricted to rows > pl */
            int64_t cnt = 0;
            int32_t *u = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
            char *seen = (char *)calloc((size_t)N, 1);
            for (int64_t j = cf; j <= pl; j++)
                for (int64_t p = lp[j]; p < lp[j + 1]; p++)
                    if (li[p] > pl && !seen[li[p]]) { seen[li[p]] = 1; u[cnt++] = li[p]; }
            nrow_off = cnt;
            free(u); free(seen);
            int64_t entries = w * (w + 1) / 2 + w * nrow_off;
            int64_t truenz = 0;
            for (int64_t j = cf; j <= pl; j++) truenz += s->colcount[j];
            int64_t zeros = entries - truenz;
            ok = (int64_t)zden * zeros <= (int64_t)znum * entries;
        }
        if (ok) {
            cl = pl;
        } else {
            sp[ns++] = cf;
            cf = pf;
            cl = pl;
        }
    }
    sp[ns++] = cf;
    sp[ns] = N;
    free(fs); free(nchild); free(region);
    s->nsuper = ns;
    s->sup = sp;
    /* panel rows: columns, then the union of off-diagonal structs (sorted) */
    s->srp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns + 1));
    int64_t rcap = 1 << 20;
    s->sri = (int32_t *)malloc(sizeof(int32_t) * (size_t)rcap);
    int32_t *mk = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *u = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int64_t j = 0; j < N; j++) mk[j] = -1;
    s->srp[0] = 0;
    for (int64_t q = 0; q < ns; q++) {
        int64_t f = sp[q], l = sp[q + 1] - 1;
        int64_t cnt = 0;
        for (int64_t j = f; j <= l; j++) u[cnt++] = (int32_t)j;
        int64_t c0 = cnt;
        for (int64_t j = f; j <= l; j++)
            for (int64_t p = lp[j]; p < lp[j + 1]; p++)
                if (li[p] > l && mk[li[p]] != q) { mk[li[p]] = (int32_t)q; u[cnt++] = li[p]; }
        qsort(u + c0, (size_t)(cnt - c0), sizeof(int32_t), cmp_i32);
        if (s->srp[q] + cnt > rcap) {
            while (s->srp[q] + cnt > rcap) rcap *= 2;
            s->sri = (int32_t *)realloc(s->sri, sizeof(int32_t) * (size_t)rcap);
        }
        memcpy(s->sri + s->srp[q], u, sizeof(int32_t) * (size_t)cnt);
        s->srp[q + 1] = s->srp[q] + cnt;
    }
    free(mk); free(u);
    *out = s;
    return 0;
}

int64_t oracle_N(const oracle_sym *s) { return s->N; }
int64_t oracle_nnzl(const oracle_sym *s) { return s->lp[s->N]; }
int64_t oracle_nsuper(const oracle_sym *s) { return s->nsuper; }
int64_t oracle_npanel(const oracle_sym *s) { return s->srp[s->nsuper]; }

void oracle_get_symbolic(const oracle_sym *s, int32_t *perm, int32_t *parent, int64_t *colcount,
                         int64_t *lp, int32_t *li, int64_t *sup, int64_t *srp, int32_t *sri) {
    int64_t N = s->N;
    if (perm) memcpy(perm, s->perm, sizeof(int32_t) * (size_t)N);
    if (parent) memcpy(parent, s->parent, sizeof(int32_t) * (size_t)N);
    if (colcount) memcpy(colcount, s->colcount, sizeof(int64_t) * (size_t)N);
    if (lp) memcpy(lp, s->lp, sizeof(int64_t) * (size_t)(N + 1));
    if (li) memcpy(li, s->li, sizeof(int32_t) * (size_t)s->lp[N]);
    if (sup) memcpy(sup, s->sup, sizeof(int64_t) * (size_t)(s->nsuper + 1));
    if (srp) memcpy(srp, s->srp, sizeof(int64_t) * (size_t)(s->nsuper + 1));
    if (sri) memcpy(sri, s->sri, sizeof(int32_t) * (size_t)s->srp[s->nsuper]);
}

/* ------------------------------------------------------------ numeric */

static void build_rows(oracle_sym *s) {
    if (s->rp) return;
    int64_t N = s->N, nz = s->lp[N];
    s->rp = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    s->rk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nz + 1));
    s->rpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nz + 1));
    for (int64_t p = 0; p < nz; p++) s->rp[s->li[p] + 1]++;
    for (int64_t j = 0; j < N; j++) s->rp[j + 1] += s->rp[j];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    memcpy(fill, s->rp, sizeof(int64_t) * (size_t)N);
    for (int64_t k = 0; k < N; k++)          /* increasing k: row lists come out sorted */
        for (int64_t p = s->lp[k]; p < s->lp[k + 1]; p++) {
            int64_t q = fill[s->li[p]]++;
            s->rk[q] = (int32_t)k;
            s->rpos[q] = p;
        }
    free(fill);
}

/* left-looking elimination of columns [c0, c1) using work vector w (dense, N) */
static void factor_range(oracle_sym *s, const int64_t *ap, const int32_t *ai, const double *ax,
                         int64_t c0, int64_t c1, double *w) {
    const int64_t *lp = s->lp;
    const int32_t *li = s->li;
    double *lx = s->lx, *d = s->d;
    for (int64_t j = c0; j < c1; j++) {
        /* load column j of the permuted lower triangle into w (rows >= j) */
        for (int64_t p = ap[j]; p < ap[j + 1]; p++) w[ai[p]] += ax[p];
        /* subtract l_ik d_k l_jk for every k < j with l_jk != 0, k increasing */
        for (int64_t q = s->rp[j]; q < s->rp[j + 1]; q++) {
            int64_t k = s->rk[q], pj = s->rpos[q];
            double f = lx[pj] * d[k];
            w[j] -= lx[pj] * f;
            for (int64_t p = pj + 1; p < lp[k + 1]; p++) w[li[p]] -= lx[p] * f;
        }
        double dj = w[j];
        d[j] = dj;
        w[j] = 0.0;
        for (int64_t p = lp[j]; p < lp[j + 1]; p++) {
            lx[p] = w[li[p]] / dj;
            w[li[p]] = 0.0;
        }
    }
}

/* Numeric factorisation.  A: lower triangle of the ORIGINAL (layout-order)
 * matrix, CSC colptr/rowind/vals.  Blocks run in parallel, then the border. */
int oracle_factor(oracle_sym *s, const int64_t *colptr, const int32_t *rowind, const double *vals,
                  int32_t nthreads) {
    int64_t N = s->N;
    build_rows(s);
    /* permuted lower triangle, CSC in the new numbering */
    int64_t nz = colptr[N];
    int64_t *cnt = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    for (int64_t j = 0; j < N; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int64_t a = s->iperm[rowind[p]], b = s->iperm[j];
            cnt[(a < b ? a : b) + 1]++;
        }
    for (int64_t j = 0; j < N; j++) cnt[j + 1] += cnt[j];
    int64_t *ap = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    memcpy(ap, cnt, sizeof(int64_t) * (size_t)(N + 1));
    int32_t *ai = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nz + 1));
    double *ax = (double *)malloc(sizeof(double) * (size_t)(nz + 1));
    for (int64_t j = 0; j < N; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int64_t a = s->iperm[rowind[p]], b = s->iperm[j];
            int64_t c = a < b ? a : b, r = a < b ? b : a;
            int64_t q = cnt[c]++;
            ai[q] = (int32_t)r;
            ax[q] = vals[p];
        }
    free(cnt);
    free(s->lx);
    free(s->d);
    s->lx = (double *)calloc((size_t)s->lp[N] + 1, sizeof(double));
    s->d = (double *)calloc((size_t)N, sizeof(double));
    int nt = nthreads > 0 ? nthreads : 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        double *w = (double *)calloc((size_t)N, sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int b = 0; b < s->nblk; b++) factor_range(s, ap, ai, ax, s->block_off[b], s->block_off[b + 1], w);
        free(w);
    }
    (void)nt;
    double *w = (double *)calloc((size_t)N, sizeof(double));
    factor_range(s, ap, ai, ax, s->block_off[s->nblk], N, w);
    free(w);
    free(ap); free(ai); free(ax);
    s->npos = s->nneg = s->nzero = 0;
    s->first_bad = -1;
    for (int64_t j = 0; j < N; j++) {
        double dj = s->d[j];
        if (dj > 0) s->npos++;
        else if (dj < 0) s->nneg++;
        else s->nzero++;
        if ((!isfinite(dj) || dj == 0.0) && s->first_bad < 0) s->first_bad = j;
    }
    return s->first_bad < 0 ? 0 : -5;
}

void oracle_get_numeric(const oracle_sym *s, double *lx, double *d, int64_t *inertia) {
    if (lx) memcpy(lx, s->lx, sizeof(double) * (size_t)s->lp[s->N]);
    if (d) memcpy(d, s->d, sizeof(double) * (size_t)s->N);
    if (inertia) { inertia[0] = s->npos; inertia[1] = s->nneg; inertia[2] = s->nzero; inertia[3] = s->first_bad; }
}

/* x = K^{-1} b for nrhs columns (layout order, leading dimension ld). */
int oracle_solve(const oracle_sym *s, const double *b, double *x, int32_t nrhs, int64_t ld) {
    int64_t N = s->N;
    if (!s->lx) return -4;
    double *y = (double *)malloc(sizeof(double) * (size_t)N);
    for (int32_t r = 0; r < nrhs; r++) {
        const double *br = b + (int64_t)r * ld;
        for (int64_t j = 0; j < N; j++) y[j] = br[s->perm[j]];
        for (int64_t j = 0; j < N; j++) {
            double yj = y[j];
            for (int64_t p = s->lp[j]; p < s->lp[j + 1]; p++) y[s->li[p]] -= s->lx[p] * yj;
        }
        for (int64_t j = 0; j < N; j++) y[j] /= s->d[j];
        for (int64_t j = N - 1; j >= 0; j--) {
            double a = y[j];
            for (int64_t p = s->lp[j]; p < s->lp[j + 1]; p++) a -= s->lx[p] * y[s->li[p]];
            y[j] = a;
        }
        double *xr = x + (int64_t)r * ld;
        for (int64_t j = 0; j < N; j++) xr[s->perm[j]] = y[j];
    }
    free(y);
    return 0;
}
