"""Seeded synthetic grids and KKT states (test and benchmark inputs).

This module draws the random inputs that both the CPU oracle and the GPU
library consume: a network topology with branch impedances, generator
placement, branch-outage contingencies, and per-iteration primal/dual
states.  It holds none of the method's arithmetic (no admittances, no
derivatives, no factorisation); it only knows how many variables and rows
of each kind a block has, so that it can draw each value from the right
distribution, in the layout order described below.

The paper's benchmark uses MATPOWER cases (ACTIVSg500, ACTIVSg2000, ...)
that are not reproduced here; these seeded grids stand in for them with
the same sizes (Section V, Tables II and III).

Layout (per block, block-local order)
-------------------------------------
primal: vm[nb], va[nb], qg[ng], and with complementarity rows
        nu_plus[ng], nu_minus[ng], s_up[ng], s_lo[ng]
        (a single-block network also has pg[ng] after qg; in the
        complementarity base block vm at generator buses is absent: those
        voltages are the border variables vm0); with AGC rows a
        contingency block then adds pgk[ng], pi_plus[ng], pi_minus[ng],
        sp_up[ng], sp_lo[ng] and its adjustment delta[1]
dual:   P[nb], Q[nb], Ffrom[nl], Fto[nl], and with complementarity rows
        LIN[ng], DUP[ng], DLO[ng], CUP[ng], CLO[ng]; with AGC rows a
        contingency block then adds ALIN[ng], ADUP[ng], ADLO[ng],
        ACUP[ng], ACLO[ng]
global: block 0 (base case), blocks 1..K (contingencies), then the border
        pg[ng] followed (complementarity only) by vm0[ng].  A screening
        network (first-stage pg and vm0 fixed) has the K contingency
        blocks alone, with no base block and no border.

Seeds: numpy PCG64 seeded by SeedSequence([2510, 13333, cfg, instance,
iteration]); draws follow a fixed order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# kind codes of layout positions
VM, VA, QG, PG, NUP, NUM, SUP, SLO, VM0, PGK, PIP, PIM, SPU, SPL, DELTA = range(15)
ROW_P, ROW_Q, ROW_FF, ROW_FT, ROW_LIN, ROW_DUP, ROW_DLO, ROW_CUP, ROW_CLO = range(16, 25)
ROW_ALIN, ROW_ADUP, ROW_ADLO, ROW_ACUP, ROW_ACLO = range(25, 30)
PRIMAL_KINDS = (VM, VA, QG, PG, NUP, NUM, SUP, SLO, VM0, PGK, PIP, PIM, SPU, SPL, DELTA)


def rng(cfg: int, instance: int = 0, iteration: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([2510, 13333, int(cfg), int(instance), int(iteration)])))


@dataclasses.dataclass
class Network:
    nb: int
    nl: int
    ng: int
    br_from: np.ndarray   # int32 [nl], from = min endpoint
    br_to: np.ndarray     # int32 [nl]
    br_r: np.ndarray      # float64 [nl]
    br_x: np.ndarray      # float64 [nl]
    gen_bus: np.ndarray   # int32 [ng], distinct buses, draw order
    gen_c2: np.ndarray    # float64 [ng] quadratic cost coefficient
    outage: np.ndarray    # int32 [K] outaged branch of contingency k+1
    pvpq: bool            # complementarity (PV/PQ switching) rows present
    rho: float
    screen: bool = False  # contingency screening: first-stage pg (and vm0) fixed, blocks = contingencies
    agc: bool = False     # AGC droop complementarity rows in the contingency blocks
    gen_alpha: np.ndarray = None   # float64 [ng] participation factors (AGC only)

    @property
    def ncont(self) -> int:
        return int(self.outage.shape[0])

    @property
    def nblk(self) -> int:
        return self.ncont if self.screen else self.ncont + 1

    @property
    def single(self) -> bool:
        return self.ncont == 0 and not self.screen

    def cont_block(self, blk: int) -> bool:
        """Whether block blk is a contingency block (its outage: outage_of)."""
        return self.screen or blk > 0

    def outage_of(self, blk: int) -> int:
        """Outaged branch of block blk, or -1 for the base case."""
        if self.screen:
            return int(self.outage[blk])
        return int(self.outage[blk - 1]) if blk > 0 else -1


def _geo_topology(g: np.random.Generator, nb: int, nl: int):
    """Near-planar random grid: buses ~U[0,1]^2, a spanning tree that joins
    each bus to one of its 3 nearest earlier buses, then extra edges from a
    random bus to one of its 6 nearest buses (duplicates rejected)."""
    if nl < nb - 1:
        raise ValueError("need at least nb-1 branches for a connected grid")
    pts = g.random((nb, 2))
    edges = set()
    for i in range(1, nb):
        d = np.hypot(pts[:i, 0] - pts[i, 0], pts[:i, 1] - pts[i, 1])
        k = min(3, i)
        near = np.argsort(d, kind="stable")[:k]
        j = int(near[g.integers(k)])
        edges.add((min(i, j), max(i, j)))
    kn = min(6, nb - 1)
    guard = 0
    while len(edges) < nl:
        i = int(g.integers(nb))
        d = np.hypot(pts[:, 0] - pts[i, 0], pts[:, 1] - pts[i, 1])
        d[i] = np.inf
        near = np.argsort(d, kind="stable")[:kn]
        j = int(near[g.integers(kn)])
        e = (min(i, j), max(i, j))
        edges.add(e)
        guard += 1
        if guard > 100 * nl:
            raise RuntimeError("could not place extra branches")
    e = np.array(sorted(edges), dtype=np.int64)
    return e[:, 0].astype(np.int32), e[:, 1].astype(np.int32)


def _uniform_topology(g: np.random.Generator, nb: int, nl: int):
    """Random spanning tree (each bus joins a uniform earlier bus) plus
    uniform random chords."""
    edges = set()
    for i in range(1, nb):
        j = int(g.integers(i))
        edges.add((j, i))
    while len(edges) < nl:
        i, j = int(g.integers(nb)), int(g.integers(nb))
        if i != j:
            edges.add((min(i, j), max(i, j)))
    e = np.array(sorted(edges), dtype=np.int64)
    return e[:, 0].astype(np.int32), e[:, 1].astype(np.int32)


def bridges(nb: int, f: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Boolean mask of bridge branches (iterative Tarjan low-link)."""
    nl = f.shape[0]
    adj = [[] for _ in range(nb)]
    for l in range(nl):
        adj[f[l]].append((t[l], l))
        adj[t[l]].append((f[l], l))
    disc = [-1] * nb
    low = [0] * nb
    isb = np.zeros(nl, dtype=bool)
    timer = 0
    for root in range(nb):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = timer
        timer += 1
        stack = [(root, -1, 0)]
        while stack:
            u, pe, it = stack[-1]
            if it < len(adj[u]):
                stack[-1] = (u, pe, it + 1)
                v, l = adj[u][it]
                if l == pe:
                    continue
                if disc[v] < 0:
                    disc[v] = low[v] = timer
                    timer += 1
                    stack.append((v, l, 0))
                else:
                    low[u] = min(low[u], disc[v])
            else:
                stack.pop()
                if stack:
                    p = stack[-1][0]
                    low[p] = min(low[p], low[u])
                    if low[u] > disc[p]:
                        isb[pe] = True
    return isb


def make_network(cfg: int, nb: int, nl: int, ng: int, ncont: int, *, pvpq: bool = False,
                 rho: float = 1e4, instance: int = 0, topology: str = "geo", screen: bool = False,
                 agc: bool = False) -> Network:
    """Draw a network.  Draw order: topology, impedances, generators, costs,
    outages, and with AGC rows the participation factors alpha_g ~
    U[0.5, 1.5] scaled to sum to 1 (drawn last, so the rest of the network
    is that of the same seed without AGC)."""
    g = rng(cfg, instance, 0)
    if topology == "geo":
        f, t = _geo_topology(g, nb, nl)
    elif topology == "uniform":
        f, t = _uniform_topology(g, nb, nl)
    else:
        raise ValueError(topology)
    r = g.uniform(0.01, 0.1, nl)
    x = g.uniform(0.05, 0.3, nl)
    gen_bus = g.choice(nb, size=ng, replace=False).astype(np.int32)
    c2 = g.uniform(0.01, 0.1, ng)
    if ncont > 0:
        cand = np.flatnonzero(~bridges(nb, f, t))
        if cand.shape[0] < ncont:
            raise ValueError(f"only {cand.shape[0]} non-bridge branches for {ncont} outages")
        outage = np.sort(g.choice(cand, size=ncont, replace=False)).astype(np.int32)
    else:
        outage = np.zeros(0, dtype=np.int32)
    if screen and ncont == 0:
        raise ValueError("screening needs contingencies")
    alpha = None
    if agc:
        if ncont == 0:
            raise ValueError("AGC rows need contingencies")
        alpha = g.uniform(0.5, 1.5, ng)
        alpha = alpha / alpha.sum()
    return Network(nb, nl, ng, f, t, r, x, gen_bus, c2, outage, bool(pvpq), float(rho), bool(screen),
                   bool(agc), alpha)


# ---------------------------------------------------------------- layout kinds

def block_kinds(net: Network, blk: int):
    """Per-position (kind, index) arrays of one block, in block-local order.
    index = bus, generator or branch number of the position."""
    nb, nl, ng = net.nb, net.nl, net.ng
    gb = set(int(b) for b in net.gen_bus)
    kinds, idx = [], []

    def add(k, ids):
        ids = list(ids)
        kinds.extend([k] * len(ids))
        idx.extend(ids)

    base_c = net.pvpq and not net.cont_block(blk)
    add(VM, [i for i in range(nb) if not (base_c and i in gb)])
    add(VA, range(nb))
    add(QG, range(ng))
    if net.single:
        add(PG, range(ng))
    if net.pvpq and net.cont_block(blk):
        for k in (NUP, NUM, SUP, SLO):
            add(k, range(ng))
    if net.agc and net.cont_block(blk):
        for k in (PGK, PIP, PIM, SPU, SPL):
            add(k, range(ng))
        add(DELTA, [0])
    nprim = len(kinds)
    add(ROW_P, range(nb))
    add(ROW_Q, range(nb))
    add(ROW_FF, range(nl))
    add(ROW_FT, range(nl))
    if net.pvpq and net.cont_block(blk):
        for k in (ROW_LIN, ROW_DUP, ROW_DLO, ROW_CUP, ROW_CLO):
            add(k, range(ng))
    if net.agc and net.cont_block(blk):
        for k in (ROW_ALIN, ROW_ADUP, ROW_ADLO, ROW_ACUP, ROW_ACLO):
            add(k, range(ng))
    return np.array(kinds, np.int32), np.array(idx, np.int32), nprim


def layout(net: Network):
    """Global (kind, index, block) arrays of length N and block offsets."""
    ks, ids, bl, offs = [], [], [], [0]
    for b in range(net.nblk):
        k, i, _ = block_kinds(net, b)
        ks.append(k)
        ids.append(i)
        bl.append(np.full(k.shape[0], b, np.int32))
        offs.append(offs[-1] + k.shape[0])
    if not net.single and not net.screen:
        ng = net.ng
        ks.append(np.full(ng, PG, np.int32))
        ids.append(np.arange(ng, dtype=np.int32))
        if net.pvpq:
            ks.append(np.full(ng, VM0, np.int32))
            ids.append(np.arange(ng, dtype=np.int32))
        nbd = ng * (2 if net.pvpq else 1)
        bl.append(np.full(nbd, -1, np.int32))
    kind = np.concatenate(ks)
    index = np.concatenate(ids)
    block = np.concatenate(bl)
    return kind, index, block, np.array(offs, np.int64)


def is_primal(kind: np.ndarray) -> np.ndarray:
    return kind < 16


# ---------------------------------------------------------------- states

def draw_point(net: Network, cfg: int, instance: int = 0, iteration: int = 0):
    """One primal/dual state in layout order.

    Returns (z, sigma): z[N] holds primal values at primal positions and
    multipliers at dual positions (the CUP/CLO and ACUP/ACLO rows hold
    nu0); sigma[N] holds the barrier diagonal at primal positions and the
    complementarity slack s at those rows (zero elsewhere).

    Draw order: primal values by kind, multipliers, nu0 and s, Sigma; a
    network with AGC rows then draws its AGC values (pgk ~ U[0, 1], the
    four complementarity variables 10^U(-8, 0), delta ~ 0.1 N(0, 1), row
    multipliers N(0, 1), nu0 10^U(-4, 2) and s 10^U(-8, 0)) after the
    rest, so that the other values stay those of the same network without
    them, except Sigma, whose draw covers every primal.
    """
    kind, _, _, _ = layout(net)
    g = rng(cfg, instance, 1000 + iteration)
    N = kind.shape[0]
    z = np.zeros(N)
    sig = np.zeros(N)

    def fill(k, sampler):
        m = kind == k
        z[m] = sampler(int(m.sum()))

    fill(VM, lambda n: g.uniform(0.95, 1.05, n))
    fill(VM0, lambda n: g.uniform(0.95, 1.05, n))
    fill(VA, lambda n: g.uniform(-0.3, 0.3, n))
    fill(QG, lambda n: g.uniform(-0.5, 0.5, n))
    fill(PG, lambda n: g.uniform(0.0, 1.0, n))
    for k in (NUP, NUM, SUP, SLO):
        fill(k, lambda n: 10.0 ** g.uniform(-8.0, 0.0, n))
    for k in (ROW_P, ROW_Q, ROW_LIN, ROW_DUP, ROW_DLO):
        fill(k, lambda n: g.standard_normal(n))
    for k in (ROW_FF, ROW_FT):
        fill(k, lambda n: g.uniform(0.0, 1.0, n))
    for k in (ROW_CUP, ROW_CLO):
        fill(k, lambda n: 10.0 ** g.uniform(-4.0, 2.0, n))
        m = kind == k
        sig[m] = 10.0 ** g.uniform(-8.0, 0.0, int(m.sum()))
    pm = is_primal(kind)
    sig[pm] = 10.0 ** g.uniform(-8.0, 8.0, int(pm.sum()))
    if net.agc:
        fill(PGK, lambda n: g.uniform(0.0, 1.0, n))
        for k in (PIP, PIM, SPU, SPL):
            fill(k, lambda n: 10.0 ** g.uniform(-8.0, 0.0, n))
        fill(DELTA, lambda n: 0.1 * g.standard_normal(n))
        for k in (ROW_ALIN, ROW_ADUP, ROW_ADLO):
            fill(k, lambda n: g.standard_normal(n))
        for k in (ROW_ACUP, ROW_ACLO):
            fill(k, lambda n: 10.0 ** g.uniform(-4.0, 2.0, n))
            m = kind == k
            sig[m] = 10.0 ** g.uniform(-8.0, 0.0, int(m.sum()))
    return z, sig


def draw_trajectory_point(net: Network, cfg: int, iteration: int, z0: np.ndarray, sig0: np.ndarray):
    """State t of a seeded trajectory: primal values move by 0.01*N(0,1)
    (clipped to the draw ranges), multipliers and Sigma are redrawn."""
    if iteration == 0:
        return z0.copy(), sig0.copy()
    kind, _, _, _ = layout(net)
    z, sig = draw_point(net, cfg, 0, iteration)
    g = rng(cfg, 0, 5000 + iteration)
    pm = is_primal(kind)
    step = z0 + 0.01 * g.standard_normal(z0.shape[0])
    lo = np.select([kind == VM, kind == VM0, kind == VA, kind == QG, kind == PG, kind == PGK, kind == DELTA],
                   [0.95, 0.95, -0.3, -0.5, 0.0, 0.0, -1.0], 1e-8)
    hi = np.select([kind == VM, kind == VM0, kind == VA, kind == QG, kind == PG, kind == PGK, kind == DELTA],
                   [1.05, 1.05, 0.3, 0.5, 1.0, 1.0, 1.0], 1.0)
    z[pm] = np.clip(step, lo, hi)[pm]
    return z, sig


def draw_rhs(N: int, nrhs: int, cfg: int, instance: int = 0, iteration: int = 0) -> np.ndarray:
    """Right-hand sides ~N(0,1), column-major [nrhs][N] as a (nrhs, N) array."""
    g = rng(cfg, instance, 9000 + iteration)
    return g.standard_normal((nrhs, N))


def draw_loads(net: Network, cfg: int, instance: int = 0, iteration: int = 0) -> np.ndarray:
    """Active loads pd ~ U[0,1] p.u. per bus (reactive loads are 0.3 pd)."""
    g = rng(cfg, instance, 7000 + iteration)
    return g.uniform(0.0, 1.0, net.nb)


def draw_directions(n: int, count: int, cfg: int, instance: int = 0) -> np.ndarray:
    """Unit-norm random directions (count, n) for finite-difference checks."""
    g = rng(cfg, instance, 8000)
    d = g.standard_normal((count, n))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def draw_ipm_point(net: Network, cfg: int, instance: int = 0, iteration: int = 0):
    """One interior point of the NCL subproblem's primal-dual IPM: a dict of
    arrays in layout order (bounds lo/hi, z, rt, s, zl, zu, y_n) and the
    loads pd.

    Bounds (the subproblem's data): vm and vm0 in [0.9, 1.1]; pg in [0, 8];
    qg in [-3, 3] in blocks without complementarity rows (in the others the
    DUP/DLO rows bound it through s_up, s_lo); the complementarity variables
    (with AGC rows also pi+, pi-, sp_up, sp_lo) >= 0; angles free, and so
    are pgk and delta (the ADUP/ADLO rows bound pgk).  Values strictly inside: z as draw_point gives it
    except the flow-row multipliers, 10^U(-3, 0) (> 0, they are inequality
    multipliers); slacks 10^U(-2, 1) on flow rows and draw_point's s on
    CUP/CLO rows; bound multipliers 10^U(-3, 1); rt ~ 1e-3 N(0, 1);
    y_n = y + 0.1 N(0, 1) at dual rows.

    Draw order: draw_point's, then flow multipliers, flow slacks, zl, zu,
    rt, y_n, loads (a stream of its own)."""
    kind, _, block, _ = layout(net)
    z, sig = draw_point(net, cfg, instance, iteration)
    g = rng(cfg, instance, 11000 + iteration)
    N = kind.shape[0]
    inf = np.inf
    lo = np.full(N, -inf)
    hi = np.full(N, inf)
    for k in (VM, VM0):
        lo[kind == k], hi[kind == k] = 0.9, 1.1
    lo[kind == PG], hi[kind == PG] = 0.0, 8.0
    comp_blk = np.array([net.pvpq and b >= 0 and net.cont_block(int(b)) for b in block])
    q = (kind == QG) & ~comp_blk
    lo[q], hi[q] = -3.0, 3.0
    for k in (NUP, NUM, SUP, SLO, PIP, PIM, SPU, SPL):
        lo[kind == k] = 0.0
    flow = (kind == ROW_FF) | (kind == ROW_FT)
    comp = (kind == ROW_CUP) | (kind == ROW_CLO) | (kind == ROW_ACUP) | (kind == ROW_ACLO)
    z[flow] = 10.0 ** g.uniform(-3.0, 0.0, int(flow.sum()))
    s = np.zeros(N)
    s[flow] = 10.0 ** g.uniform(-2.0, 1.0, int(flow.sum()))
    s[comp] = sig[comp]
    pm = is_primal(kind)
    zl = np.zeros(N)
    zu = np.zeros(N)
    a = pm & np.isfinite(lo)
    zl[a] = 10.0 ** g.uniform(-3.0, 1.0, int(a.sum()))
    a = pm & np.isfinite(hi)
    zu[a] = 10.0 ** g.uniform(-3.0, 1.0, int(a.sum()))
    rt = np.zeros(N)
    rt[~pm] = 1e-3 * g.standard_normal(int((~pm).sum()))
    y_n = np.zeros(N)
    y_n[~pm] = z[~pm] + 0.1 * g.standard_normal(int((~pm).sum()))
    pd = draw_loads(net, cfg, instance, 11000 + iteration)
    return dict(lo=lo, hi=hi, z=z, rt=rt, s=s, zl=zl, zu=zu, y_n=y_n), pd


def ncl_bounds(net: Network):
    """Bounds of the NCL subproblem's variables, layout order (the problem's
    data, as draw_ipm_point sets them): vm, vm0 in [0.9, 1.1]; pg in [0, 8];
    qg in [-3, 3] in blocks without PV/PQ rows; the complementarity
    variables >= 0; everything else free."""
    kind, _, block, _ = layout(net)
    N = kind.shape[0]
    lo = np.full(N, -np.inf)
    hi = np.full(N, np.inf)
    for k in (VM, VM0):
        lo[kind == k], hi[kind == k] = 0.9, 1.1
    lo[kind == PG], hi[kind == PG] = 0.0, 8.0
    comp_blk = np.array([net.pvpq and b >= 0 and net.cont_block(int(b)) for b in block])
    q = (kind == QG) & ~comp_blk
    lo[q], hi[q] = -3.0, 3.0
    for k in (NUP, NUM, SUP, SLO, PIP, PIM, SPU, SPL):
        lo[kind == k] = 0.0
    return lo, hi


def ncl_start(net: Network, smax2: float = 100.0, mu0: float = 0.1):
    """A strictly interior, centred start of the NCL solve, layout order
    (fixed values, no draws), at the flat voltage profile where every branch
    flow is zero: vm, vm0 = 1, va = 0, pg = 4, qg = 0; nu+, nu- = 0.01 and
    s_up, s_lo = 3 (DUP and DLO hold at qg = 0); with AGC rows pgk = 4,
    pi+, pi- = 0.01, sp_up, sp_lo = 4, delta = 0 (ALIN, ADUP and ADLO
    hold); flow-row slacks smax2 (the flow rows hold at zero flow), the
    other inequality rows' slacks 1, and every inequality row's multiplier
    mu0 / s (each product s y starts at mu0); multipliers 0 on equality
    rows; rt = 0; bound multipliers 1 where the bound is finite."""
    kind, _, _, _ = layout(net)
    lo, hi = ncl_bounds(net)
    N = kind.shape[0]
    z = np.zeros(N)
    z[(kind == VM) | (kind == VM0)] = 1.0
    z[(kind == PG) | (kind == PGK)] = 4.0
    z[(kind == NUP) | (kind == NUM) | (kind == PIP) | (kind == PIM)] = 0.01
    z[(kind == SUP) | (kind == SLO)] = 3.0
    z[(kind == SPU) | (kind == SPL)] = 4.0
    flow = (kind == ROW_FF) | (kind == ROW_FT)
    comp = (kind == ROW_CUP) | (kind == ROW_CLO) | (kind == ROW_ACUP) | (kind == ROW_ACLO)
    s = np.where(flow, smax2, np.where(comp, 1.0, 0.0))
    ineq = flow | comp
    z[ineq] = mu0 / s[ineq]
    pm = is_primal(kind)
    zl = np.where(pm & np.isfinite(lo), 1.0, 0.0)
    zu = np.where(pm & np.isfinite(hi), 1.0, 0.0)
    return dict(lo=lo, hi=hi, z=z, rt=np.zeros(N), s=s, zl=zl, zu=zu)


# ---------------------------------------------------------------- configurations

CONFIGS = {
    1: dict(nb=30, nl=41, ng=6, ncont=0, pvpq=False, rho=1e3),
    2: dict(nb=500, nl=700, ng=90, ncont=16, pvpq=False, rho=1e4),
    3: dict(nb=500, nl=700, ng=90, ncont=256, pvpq=True, rho=1e5),
    5: dict(nb=2000, nl=2800, ng=360, ncont=64, pvpq=False, rho=1e4),
    # screening of the 500-bus x 256 grid's contingencies (the same grid and
    # outages: drawn with config 3's seed), first-stage variables fixed
    6: dict(nb=500, nl=700, ng=90, ncont=256, pvpq=True, rho=1e5, screen=True, seed_cfg=3),
    # the 500-bus x 256 grid with AGC droop rows added to the PV/PQ rows of
    # every contingency block (the same grid and outages: config 3's seed)
    7: dict(nb=500, nl=700, ng=90, ncont=256, pvpq=True, rho=1e5, agc=True, seed_cfg=3),
    # screening of that grid's 256 contingencies with PV/PQ and AGC rows
    8: dict(nb=500, nl=700, ng=90, ncont=256, pvpq=True, rho=1e5, agc=True, screen=True, seed_cfg=3),
    # the 2000-bus x 64 grid (config 5's) with AGC droop rows; no PV/PQ rows,
    # which would double its 360-row border past the dense border's limit
    9: dict(nb=2000, nl=2800, ng=360, ncont=64, pvpq=False, rho=1e5, agc=True, seed_cfg=5),
}


def config_network(cfg: int, **over) -> Network:
    p = dict(CONFIGS[cfg])
    p.update(over)
    return make_network(p.get("seed_cfg", cfg), p["nb"], p["nl"], p["ng"], p["ncont"], pvpq=p["pvpq"],
                        rho=p["rho"], topology=p.get("topology", "geo"), screen=p.get("screen", False),
                        agc=p.get("agc", False))


def batched_networks(count: int = 64, cfg: int = 4):
    """Uneven instances: nb = round(exp(U[ln 118, ln 2000])), ng = round(0.18 nb),
    nl = round(1.4 nb), K ~ U{4..32}; one seed per instance."""
    nets = []
    for inst in range(count):
        g = rng(cfg, inst, 77)
        nb = int(round(math.exp(g.uniform(math.log(118), math.log(2000)))))
        ng = int(round(0.18 * nb))
        nl = int(round(1.4 * nb))
        k = int(g.integers(4, 33))
        nets.append(make_network(cfg, nb, nl, ng, k, pvpq=False, rho=1e4, instance=inst))
    return nets
