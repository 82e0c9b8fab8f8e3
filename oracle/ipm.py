"""Oracle: one primal-dual interior-point step of the NCL subproblem (TEST
INFRASTRUCTURE ONLY).  Plain FP64 numpy; only tests/, the smoke check and
the benchmark's CPU-baseline leg may import it, the product path never does.

The subproblem (Section IV-A, eq. (nclsubpb)) at outer iteration n, for the
corrective SCOPF of Section II-B with the PV/PQ rows of eq. (pvpq):

    min  phi(w) + lam_n' r + nu0_n' t + rho/2 (|r|^2 + |t|^2)
    s.t. c_E(w) - r_E = 0                   (balance, LIN, DUP, DLO rows)
         c_I(w) + s - r_I = 0,  s >= 0      (flow rows h <= smax2, and the
                                             CUP/CLO rows W1 W2 e <= t)
         lo <= w <= hi                      (finite entries only)

phi(w) = sum_g c2_g pg_g^2 + (eps/2) sum_k va_{k,0}^2 (the second term fixes
each block's angle reference, as in the dispatch map).  A screening network
(eq. (screening)) fixes the first-stage pg0 and vm0, given as data: its
blocks are the contingencies' feasibility problems (eq. (feaspb) once NCL
drives r, t to zero or to their least violation), phi keeps only the angle
term.  Every dual row
carries one regularisation variable: r on the rows of c(w), t on the
complementarity rows (both called rt here, one vector over the dual rows).
The slack of an inequality row has the row multiplier as its own bound
multiplier, as the paper writes S V0 = mu e for the complementarity rows;
the flow rows follow the same form.

Constraint values c(w) (loads pd on P rows, qd_ratio pd on Q rows):
    P_i = sum of P_so over branch ends at bus i - pg at i + pd_i
    Q_i = sum of Q_so over branch ends at bus i - qg at i + qd_ratio pd_i
    F   = P_so^2 + Q_so^2 - smax2               (each branch end)
    LIN = nu+ - nu- - vm_i + vm0_g,   DUP = s_up - (qmax - qg),
    DLO = s_lo - (qg + qmax),         CUP = nu- s_up,   CLO = nu+ s_lo,
and with AGC rows (eq. (droopmpec); the block's own pgk then takes the
place of pg in its P rows, and pmin = 0, the lower bound of pg):
    ALIN = pi+ - pi- - pgk + pg + alpha delta,   ADUP = sp_up - (pmax - pgk),
    ADLO = sp_lo - (pgk - pmin),   ACUP = pi- sp_up,   ACLO = pi+ sp_lo.
ACUP and ACLO are inequality rows like CUP and CLO.

Barrier form of the KKT conditions (eq. (kktncl); the complementarity
conditions replaced by their mu-perturbed products as Section IV-B
describes), unknowns u = (w, y, rt, s, zl, zu):

    G_w  = grad phi + J' y - zl + zu        G_rt = y_n + rho rt - y
    G_y  = c(w) + [I] s - rt                G_s  = s y - mu        (I rows)
    G_zl = (w - lo) zl - mu                 G_zu = (hi - w) zu - mu

A Newton step on G, with zl, zu, s and rt eliminated, is the reduced system
of eq. (newtonsystem), K [dw; dy] = [r1; r2], with K the assembled KKT matrix
(no diagonal shift) for

    Sigma = zl / (w - lo) + zu / (hi - w)  (+ eps at the reference angles)
    sigma at CUP/CLO rows = s   (the assembly takes s / nu0 there),
    sigma at flow rows    = s / y,

and, derived by eliminating in the order zl, zu, s, rt (the paper's printed
recovery formulas carry the opposite sign on the mu terms and on d lam; the
signs here follow from linearising G):

    r1 = -(grad phi + J' y) + mu / (w - lo) - mu / (hi - w)
    r2 = -c(w) + (y - y_n) / rho - [I] mu / y
    d rt = (dy + y - y_n - rho rt) / rho
    d s  = mu / y - s - (s / y) dy                          (I rows)
    d zl = (mu - (w - lo) zl - zl dw) / (w - lo)
    d zu = (mu - (hi - w) zu + zu dw) / (hi - w).

Every function accepts complex inputs where it is analytic, so a complex-
step Jacobian of ``kkt_residual`` gives the unreduced Newton matrix exactly.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import assemble as _asm


@dataclass
class Problem:
    """Data of the subproblem at one outer iteration and barrier value."""
    pd: np.ndarray                      # [nb] active loads
    lo: np.ndarray                      # [N] lower bounds at primal positions (-inf: none)
    hi: np.ndarray                      # [N] upper bounds at primal positions (+inf: none)
    y_n: np.ndarray                     # [N] multiplier estimates lam_n, nu0_n at the dual rows
    mu: float = 0.1
    rho: float = 1e5
    qd_ratio: float = 0.3
    qmax: float = 3.0
    pmax: float = 8.0
    smax2: float = 100.0
    eps: float = 1.0
    pg0: np.ndarray = None              # [ng] fixed first-stage pg (screening networks)
    vm0: np.ndarray = None              # [ng] fixed first-stage PV voltages (screening with PV/PQ rows)


@dataclass
class State:
    """One primal-dual point; every array has length N in layout order."""
    z: np.ndarray                       # w at primal positions, y = (lam, nu0) at dual rows
    rt: np.ndarray                      # r (rows of c) or t (CUP/CLO rows) at dual rows
    s: np.ndarray                       # slack at inequality rows
    zl: np.ndarray                      # lower-bound multipliers at primal positions
    zu: np.ndarray                      # upper-bound multipliers at primal positions

    def copy(self):
        return State(*(np.array(a) for a in (self.z, self.rt, self.s, self.zl, self.zu)))


@dataclass
class Masks:
    primal: np.ndarray
    dual: np.ndarray
    ineq: np.ndarray                    # flow rows and CUP/CLO (ACUP/ACLO) rows
    comp: np.ndarray                    # CUP/CLO (ACUP/ACLO) rows
    flow: np.ndarray
    has_lo: np.ndarray
    has_hi: np.ndarray
    vref: np.ndarray                    # reference-angle positions (bus 0 of every block)
    pos: object = field(repr=False, default=None)


def masks(net, prob: Problem) -> Masks:
    if getattr(net, "screen", False) and (prob.pg0 is None or (net.pvpq and prob.vm0 is None)):
        raise ValueError("a screening network needs the fixed first-stage values pg0 (and vm0)")
    pos = _asm.Positions(net)
    N = pos.N
    primal = pos.is_primal.copy()
    flow = np.zeros(N, bool)
    comp = np.zeros(N, bool)
    vref = np.zeros(N, bool)
    for k in range(net.nblk):
        flow[pos.rowFf[k]] = True
        flow[pos.rowFt[k]] = True
        vref[pos.va[k][0]] = True
        for rc in (pos.rowC[k], pos.rowA[k]):
            if rc[3][0] >= 0:
                comp[rc[3]] = True
                comp[rc[4]] = True
    lo, hi = np.asarray(prob.lo), np.asarray(prob.hi)
    return Masks(primal=primal, dual=~primal, ineq=flow | comp, comp=comp, flow=flow,
                 has_lo=primal & np.isfinite(lo), has_hi=primal & np.isfinite(hi), vref=vref, pos=pos)


def _flows(g, b, vs, vo, th):
    """P_so, Q_so leaving end s and their gradients in (v_s, v_o, th_s, th_o)."""
    c, s = np.cos(th), np.sin(th)
    A = g * c + b * s
    Bq = g * s - b * c
    P = g * vs * vs - vs * vo * A
    Q = -b * vs * vs - vs * vo * Bq
    dP = np.stack([2 * g * vs - vo * A, -vs * A, vs * vo * Bq, -vs * vo * Bq], 1)
    dQ = np.stack([-2 * b * vs - vo * Bq, -vs * Bq, -vs * vo * A, vs * vo * A], 1)
    return P, Q, dP, dQ


def _series(net):
    den = net.br_r ** 2 + net.br_x ** 2
    return net.br_r / den, -net.br_x / den


def constraints(net, z, prob: Problem, m: Masks = None):
    """c(w) at every dual row (zero at primal positions)."""
    m = m or masks(net, prob)
    pos = m.pos
    c = np.zeros(pos.N, np.result_type(z, np.float64))
    gser, bser = _series(net)
    f, t = net.br_from.astype(np.int64), net.br_to.astype(np.int64)
    gb = net.gen_bus.astype(np.int64)
    screen = pos.screen
    pg = np.asarray(prob.pg0, np.float64) if screen else z[pos.pg]
    vm0 = (np.asarray(prob.vm0, np.float64) if screen else z[pos.vm0]) if net.pvpq else None
    for k in range(net.nblk):
        st = _asm.branch_status(net, k)
        g, b = st * gser, st * bser
        v, th = z[pos.vm[k]], z[pos.va[k]]
        Pinj = np.zeros(net.nb, c.dtype)
        Qinj = np.zeros(net.nb, c.dtype)
        for s_bus, o_bus, rowF in ((f, t, pos.rowFf[k]), (t, f, pos.rowFt[k])):
            P, Q, _, _ = _flows(g, b, v[s_bus], v[o_bus], th[s_bus] - th[o_bus])
            np.add.at(Pinj, s_bus, P)
            np.add.at(Qinj, s_bus, Q)
            c[rowF] = P * P + Q * Q - prob.smax2
        qg = z[pos.qg[k]]
        agc = pos.pgk[k][0] >= 0
        pgk = z[pos.pgk[k]] if agc else pg
        np.add.at(Pinj, gb, -pgk)
        np.add.at(Qinj, gb, -qg)
        c[pos.rowP[k]] = Pinj + prob.pd
        c[pos.rowQ[k]] = Qinj + prob.qd_ratio * prob.pd
        lin, dup, dlo, cup, clo = pos.rowC[k]
        if lin[0] >= 0:
            nup, num, sup, slo = (z[i] for i in pos.comp[k])
            c[lin] = nup - num - v[gb] + vm0
            c[dup] = sup - (prob.qmax - qg)
            c[dlo] = slo - (qg + prob.qmax)
            c[cup] = num * sup
            c[clo] = nup * slo
        if agc:
            alin, adup, adlo, acup, aclo = pos.rowA[k]
            pip, pim, spu, spl = (z[i] for i in pos.acomp[k])
            c[alin] = pip - pim - pgk + pg + net.gen_alpha * z[pos.delta[k]]
            c[adup] = spu - (prob.pmax - pgk)
            c[adlo] = spl - pgk
            c[acup] = pim * spu
            c[aclo] = pip * spl
    return c


def objective(net, z, prob: Problem, m: Masks = None):
    m = m or masks(net, prob)
    pos = m.pos
    va0 = z[m.vref]
    f = 0.5 * prob.eps * np.sum(va0 * va0)
    if pos.screen:                       # pg fixed: the feasibility problem has no cost term
        return f
    pg = z[pos.pg]
    return np.sum(net.gen_c2 * pg * pg) + f


def grad_lagrangian(net, z, prob: Problem, m: Masks = None):
    """grad phi + J' y at every primal position (zero at dual rows), from the
    derivative formulas of c(w)."""
    m = m or masks(net, prob)
    pos = m.pos
    gL = np.zeros(pos.N, np.result_type(z, np.float64))
    gser, bser = _series(net)
    f, t = net.br_from.astype(np.int64), net.br_to.astype(np.int64)
    gb = net.gen_bus.astype(np.int64)
    screen = pos.screen
    if not screen:
        gL[pos.pg] += 2.0 * net.gen_c2 * z[pos.pg]
    gL[m.vref] += prob.eps * z[m.vref]
    for k in range(net.nblk):
        st = _asm.branch_status(net, k)
        g, b = st * gser, st * bser
        vm_p, va_p = pos.vm[k], pos.va[k]
        v, th = z[vm_p], z[va_p]
        yP, yQ = z[pos.rowP[k]], z[pos.rowQ[k]]
        for s_bus, o_bus, rowF in ((f, t, pos.rowFf[k]), (t, f, pos.rowFt[k])):
            P, Q, dP, dQ = _flows(g, b, v[s_bus], v[o_bus], th[s_bus] - th[o_bus])
            yF = z[rowF]
            dh = 2.0 * P[:, None] * dP + 2.0 * Q[:, None] * dQ
            var = np.stack([vm_p[s_bus], vm_p[o_bus], va_p[s_bus], va_p[o_bus]], 1)
            np.add.at(gL, var, yP[s_bus][:, None] * dP + yQ[s_bus][:, None] * dQ + yF[:, None] * dh)
        np.add.at(gL, pos.qg[k], -yQ[gb])
        agc = pos.pgk[k][0] >= 0
        if agc:
            np.add.at(gL, pos.pgk[k], -yP[gb])
        elif not screen:
            np.add.at(gL, pos.pg, -yP[gb])
        if agc:
            alin, adup, adlo, acup, aclo = pos.rowA[k]
            ipip, ipim, ispu, ispl = pos.acomp[k]
            ya, yu, yd, ycu, ycl = z[alin], z[adup], z[adlo], z[acup], z[aclo]
            np.add.at(gL, ipip, ya + ycl * z[ispl])
            np.add.at(gL, ipim, -ya + ycu * z[ispu])
            np.add.at(gL, ispu, yu + ycu * z[ipim])
            np.add.at(gL, ispl, yd + ycl * z[ipip])
            np.add.at(gL, pos.pgk[k], -ya + yu - yd)
            if not screen:
                np.add.at(gL, pos.pg, ya)
            gL[pos.delta[k]] += np.sum(net.gen_alpha * ya)
        lin, dup, dlo, cup, clo = pos.rowC[k]
        if lin[0] >= 0:
            inup, inum, isup, islo = pos.comp[k]
            yl, yu, yd, ycu, ycl = z[lin], z[dup], z[dlo], z[cup], z[clo]
            np.add.at(gL, inup, yl + ycl * z[islo])
            np.add.at(gL, inum, -yl + ycu * z[isup])
            np.add.at(gL, isup, yu + ycu * z[inum])
            np.add.at(gL, islo, yd + ycl * z[inup])
            np.add.at(gL, vm_p[gb], -yl)
            if not screen:
                np.add.at(gL, pos.vm0, yl)
            np.add.at(gL, pos.qg[k], yu - yd)
    gL[m.dual] = 0.0
    return gL


# ---------------------------------------------------------------- the unreduced system

class Unknowns:
    """Index sets of u = (w, y, rt, s, zl, zu) inside one flat vector."""

    def __init__(self, m: Masks):
        self.iw = np.flatnonzero(m.primal)
        self.iy = np.flatnonzero(m.dual)
        self.irt = self.iy
        self.i_s = np.flatnonzero(m.ineq)
        self.izl = np.flatnonzero(m.has_lo)
        self.izu = np.flatnonzero(m.has_hi)
        sizes = [len(self.iw), len(self.iy), len(self.irt), len(self.i_s), len(self.izl), len(self.izu)]
        self.off = np.concatenate([[0], np.cumsum(sizes)])
        self.n = int(self.off[-1])

    def pack(self, st: State):
        parts = [st.z[self.iw], st.z[self.iy], st.rt[self.irt], st.s[self.i_s], st.zl[self.izl], st.zu[self.izu]]
        return np.concatenate(parts)

    def unpack(self, u, N):
        dt = u.dtype
        z, rt, s, zl, zu = (np.zeros(N, dt) for _ in range(5))
        o = self.off
        z[self.iw] = u[o[0]:o[1]]
        z[self.iy] = u[o[1]:o[2]]
        rt[self.irt] = u[o[2]:o[3]]
        s[self.i_s] = u[o[3]:o[4]]
        zl[self.izl] = u[o[4]:o[5]]
        zu[self.izu] = u[o[5]:o[6]]
        return State(z, rt, s, zl, zu)


def kkt_residual(net, st: State, prob: Problem, m: Masks = None):
    """G(u), its equations ordered to pair with the unknowns of ``Unknowns``
    (each eliminated group by the equation that eliminates it):
    (G_w, G_y, G_rt, G_s, G_zl, G_zu)."""
    m = m or masks(net, prob)
    U = Unknowns(m)
    z = st.z
    lo, hi = np.asarray(prob.lo), np.asarray(prob.hi)
    gL = grad_lagrangian(net, z, prob, m)
    c = constraints(net, z, prob, m)
    Gw = (gL - st.zl + st.zu)[U.iw]
    Gy = (c + np.where(m.ineq, st.s, 0.0) - st.rt)[U.iy]
    Grt = (prob.y_n + prob.rho * st.rt - z)[U.irt]
    Gs = (st.s * z - prob.mu)[U.i_s]
    Gzl = (z[U.izl] - lo[U.izl]) * st.zl[U.izl] - prob.mu
    Gzu = (hi[U.izu] - z[U.izu]) * st.zu[U.izu] - prob.mu
    return np.concatenate([Gw, Gy, Grt, Gs, Gzl, Gzu])


# ---------------------------------------------------------------- the reduced step

def sigma(net, st: State, prob: Problem, m: Masks = None):
    """The sigma the assembly takes for the Newton matrix of this state."""
    m = m or masks(net, prob)
    z = st.z
    lo, hi = np.asarray(prob.lo), np.asarray(prob.hi)
    sg = np.zeros(z.shape[0])
    a = m.has_lo
    sg[a] += st.zl[a] / (z[a] - lo[a])
    a = m.has_hi
    sg[a] += st.zu[a] / (hi[a] - z[a])
    sg[m.vref] += prob.eps
    sg[m.comp] = st.s[m.comp]
    sg[m.flow] = st.s[m.flow] / z[m.flow]
    return sg


def reduced_rhs(net, st: State, prob: Problem, m: Masks = None):
    """(r1, r2) of the reduced Newton system, one vector in layout order."""
    m = m or masks(net, prob)
    z = st.z
    lo, hi = np.asarray(prob.lo), np.asarray(prob.hi)
    r = np.zeros(z.shape[0])
    gL = grad_lagrangian(net, z, prob, m)
    r[m.primal] = -gL[m.primal]
    a = m.has_lo
    r[a] += prob.mu / (z[a] - lo[a])
    a = m.has_hi
    r[a] -= prob.mu / (hi[a] - z[a])
    c = constraints(net, z, prob, m)
    d = m.dual
    r[d] = -c[d] + (z[d] - prob.y_n[d]) / prob.rho
    r[m.ineq] -= prob.mu / z[m.ineq]
    return r


def recover(net, st: State, prob: Problem, dz, m: Masks = None) -> State:
    """The eliminated directions from (dw, dy) = dz: a State of directions
    (its z is dz itself)."""
    m = m or masks(net, prob)
    z = st.z
    lo, hi = np.asarray(prob.lo), np.asarray(prob.hi)
    N = z.shape[0]
    drt, ds, dzl, dzu = (np.zeros(N) for _ in range(4))
    d = m.dual
    drt[d] = (dz[d] + z[d] - prob.y_n[d] - prob.rho * st.rt[d]) / prob.rho
    q = m.ineq
    ds[q] = prob.mu / z[q] - st.s[q] - st.s[q] / z[q] * dz[q]
    a = m.has_lo
    gap = z[a] - lo[a]
    dzl[a] = (prob.mu - gap * st.zl[a] - st.zl[a] * dz[a]) / gap
    a = m.has_hi
    gap = hi[a] - z[a]
    dzu[a] = (prob.mu - gap * st.zu[a] + st.zu[a] * dz[a]) / gap
    return State(np.array(dz, np.float64), drt, ds, dzl, dzu)


def newton_matrix(net, st: State, prob: Problem, dw=0.0, m: Masks = None):
    """Lower CSC (colptr, rowind, vals) of the reduced matrix: the assembly
    without the diagonal-dominance shift, at this state's sigma, with dw
    added on the primal diagonal."""
    from . import lower_csc
    m = m or masks(net, prob)
    sg = sigma(net, st, prob, m)
    sg[m.primal] += dw
    r, c, v, pos = _asm.assemble(net, st.z, sg, diag_shift=False)
    return lower_csc(r, c, v, pos.N)


# the primal-shift sequence of the inertia correction: the exact matrix
# first; then from a third of the last accepted shift (or 1e-4), growing x8
# below 1e12 (the same rule as the dispatch map's Newton method)
SHIFT_FIRST, SHIFT_GROW, SHIFT_SHRINK, SHIFT_MAX = 1e-4, 8.0, 3.0, 1e12


def shift_sequence(dw_last):
    yield 0.0
    dw = dw_last / SHIFT_SHRINK if dw_last > 0 else SHIFT_FIRST
    while dw < SHIFT_MAX:
        yield dw
        dw *= SHIFT_GROW


def inertia_ok(inertia, nprimal, N):
    npos, nneg, nzero = inertia
    return npos == nprimal and nneg == N - nprimal and nzero == 0


def inertia_correction(net, st: State, prob: Problem, dw_last=0.0, m: Masks = None, factor=None):
    """Factor the reduced matrix with the smallest shift of the sequence
    whose LDL^T has the inertia (n primal positive, m dual negative)
    (Section V-C: extra factorisations when the inertia is wrong).
    Returns (dw, number of factorisations, Factor, (colptr, rowind, vals))."""
    from . import Factor
    m = m or masks(net, prob)
    nprimal = int(m.primal.sum())
    N = m.primal.shape[0]
    F = factor or Factor.from_network(net)
    nfac = 0
    for dw in shift_sequence(dw_last):
        cp, ri, v = newton_matrix(net, st, prob, dw, m)
        F.factor(cp, ri, v)
        nfac += 1
        if inertia_ok(F.inertia, nprimal, N):
            return dw, nfac, F, (cp, ri, v)
    raise RuntimeError("no primal shift below 1e12 gives the inertia")


def step(net, st: State, prob: Problem, dw_last=0.0, factor=None):
    """One Newton direction of the IPM: (direction State, dw, factorisations)."""
    m = masks(net, prob)
    dw, nfac, F, _ = inertia_correction(net, st, prob, dw_last, m, factor)
    r = reduced_rhs(net, st, prob, m)
    dz = F.solve(r)
    return recover(net, st, prob, dz, m), dw, nfac
