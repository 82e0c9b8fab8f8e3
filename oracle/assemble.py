"""Oracle: assembly of the regularised KKT matrix (TEST INFRASTRUCTURE ONLY).

Plain FP64 numpy.  Only tests/, the smoke check and the benchmark's CPU
baseline may import this module; the product path never does.

What is built (Section IV-B, Newton system and the blocks A, B, C):

    K = [ H + diag(delta) + Sigma ,  J^T ]
        [ J                       , -C   ]

* J = gradient of the constraints c(w) (rows below), B = [J; 0 W2 W1] with
  the complementarity rows carrying w2 in the w1 column and w1 in the w2
  column.
* H = Hessian of the Lagrangian: sum_i y_i * Hess c_i + Hess phi, plus the
  nu0 entry on each (w1, w2) off-diagonal pair of the complementarity
  products (the V0 term of block A).
* C = diag(1/rho) on every row, plus s/nu0 on the complementarity rows
  (the V0^{-1} S term of block C), plus sigma on any other dual row (the
  same term for an eliminated inequality slack; zero unless given).
* Sigma = primal barrier diagonal (W0^{-1} Xi etc.), given as an input.
* delta_i = max(0, sum_{j!=i} |H_ij| - H_ii): a per-row shift that makes
  H + diag(delta) diagonally dominant, so that K is quasi-definite at any
  (non-optimal) synthetic state.  The paper handles the same issue with
  inertia correction (Section V-C); this shift is the reading used here.

Power flow (the paper cites the textbook polar form without writing it):
branch l = (f, t) with series admittance g + jb = 1/(r + jx), status 1 (0
for the outaged branch of a contingency block), no shunts or taps.  The
flow leaving end s towards end o with theta = theta_s - theta_o is

    P_so = g v_s^2 - v_s v_o (g cos theta + b sin theta)
    Q_so = -b v_s^2 - v_s v_o (g sin theta - b cos theta)

Rows: P_i = sum of P over branch ends at bus i - sum pg at i (+ load),
Q_i likewise with qg; flow-limit rows h = P_so^2 + Q_so^2 at both ends;
complementarity rows (PV/PQ switching, eq. pvpq):
LIN_g = nu+ - nu- - v_i + v0_i, DUP_g = s_up - (qmax - qg),
DLO_g = s_lo - (qg - qmin), CUP_g = nu- * s_up, CLO_g = nu+ * s_lo.
AGC droop rows (eq. droopmpec) in a contingency block, when present: the
block's own generation pgk replaces the first-stage pg in its P balance,
and per generator ALIN_g = pi+ - pi- - pgk + pg_g + alpha_g delta (delta
the block's one adjustment variable, alpha the participation factors),
ADUP_g = sp_up - (pmax - pgk), ADLO_g = sp_lo - (pgk - pmin),
ACUP_g = pi- * sp_up, ACLO_g = pi+ * sp_lo; the last two are
complementarity rows like CUP and CLO (nu0 Hessian pair, s/nu0 in C).
Objective phi = sum_g c2_g pg_g^2.

Output: the lower triangle (row >= col) in layout order as COO arrays.
Every entry of the union pattern is emitted, also those that are exactly
zero because the branch is out of service.
"""
from __future__ import annotations

import numpy as np

# position kinds (must agree with the layout documented in gridgen)
_VM, _VA, _QG, _PG, _NUP, _NUM, _SUP, _SLO, _VM0 = range(9)


class Positions:
    """Global layout positions, computed from the network sizes alone."""

    def __init__(self, net):
        nb, nl, ng = net.nb, net.nl, net.ng
        self.nb, self.nl, self.ng = nb, nl, ng
        self.nblk = net.nblk
        self.pvpq = net.pvpq
        self.agc = bool(getattr(net, "agc", False))
        self.single = net.single
        self.screen = bool(getattr(net, "screen", False))
        isgen = np.zeros(nb, bool)
        isgen[net.gen_bus] = True
        self.vm = np.full((self.nblk, nb), -1, np.int64)
        self.va = np.zeros((self.nblk, nb), np.int64)
        self.qg = np.zeros((self.nblk, ng), np.int64)
        self.comp = np.full((self.nblk, 4, ng), -1, np.int64)      # nu+, nu-, s_up, s_lo
        self.rowP = np.zeros((self.nblk, nb), np.int64)
        self.rowQ = np.zeros((self.nblk, nb), np.int64)
        self.rowFf = np.zeros((self.nblk, nl), np.int64)
        self.rowFt = np.zeros((self.nblk, nl), np.int64)
        self.rowC = np.full((self.nblk, 5, ng), -1, np.int64)      # LIN, DUP, DLO, CUP, CLO
        self.pgk = np.full((self.nblk, ng), -1, np.int64)
        self.acomp = np.full((self.nblk, 4, ng), -1, np.int64)     # pi+, pi-, sp_up, sp_lo
        self.delta = np.full(self.nblk, -1, np.int64)
        self.rowA = np.full((self.nblk, 5, ng), -1, np.int64)      # ALIN, ADUP, ADLO, ACUP, ACLO
        self.pg = np.zeros(0 if self.screen else ng, np.int64)
        self.vm0 = np.full(ng, -1, np.int64)
        self.primal = []
        off = 0
        self.block_off = []
        for k in range(self.nblk):
            self.block_off.append(off)
            cont = self.screen or k > 0          # a contingency block
            basec = self.pvpq and not cont
            for i in range(nb):
                if basec and isgen[i]:
                    continue
                self.vm[k, i] = off
                off += 1
            self.va[k] = off + np.arange(nb)
            off += nb
            self.qg[k] = off + np.arange(ng)
            off += ng
            if self.single:
                self.pg = off + np.arange(ng)
                off += ng
            if self.pvpq and cont:
                for c in range(4):
                    self.comp[k, c] = off + np.arange(ng)
                    off += ng
            if self.agc and cont:
                self.pgk[k] = off + np.arange(ng)
                off += ng
                for c in range(4):
                    self.acomp[k, c] = off + np.arange(ng)
                    off += ng
                self.delta[k] = off
                off += 1
            nprim_end = off
            self.primal.append((self.block_off[-1], nprim_end))
            self.rowP[k] = off + np.arange(nb)
            off += nb
            self.rowQ[k] = off + np.arange(nb)
            off += nb
            self.rowFf[k] = off + np.arange(nl)
            off += nl
            self.rowFt[k] = off + np.arange(nl)
            off += nl
            if self.pvpq and cont:
                for c in range(5):
                    self.rowC[k, c] = off + np.arange(ng)
                    off += ng
            if self.agc and cont:
                for c in range(5):
                    self.rowA[k, c] = off + np.arange(ng)
                    off += ng
        self.block_off.append(off)
        if not self.single and not self.screen:
            self.pg = off + np.arange(ng)
            off += ng
            if self.pvpq:
                self.vm0 = off + np.arange(ng)
                off += ng
                # in the base block the generator-bus voltages are the border vm0
                self.vm[0, net.gen_bus] = self.vm0
        self.N = off
        self.is_primal = np.zeros(self.N, bool)
        for a, b in self.primal:
            self.is_primal[a:b] = True
        if not self.single and not self.screen:
            self.is_primal[self.block_off[-1]:] = True
        self.nborder = self.N - self.block_off[-1]


def branch_status(net, k):
    """Status of every branch in block k: 0 for the block's outaged branch
    (block k > 0 is contingency k; with screening, block k is contingency
    k + 1, there being no base block)."""
    st = np.ones(net.nl)
    if getattr(net, "screen", False):
        st[net.outage[k]] = 0.0
    elif k > 0:
        st[net.outage[k - 1]] = 0.0
    return st


def _end_derivs(g, b, vs, vo, th):
    """Value, gradient and Hessian of P_so and Q_so in the variables
    (v_s, v_o, theta_s, theta_o).  Arrays over branches."""
    c, s = np.cos(th), np.sin(th)
    A = g * c + b * s
    Bq = g * s - b * c
    n = g.shape[0]
    P = g * vs * vs - vs * vo * A
    Q = -b * vs * vs - vs * vo * Bq
    dP = np.stack([2 * g * vs - vo * A, -vs * A, vs * vo * Bq, -vs * vo * Bq], 1)
    dQ = np.stack([-2 * b * vs - vo * Bq, -vs * Bq, -vs * vo * A, vs * vo * A], 1)
    hP = np.zeros((n, 4, 4))
    hQ = np.zeros((n, 4, 4))
    # P: d2/dvs2 = 2g, d2/dvs dvo = -A, d2/dv dth = +-v Bq, d2/dth2 = +-vs vo A
    hP[:, 0, 0] = 2 * g
    hP[:, 0, 1] = hP[:, 1, 0] = -A
    pt = vo * Bq
    hP[:, 0, 2] = hP[:, 2, 0] = pt
    hP[:, 0, 3] = hP[:, 3, 0] = -pt
    pt = vs * Bq
    hP[:, 1, 2] = hP[:, 2, 1] = pt
    hP[:, 1, 3] = hP[:, 3, 1] = -pt
    tt = vs * vo * A
    hP[:, 2, 2] = hP[:, 3, 3] = tt
    hP[:, 2, 3] = hP[:, 3, 2] = -tt
    # Q: d2/dvs2 = -2b, d2/dvs dvo = -Bq, d2/dv dth = -+v A, d2/dth2 = +-vs vo Bq
    hQ[:, 0, 0] = -2 * b
    hQ[:, 0, 1] = hQ[:, 1, 0] = -Bq
    qt = -vo * A
    hQ[:, 0, 2] = hQ[:, 2, 0] = qt
    hQ[:, 0, 3] = hQ[:, 3, 0] = -qt
    qt = -vs * A
    hQ[:, 1, 2] = hQ[:, 2, 1] = qt
    hQ[:, 1, 3] = hQ[:, 3, 1] = -qt
    tt = vs * vo * Bq
    hQ[:, 2, 2] = hQ[:, 3, 3] = tt
    hQ[:, 2, 3] = hQ[:, 3, 2] = -tt
    return P, Q, dP, dQ, hP, hQ


def assemble(net, z, sigma, diag_shift=True):
    """Return (rows, cols, vals, pos) of the lower triangle of K in layout
    order (rows >= cols), one entry per (row, col) of the union pattern."""
    pos = Positions(net)
    z = np.asarray(z, np.float64)
    sigma = np.asarray(sigma, np.float64)
    nb, nl, ng = net.nb, net.nl, net.ng
    rr, cc, vv = [], [], []      # Jacobian entries (dual row, primal col)
    hr, hc, hv = [], [], []      # Hessian entries (both triangles, primal x primal)

    def jac(r, c, v):
        rr.append(np.asarray(r, np.int64).ravel())
        cc.append(np.asarray(c, np.int64).ravel())
        vv.append(np.broadcast_to(np.asarray(v, np.float64), np.shape(r)).ravel())

    def hess(r, c, v):
        hr.append(np.asarray(r, np.int64).ravel())
        hc.append(np.asarray(c, np.int64).ravel())
        hv.append(np.broadcast_to(np.asarray(v, np.float64), np.shape(r)).ravel())

    den = net.br_r ** 2 + net.br_x ** 2
    gser = net.br_r / den
    bser = -net.br_x / den
    f, t = net.br_from.astype(np.int64), net.br_to.astype(np.int64)
    for k in range(net.nblk):
        st = branch_status(net, k)
        g = st * gser
        b = st * bser
        vm_p, va_p = pos.vm[k], pos.va[k]
        v = z[vm_p]
        th = z[va_p]
        yP, yQ = z[pos.rowP[k]], z[pos.rowQ[k]]
        yFf, yFt = z[pos.rowFf[k]], z[pos.rowFt[k]]
        for (s_bus, o_bus, rowF, yF) in ((f, t, pos.rowFf[k], yFf), (t, f, pos.rowFt[k], yFt)):
            P, Q, dP, dQ, hP, hQ = _end_derivs(g, b, v[s_bus], v[o_bus], th[s_bus] - th[o_bus])
            var = np.stack([vm_p[s_bus], vm_p[o_bus], va_p[s_bus], va_p[o_bus]], 1)   # [nl,4]
            # power-balance rows of the sending bus
            jac(np.repeat(pos.rowP[k][s_bus][:, None], 4, 1), var, dP)
            jac(np.repeat(pos.rowQ[k][s_bus][:, None], 4, 1), var, dQ)
            # flow-limit row: h = P^2 + Q^2
            dh = 2 * P[:, None] * dP + 2 * Q[:, None] * dQ
            jac(np.repeat(rowF[:, None], 4, 1), var, dh)
            hh = 2 * (dP[:, :, None] * dP[:, None, :] + P[:, None, None] * hP
                      + dQ[:, :, None] * dQ[:, None, :] + Q[:, None, None] * hQ)
            W = (yP[s_bus][:, None, None] * hP + yQ[s_bus][:, None, None] * hQ
                 + yF[:, None, None] * hh)
            hess(np.repeat(var[:, :, None], 4, 2), np.repeat(var[:, None, :], 4, 1), W)
        # generator columns of the balance rows
        gb = net.gen_bus.astype(np.int64)
        jac(pos.rowQ[k][gb], pos.qg[k], -1.0)
        agc_blk = pos.agc and (k > 0 or pos.screen)
        if agc_blk:                              # the block's own generation
            jac(pos.rowP[k][gb], pos.pgk[k], -1.0)
        elif not pos.screen:                     # screening: pg fixed, no column
            jac(pos.rowP[k][gb], pos.pg, -1.0)
        if agc_blk:
            pip, pim, spu, spl = pos.acomp[k]
            pgk = pos.pgk[k]
            alin, adup, adlo, acup, aclo = pos.rowA[k]
            jac(alin, pip, 1.0)
            jac(alin, pim, -1.0)
            jac(alin, pgk, -1.0)
            if not pos.screen:                   # screening: pg fixed, no column
                jac(alin, pos.pg, 1.0)
            jac(alin, np.full(ng, pos.delta[k]), net.gen_alpha)
            jac(adup, spu, 1.0)
            jac(adup, pgk, 1.0)
            jac(adlo, spl, 1.0)
            jac(adlo, pgk, -1.0)
            jac(acup, pim, z[spu])
            jac(acup, spu, z[pim])
            jac(aclo, pip, z[spl])
            jac(aclo, spl, z[pip])
            hess(pim, spu, z[acup])
            hess(spu, pim, z[acup])
            hess(pip, spl, z[aclo])
            hess(spl, pip, z[aclo])
        if net.pvpq and (k > 0 or pos.screen):
            nup, num, sup, slo = pos.comp[k]
            lin, dup, dlo, cup, clo = pos.rowC[k]
            jac(lin, nup, 1.0)
            jac(lin, num, -1.0)
            jac(lin, vm_p[gb], -1.0)
            if not pos.screen:                   # screening: vm0 fixed, no column
                jac(lin, pos.vm0, 1.0)
            jac(dup, sup, 1.0)
            jac(dup, pos.qg[k], 1.0)
            jac(dlo, slo, 1.0)
            jac(dlo, pos.qg[k], -1.0)
            jac(cup, num, z[sup])
            jac(cup, sup, z[num])
            jac(clo, nup, z[slo])
            jac(clo, slo, z[nup])
            # nu0 on the (w1, w2) off-diagonal pairs
            hess(num, sup, z[cup])
            hess(sup, num, z[cup])
            hess(nup, slo, z[clo])
            hess(slo, nup, z[clo])
    # objective (screening: pg fixed, no objective term in the variables)
    if not pos.screen:
        hess(pos.pg, pos.pg, 2.0 * net.gen_c2)
    # every primal keeps its diagonal in the pattern
    prim = np.flatnonzero(pos.is_primal)
    hess(prim, prim, 0.0)

    N = pos.N
    hr = np.concatenate(hr)
    hc = np.concatenate(hc)
    hv = np.concatenate(hv)
    # sum duplicate Hessian contributions per (row, col)
    key = hr * N + hc
    uk, inv = np.unique(key, return_inverse=True)
    hsum = np.zeros(uk.shape[0])
    np.add.at(hsum, inv, hv)
    Hr, Hc = uk // N, uk % N
    # diagonal shift
    offd = Hr != Hc
    rowabs = np.zeros(N)
    np.add.at(rowabs, Hr[offd], np.abs(hsum[offd]))
    hdiag = np.zeros(N)
    dmask = ~offd
    hdiag[Hr[dmask]] = hsum[dmask]
    delta = np.maximum(0.0, rowabs - hdiag) if diag_shift else np.zeros(N)
    hsum = hsum.copy()
    hsum[dmask] += delta[Hr[dmask]] + sigma[Hr[dmask]]

    jr = np.concatenate(rr)
    jcol = np.concatenate(cc)
    jv = np.concatenate(vv)
    key = jr * N + jcol
    uk, inv = np.unique(key, return_inverse=True)
    jsum = np.zeros(uk.shape[0])
    np.add.at(jsum, inv, jv)
    Jr, Jc = uk // N, uk % N

    # dual diagonal: -1/rho, -(1/rho + s/nu0) on complementarity rows (CUP,
    # CLO, ACUP, ACLO), and
    # -(1/rho + sigma) on any other row with a nonzero sigma (an eliminated
    # inequality slack, block C)
    duals = np.flatnonzero(~pos.is_primal)
    ddiag = np.full(duals.shape[0], -1.0 / net.rho)
    cmask = np.zeros(duals.shape[0], bool)
    c0 = 0 if pos.screen else 1
    crow = np.concatenate([pos.rowC[c0:, 3:5].ravel() if pos.pvpq else np.zeros(0, np.int64),
                           pos.rowA[c0:, 3:5].ravel() if pos.agc else np.zeros(0, np.int64)])
    if crow.size:
        cmask = np.isin(duals, crow)
        ddiag[cmask] -= sigma[duals[cmask]] / z[duals[cmask]]
    ddiag[~cmask] -= sigma[duals[~cmask]]

    low = Hr >= Hc
    rows = np.concatenate([Hr[low], Jr, duals])
    cols = np.concatenate([Hc[low], Jc, duals])
    vals = np.concatenate([hsum[low], jsum, ddiag])
    # Jacobian rows follow all primal columns only when dual index > primal index;
    # in this layout a block's rows follow its primals, but border primals come
    # last, so entries (dual row, border col) lie in the upper triangle: mirror them.
    up = rows < cols
    rows[up], cols[up] = cols[up], rows[up]
    order = np.lexsort((rows, cols))
    return rows[order], cols[order], vals[order], pos


def to_dense(rows, cols, vals, N):
    K = np.zeros((N, N))
    K[rows, cols] = vals
    K[cols, rows] = vals
    return K


def to_csc_full(rows, cols, vals, N):
    """Full symmetric CSC (scipy) from the lower triangle."""
    import scipy.sparse as sp
    off = rows != cols
    r = np.concatenate([rows, cols[off]])
    c = np.concatenate([cols, rows[off]])
    v = np.concatenate([vals, vals[off]])
    return sp.csc_matrix((v, (r, c)), shape=(N, N))


def delta_shift(net, z, sigma):
    """The diagonal shift delta (for tests): K11 diagonal minus H diagonal minus Sigma."""
    r0, c0, v0, pos = assemble(net, z, np.zeros_like(sigma), diag_shift=False)
    r1, c1, v1, _ = assemble(net, z, np.zeros_like(sigma), diag_shift=True)
    d = np.zeros(pos.N)
    m = r1 == c1
    d[r1[m]] += v1[m]
    d[r0[r0 == c0]] -= v0[r0 == c0]
    return d
