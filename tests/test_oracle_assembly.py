"""Pins for the oracle's KKT assembly.

* Jacobian and Hessian against exact hyper-dual derivatives of the
  constraints and Lagrangian written in the bus-admittance / complex-power
  form (tests/_hd.py), on a single-block network and on a small
  multi-block network with PV/PQ complementarity rows and a border.
* Invariants of the power-flow equations: angle-shift invariance, the
  lossless case, Euler homogeneity in the voltage magnitudes.
* A two-bus closed form derived by hand.
* Regularisation: the dual diagonal is -1/rho (and -(1/rho + s/nu0) on
  complementarity rows), the shifted (1,1) block is positive definite, so
  K is quasi-definite with inertia (n, m) (Section IV-B, blocks A, B, C).
"""
import numpy as np
import pytest

import gridgen as G
from oracle import assemble as A
from tests import _hd


def small_pvpq():
    return G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5)


def small_agc(pvpq=True):
    return G.make_network(99, 9, 12, 3, 2, pvpq=pvpq, rho=1e5, agc=True)


def _positions(net):
    kind, index, block, _ = G.layout(net)
    pm = {}
    for p, (k, i, b) in enumerate(zip(kind, index, block)):
        pm[(int(k), int(b), int(i))] = p
    gen_of_bus = {int(b): g for g, b in enumerate(net.gen_bus)}
    bb = 0 if net.single else -1

    def var_pos(name, k, i):
        if name == "vm":
            if net.pvpq and k == 0 and i in gen_of_bus:
                return pm[(G.VM0, -1, gen_of_bus[i])]
            return pm[(G.VM, k, i)]
        if name == "pg":
            return pm[(G.PG, bb, i)]
        if name == "vm0":
            return pm[(G.VM0, -1, i)]
        code = dict(va=G.VA, qg=G.QG, nup=G.NUP, num=G.NUM, sup=G.SUP, slo=G.SLO, pgk=G.PGK, pip=G.PIP,
                    pim=G.PIM, spu=G.SPU, spl=G.SPL, delta=G.DELTA)[name]
        return pm[(code, k, i)]

    def row_pos(key):
        name, k, i = key
        code = dict(P=G.ROW_P, Q=G.ROW_Q, Ff=G.ROW_FF, Ft=G.ROW_FT, LIN=G.ROW_LIN, DUP=G.ROW_DUP,
                    DLO=G.ROW_DLO, CUP=G.ROW_CUP, CLO=G.ROW_CLO, ALIN=G.ROW_ALIN, ADUP=G.ROW_ADUP,
                    ADLO=G.ROW_ADLO, ACUP=G.ROW_ACUP, ACLO=G.ROW_ACLO)[name]
        return pm[(code, k, i)]

    return kind, var_pos, row_pos


def hd_jacobian_hessian(net, z):
    kind, var_pos, row_pos = _positions(net)
    prim = np.flatnonzero(G.is_primal(kind))
    N = kind.shape[0]
    # Jacobian: e1 along every primal at once (vectorised over the primal list)
    sel = {p: (prim == p).astype(float) for p in prim}

    def var_j(name, k, i):
        p = var_pos(name, k, i)
        return _hd.HD(z[p], sel[p], 0.0, 0.0)

    rows, _ = _hd.constraints_and_objective(net, var_j, None)
    J = np.zeros((N, N))
    for key, val in rows:
        J[row_pos(key), prim] = np.broadcast_to(val.b, prim.shape)
    # Hessian of the Lagrangian: every pair (a, b) of primals
    ia, ib = np.triu_indices(prim.shape[0])
    pa, pb = prim[ia], prim[ib]

    def var_h(name, k, i):
        p = var_pos(name, k, i)
        return _hd.HD(z[p], (pa == p).astype(float), (pb == p).astype(float), 0.0)

    rows, obj = _hd.constraints_and_objective(net, var_h, None)
    lag = obj
    for key, val in rows:
        lag = lag + z[row_pos(key)] * val
    H = np.zeros((N, N))
    H[pa, pb] = np.broadcast_to(lag.d, pa.shape)
    H[pb, pa] = H[pa, pb]
    return J, H, prim


NETS = {
    "single": lambda: (G.config_network(1), 1),
    "pvpq": lambda: (small_pvpq(), 99),
    "agc": lambda: (small_agc(), 99),
    "agc_plain": lambda: (small_agc(pvpq=False), 99),
}


@pytest.mark.parametrize("which", list(NETS))
def test_jacobian_hessian_exact(which):
    net, cfg = NETS[which]()
    z, sig = G.draw_point(net, cfg)
    r, c, v, pos = A.assemble(net, z, np.zeros_like(sig), diag_shift=False)
    K = A.to_dense(r, c, v, pos.N)
    J, H, prim = hd_jacobian_hessian(net, z)
    isp = pos.is_primal
    Kh = K[np.ix_(isp, isp)]
    Kj = K[np.ix_(~isp, isp)]
    scale = max(1.0, np.abs(H).max())
    assert np.abs(Kh - H[np.ix_(isp, isp)]).max() <= 1e-13 * scale
    assert np.abs(Kj - J[np.ix_(~isp, isp)]).max() <= 1e-13 * max(1.0, np.abs(J).max())


@pytest.mark.parametrize("which", ["pvpq", "agc"])
def test_dual_diagonal_and_comp_rows(which):
    net, _ = NETS[which]()
    z, sig = G.draw_point(net, 99)
    r, c, v, pos = A.assemble(net, z, sig)
    K = A.to_dense(r, c, v, pos.N)
    kind, _, _, _ = G.layout(net)
    d = np.diag(K)
    for k in range(16, 30):
        m = kind == k
        if k in (G.ROW_CUP, G.ROW_CLO, G.ROW_ACUP, G.ROW_ACLO):
            np.testing.assert_allclose(d[m], -(1.0 / net.rho + sig[m] / z[m]), rtol=1e-15)
        else:
            np.testing.assert_allclose(d[m], -1.0 / net.rho, rtol=1e-15)
    # dual-dual off-diagonals are zero (C is diagonal)
    dm = ~pos.is_primal
    Kdd = K[np.ix_(dm, dm)]
    assert np.count_nonzero(Kdd - np.diag(np.diag(Kdd))) == 0


def test_angle_shift_invariance():
    """P and Q depend on angle differences only: J_theta * 1 = 0 per block."""
    net = small_pvpq()
    z, sig = G.draw_point(net, 99)
    r, c, v, pos = A.assemble(net, z, sig)
    K = A.to_dense(r, c, v, pos.N)
    for k in range(net.nblk):
        rows = np.concatenate([pos.rowP[k], pos.rowQ[k], pos.rowFf[k], pos.rowFt[k]])
        s = K[np.ix_(rows, pos.va[k])].sum(axis=1)
        assert np.abs(s).max() <= 1e-12 * max(1.0, np.abs(K[np.ix_(rows, pos.va[k])]).max())


def test_lossless_and_euler():
    """r = 0: total active injection is identically zero, so the P-row sums of
    the vm and va columns vanish.  Euler: P_i(v) is homogeneous of degree 2
    in the magnitudes, so sum_j v_j dP_i/dv_j = 2 P_i."""
    net = G.config_network(1)
    net.br_r = np.zeros_like(net.br_r)
    z, sig = G.draw_point(net, 1)
    r, c, v, pos = A.assemble(net, z, sig)
    K = A.to_dense(r, c, v, pos.N)
    cols = np.concatenate([pos.vm[0], pos.va[0]])
    colsum = K[np.ix_(pos.rowP[0], cols)].sum(axis=0)
    assert np.abs(colsum).max() <= 1e-12 * np.abs(K[np.ix_(pos.rowP[0], cols)]).max()
    # Euler homogeneity, against P_i computed independently (bus admittance form)
    net = G.config_network(1)
    z, sig = G.draw_point(net, 1)
    r, c, v, pos = A.assemble(net, z, sig)
    K = A.to_dense(r, c, v, pos.N)
    vm = z[pos.vm[0]]
    lhs = K[np.ix_(pos.rowP[0], pos.vm[0])] @ vm
    _, var_pos, row_pos = _positions(net)
    rows, _ = _hd.constraints_and_objective(net, lambda n, k, i: z[var_pos(n, k, i)], None)
    pinj = np.zeros(net.nb)
    for key, val in rows:
        if key[0] == "P":
            pinj[key[2]] = val.a
    pg = np.zeros(net.nb)
    np.add.at(pg, net.gen_bus, z[pos.pg])
    np.testing.assert_allclose(lhs, 2 * (pinj + pg), rtol=1e-12, atol=1e-12)


def test_two_bus_closed_form():
    """One branch r=0.05, x=0.2 between buses 0 and 1, no generators.
    g = r/(r^2+x^2) = 20/17, b = -x/(r^2+x^2) = -80/17.  At v=(1.02, 0.97),
    theta=(0.1, -0.05):  dP0/dv0 = 2 g v0 - v1 (g cos 0.15 + b sin 0.15),
    dP0/dth1 = -v0 v1 (g sin 0.15 - b cos 0.15)."""
    net = G.Network(2, 1, 0, np.array([0], np.int32), np.array([1], np.int32), np.array([0.05]),
                    np.array([0.2]), np.zeros(0, np.int32), np.zeros(0), np.zeros(0, np.int32), False, 1e3)
    pos = A.Positions(net)
    z = np.zeros(pos.N)
    z[pos.vm[0]] = [1.02, 0.97]
    z[pos.va[0]] = [0.1, -0.05]
    r, c, v, _ = A.assemble(net, z, np.zeros(pos.N), diag_shift=False)
    K = A.to_dense(r, c, v, pos.N)
    g, b = 20.0 / 17.0, -80.0 / 17.0
    t = 0.15
    v0, v1 = 1.02, 0.97
    dP0dv0 = 2 * g * v0 - v1 * (g * np.cos(t) + b * np.sin(t))
    dP0dth1 = -v0 * v1 * (g * np.sin(t) - b * np.cos(t))
    dQ0dv1 = -v0 * (g * np.sin(t) - b * np.cos(t))
    assert abs(K[pos.rowP[0][0], pos.vm[0][0]] - dP0dv0) < 1e-14
    assert abs(K[pos.rowP[0][0], pos.va[0][1]] - dP0dth1) < 1e-14
    assert abs(K[pos.rowQ[0][0], pos.vm[0][1]] - dQ0dv1) < 1e-14


@pytest.mark.parametrize("which", ["single", "pvpq", "agc", "agc_plain"])
def test_quasi_definite(which):
    net, _ = NETS[which]()
    z, sig = G.draw_point(net, 1)
    r, c, v, pos = A.assemble(net, z, sig)
    K = A.to_dense(r, c, v, pos.N)
    isp = pos.is_primal
    # H + diag(delta) is diagonally dominant with non-negative diagonal
    r0, c0, v0, _ = A.assemble(net, z, np.zeros_like(sig))
    K0 = A.to_dense(r0, c0, v0, pos.N)
    H = K0[np.ix_(isp, isp)]
    off = np.abs(H).sum(axis=1) - np.abs(np.diag(H))
    assert (np.diag(H) - off >= -1e-12 * max(1, np.abs(H).max())).all()
    assert np.linalg.eigvalsh(H).min() >= -1e-10 * max(1, np.abs(H).max())
    ev = np.linalg.eigvalsh(K)
    assert (ev > 0).sum() == isp.sum() and (ev < 0).sum() == (~isp).sum()


@pytest.mark.parametrize("which", ["pvpq", "agc"])
def test_union_pattern_is_value_independent(which):
    net, _ = NETS[which]()
    z1, s1 = G.draw_point(net, 99, iteration=0)
    z2, s2 = G.draw_point(net, 99, iteration=1)
    r1, c1, _, _ = A.assemble(net, z1, s1)
    r2, c2, _, _ = A.assemble(net, z2, s2)
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2)
    # contingency blocks share one pattern (union pattern)
    pos = A.Positions(net)
    pats = []
    for k in range(1, net.nblk):
        a, b = pos.block_off[k], pos.block_off[k + 1]
        m = (c1 >= a) & (c1 < b)
        rr = np.where(r1[m] < b, r1[m] - a, r1[m] - pos.block_off[-1] + 10 ** 6)
        pats.append((rr, c1[m] - a))
    for p in pats[1:]:
        assert np.array_equal(p[0], pats[0][0]) and np.array_equal(p[1], pats[0][1])


def test_screening_blocks_equal_contingency_blocks():
    """Contingency screening (eq. (screening)) fixes the first-stage
    variables, so each screening block is the KKT of its contingency alone:
    block k of the screening network must equal, entry for entry, block k+1
    of the corrective network on the same grid and outages (the part of K
    inside that block), at the same block state; the screening network has
    no base block and no border."""
    for pvpq, agc in ((False, False), (True, False), (False, True), (True, True)):
        full = G.make_network(41, 24, 33, 5, 3, pvpq=pvpq, rho=1e5, agc=agc)
        scr = G.make_network(41, 24, 33, 5, 3, pvpq=pvpq, rho=1e5, screen=True, agc=agc)
        assert np.array_equal(full.outage, scr.outage) and scr.nblk == full.nblk - 1
        zf, sf = G.draw_point(full, 41)
        pf = A.Positions(full)
        ps = A.Positions(scr)
        assert ps.N == pf.block_off[-1] - pf.block_off[1] and ps.nborder == 0
        zs = zf[pf.block_off[1]:pf.block_off[-1]].copy()
        ss = sf[pf.block_off[1]:pf.block_off[-1]].copy()
        Kf = A.to_dense(*A.assemble(full, zf, sf)[:3], pf.N)
        Ks = A.to_dense(*A.assemble(scr, zs, ss)[:3], ps.N)
        for k in range(scr.nblk):
            a0, a1 = pf.block_off[k + 1], pf.block_off[k + 2]
            b0, b1 = ps.block_off[k], ps.block_off[k + 1]
            assert np.array_equal(Ks[b0:b1, b0:b1], Kf[a0:a1, a0:a1]), (pvpq, k)
            # no coupling between screening blocks
            assert not Ks[b0:b1, :b0].any() and not Ks[b0:b1, b1:].any()
