"""Pins of the NCL-solve oracle (CPU).

* On a single-block network the NCL solution is the optimum of the
  nonlinear program itself (r -> 0): SciPy's trust-constr, an unrelated
  method, reaches the same objective and generation.
* At the returned point of an AGC network with PV/PQ rows, the KKT
  conditions of the original program hold: the regularisation r, t below
  tol, every complementarity product at the barrier level, and the
  gradient of the Lagrangian, taken by complex step of phi + y'c
  (independent of the oracle's derivative formulas), equal to the bound
  multipliers.
* The fraction-to-boundary rule on hand values; the outer iteration's
  bookkeeping (multiplier update when r is small, else rho grows).
"""
import warnings

import numpy as np
import pytest

import gridgen as G
from oracle import ipm as I
from oracle import ncl as NC


def problem(net, cfg, load_scale=0.1):
    st0 = G.ncl_start(net)
    pd = load_scale * G.draw_loads(net, cfg)
    N = st0["z"].shape[0]
    prob = I.Problem(pd=pd, lo=st0["lo"], hi=st0["hi"], y_n=np.zeros(N), mu=0.1, rho=net.rho)
    st = I.State(st0["z"], st0["rt"], st0["s"], st0["zl"], st0["zu"])
    return prob, st


def test_single_block_matches_scipy_trust_constr():
    from scipy.optimize import Bounds, NonlinearConstraint, minimize
    net = G.make_network(7, 6, 8, 2, 0, rho=1e3)
    prob, st = problem(net, 7, load_scale=0.3)
    st1, _, rep = NC.solve(net, prob, st)
    assert rep.status == 0
    m = I.masks(net, prob)
    ip = np.flatnonzero(m.primal)
    eq = np.flatnonzero(m.dual & ~m.ineq)
    ineq = np.flatnonzero(m.ineq)

    def full(w):
        z = np.zeros(m.primal.shape[0])
        z[ip] = w
        return z

    fun = lambda w: I.objective(net, full(w), prob, m)
    ceq = NonlinearConstraint(lambda w: I.constraints(net, full(w), prob, m)[eq], 0.0, 0.0)
    cin = NonlinearConstraint(lambda w: I.constraints(net, full(w), prob, m)[ineq], -np.inf, 0.0)
    lo, hi = prob.lo[ip], prob.hi[ip]
    w0 = G.ncl_start(net)["z"][ip]
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        res = minimize(fun, w0, method="trust-constr", constraints=[ceq, cin], bounds=Bounds(lo, hi),
                       options=dict(gtol=1e-10, xtol=1e-12, maxiter=3000))
    assert res.constr_violation <= 1e-7
    phi_ncl = I.objective(net, st1.z, prob, m)
    assert abs(phi_ncl - res.fun) <= 1e-5 * max(1.0, abs(res.fun)), (phi_ncl, res.fun)
    pg = st1.z[A_pg(net)]
    assert np.abs(pg - full(res.x)[A_pg(net)]).max() <= 1e-3


def A_pg(net):
    from oracle.assemble import Positions
    return Positions(net).pg


def cstep_grad(fun, x, h=1e-30):
    g = np.zeros(x.size)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for j in range(x.size):
            xc = x.astype(complex)
            xc[j] += 1j * h
            g[j] = np.imag(fun(xc)) / h
    return g


@pytest.mark.parametrize("pvpq", [True, False])
def test_solution_satisfies_the_original_kkt_conditions(pvpq):
    net = G.make_network(99, 9, 12, 3, 2, pvpq=pvpq, rho=1e5 if pvpq else 1e3, agc=True)
    prob, st = problem(net, 99)
    o = NC.Opts()
    st1, y_n, rep = NC.solve(net, prob, st, o)
    assert rep.status == 0 and rep.kkt_err <= o.tol and rep.r_inf <= o.tol
    m = I.masks(net, prob)
    z = st1.z
    # feasibility: c_E(w) = r -> 0; c_I(w) + s = t -> 0 with s >= 0
    c = I.constraints(net, z, prob, m)
    eqr = m.dual & ~m.ineq
    assert np.abs(c[eqr]).max() <= 10 * o.tol
    assert (c[m.ineq] <= 10 * o.tol).all() and (st1.s[m.ineq] > 0).all() and (z[m.ineq] > 0).all()
    # complementarity at the barrier level (the smallest mu is 1e-7)
    assert np.abs(st1.s[m.ineq] * z[m.ineq]).max() <= 10 * o.tol
    # stationarity: grad (phi + y'c) by complex step = zl - zu
    ip = np.flatnonzero(m.primal)
    y = np.where(m.dual, z, 0.0)

    def lag(w):
        zz = z.astype(complex)
        zz[ip] = w
        return I.objective(net, zz, prob, m) + np.sum(y * I.constraints(net, zz, prob, m))

    g = cstep_grad(lag, z[ip])
    assert np.abs(g - st1.zl[ip] + st1.zu[ip]).max() <= 10 * o.tol
    # AGC recourse: every generator of every contingency follows eq. (agc)
    # to the tolerance of the complementarity
    from oracle.assemble import Positions
    pos = Positions(net)
    for k in range(1, net.nblk):
        target = z[pos.pg] + net.gen_alpha * z[pos.delta[k]]
        clipped = np.clip(target, 0.0, prob.pmax)
        assert np.abs(z[pos.pgk[k]] - clipped).max() <= 1e-3


def test_fraction_to_boundary_hand_values():
    """w in [0, 2] at 1.5 moving by +1: alpha_p = tau (2 - 1.5) / 1; a slack
    at 0.2 moving by -1: tau 0.2; zl = 4 moving by -8: alpha_d = tau / 2."""
    net = G.make_network(7, 6, 8, 2, 0, rho=1e3)
    prob, st = problem(net, 7)
    m = I.masks(net, prob)
    N = m.primal.shape[0]
    lo = np.full(N, -np.inf)
    hi = np.full(N, np.inf)
    prob.lo, prob.hi = lo, hi
    j = int(np.flatnonzero(m.primal)[0])
    q = int(np.flatnonzero(m.ineq)[0])
    lo[j], hi[j] = 0.0, 2.0
    m = I.masks(net, prob)
    z = np.ones(N)
    z[j] = 1.5
    s = np.ones(N)
    s[q] = 0.2
    zl = np.zeros(N)
    zl[j] = 4.0
    st = I.State(z, np.zeros(N), s, zl, np.full(N, 1.0))
    d = I.State(np.zeros(N), np.zeros(N), np.zeros(N), np.zeros(N), np.zeros(N))
    d.z[j] = 1.0
    d.s[q] = -1.0
    d.zl[j] = -8.0
    tau = 0.99
    ap, ad = NC.max_steps(st, d, prob, m, tau)
    assert ap == pytest.approx(min(tau * 0.5, tau * 0.2)) and ad == pytest.approx(tau * 4.0 / 8.0)
    d.s[q] = 0.0
    ap, _ = NC.max_steps(st, d, prob, m, tau)
    assert ap == pytest.approx(tau * 0.5)


def test_outer_updates():
    """The first subproblem's r is above tol: with r <= eta the multiplier
    estimates become the subproblem's y, which equals y_n + rho r there
    (G_rt = 0 to the tolerance); with eta tiny the penalty grows tenfold
    instead and y_n stays."""
    net = G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True)
    prob, st = problem(net, 99)
    m = I.masks(net, prob)
    st1, y1, rep = NC.solve(net, prob, st, NC.Opts(max_outer=1))
    assert rep.status == 1 and rep.r_inf > 1e-6 and rep.history[0][3] is True
    np.testing.assert_array_equal(y1[m.dual], st1.z[m.dual])
    assert np.abs(st1.z[m.dual] - prob.rho * st1.rt[m.dual]).max() <= 1e-6
    _, y2, rep2 = NC.solve(net, prob, st, NC.Opts(max_outer=1, eta0=1e-9))
    assert rep2.history[0][3] is False and rep2.history[0][2] == 10 * prob.rho
    assert not y2[m.dual].any()


def test_screening_at_the_corrective_solution_is_feasible():
    """eq. (screening): at the first stage (pg0, vm0) of a converged
    corrective NCL solution every contingency is feasible, so the screening
    network's NCL solve over the same contingencies converges with r -> 0;
    and its blocks' primal values satisfy the AGC rule of eq. (agc)."""
    from oracle.assemble import Positions
    net = G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True)
    prob, st = problem(net, 99)
    st1, _, rep = NC.solve(net, prob, st)
    assert rep.status == 0
    pos = Positions(net)
    pg0, vm0 = st1.z[pos.pg], st1.z[pos.vm0]
    scr = G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True, screen=True)
    st0 = G.ncl_start(scr)
    N = st0["z"].shape[0]
    prob_s = I.Problem(pd=prob.pd, lo=st0["lo"], hi=st0["hi"], y_n=np.zeros(N), mu=0.1, rho=scr.rho, pg0=pg0, vm0=vm0)
    ss, _, rep_s = NC.solve(scr, prob_s, I.State(st0["z"], st0["rt"], st0["s"], st0["zl"], st0["zu"]))
    assert rep_s.status == 0 and rep_s.r_inf <= 1e-6
    ps = Positions(scr)
    for k in range(scr.nblk):
        target = pg0 + scr.gen_alpha * ss.z[ps.delta[k]]
        assert np.abs(ss.z[ps.pgk[k]] - np.clip(target, 0.0, prob_s.pmax)).max() <= 1e-3
