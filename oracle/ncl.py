"""Oracle: the NCL outer loop around the subproblem's interior-point method
(TEST INFRASTRUCTURE ONLY).  Plain FP64 numpy on top of oracle.ipm; only
tests/, the smoke check and the benchmark's CPU-baseline leg may import it,
the product path never does.

Section IV-A: the outer iterations update the penalty rho and the
multiplier estimates (lam_n, nu0_n), one vector y_n over the dual rows
here, from the solution of the subproblem eq. (nclsubpb); the inner
iterations solve that subproblem with an IPM warm-started from the previous
primal-dual point.  Section V fixes the tolerance (1e-6) and the smallest
barrier parameter (1e-7).  The paper leaves the update rules to the MadNCL
paper; the rules below are this implementation's reading.

Outer iteration n (subproblem at y_n, rho_n):
    solve the subproblem (inner loop below);
    r_inf = max |rt| over the dual rows;
    r_inf <= tol:     stop, converged;
    r_inf <= eta_n:   y_{n+1} = y (the subproblem's multipliers; at its
                      solution y_n + rho rt - y = 0, so this is the
                      first-order update y_n + rho_n r), eta_{n+1} =
                      max(eta_n / eta_shrink, tol), rho unchanged;
    otherwise:        rho_{n+1} = min(rho_grow rho_n, rho_max), y_n kept;
    the next subproblem starts at the current point with mu = mu_warm.

Inner iterations (primal-dual IPM with a monotone barrier, unknowns and
residual G of oracle.ipm):
    E_0 = max |G(u; mu = 0)|; stop when E_0 <= tol;
    while max |G(u; mu)| <= kappa_eps mu and mu > mu_min:
        mu = max(mu_min, min(kappa_mu mu, mu^theta_mu));
    the inertia-corrected Newton direction d (oracle.ipm.step);
    tau = max(tau_min, 1 - mu); fraction to the boundary: alpha_p the
    largest step in (0, 1] keeping w - lo, hi - w and s above (1 - tau)
    times their values, alpha_d the same for zl, zu and y at the
    inequality rows (their slacks' bound multipliers);
    w, y at equality rows, rt and s move by alpha_p; zl, zu and y at
    inequality rows by alpha_d.  No line search: the paper's IPM uses a
    filter line search (Section V-C), which is not reproduced here; the
    regularisation keeps these steps stable on the workloads tested (a
    merit backtracking on ||G||_2 with the two step lengths stalled).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from . import Factor
from . import ipm as _ipm


@dataclass
class Opts:
    tol: float = 1e-6
    mu_min: float = 1e-7
    mu0: float = 0.1
    mu_warm: float = 1e-5
    kappa_eps: float = 10.0
    kappa_mu: float = 0.2
    theta_mu: float = 1.5
    tau_min: float = 0.99
    eta0: float = 1e-2
    eta_shrink: float = 10.0
    rho_grow: float = 10.0
    rho_max: float = 1e12
    max_inner: int = 300
    max_outer: int = 30


@dataclass
class Report:
    status: int = 0                     # 0 converged, 1 outer limit, 2 inner limit
    outer: int = 0
    inner: int = 0                      # inner iterations over all subproblems
    factorizations: int = 0
    rho: float = 0.0
    mu: float = 0.0
    r_inf: float = 0.0
    kkt_err: float = 0.0                # E_0 at the last iterate
    history: list = field(default_factory=list)   # per outer: (inner its, r_inf, rho, updated)


def max_steps(st: _ipm.State, d: _ipm.State, prob: _ipm.Problem, m: _ipm.Masks, tau: float):
    """Fraction to the boundary: (alpha_p, alpha_d)."""
    lo, hi = np.asarray(prob.lo), np.asarray(prob.hi)

    def limit(x, dx):
        # largest a <= 1 with x + a dx >= (1 - tau) x, for x > 0
        neg = dx < 0
        if not neg.any():
            return 1.0
        return min(1.0, float(np.min(-tau * x[neg] / dx[neg])))

    w, dw = st.z, d.z
    a = m.has_lo
    ap = limit(w[a] - lo[a], dw[a])
    a = m.has_hi
    ap = min(ap, limit(hi[a] - w[a], -dw[a]))
    q = m.ineq
    ap = min(ap, limit(st.s[q], d.s[q]))
    ad = limit(st.zl[m.has_lo], d.zl[m.has_lo])
    ad = min(ad, limit(st.zu[m.has_hi], d.zu[m.has_hi]))
    ad = min(ad, limit(st.z[q], d.z[q]))
    return ap, ad


def take_step(st: _ipm.State, d: _ipm.State, m: _ipm.Masks, ap: float, ad: float) -> _ipm.State:
    """u + a d with a_p on w, y at equality rows, rt and s; a_d on zl, zu and
    y at inequality rows."""
    az = np.where(m.ineq, ad, ap)
    return _ipm.State(st.z + az * d.z, st.rt + ap * d.rt, st.s + ap * d.s, st.zl + ad * d.zl, st.zu + ad * d.zu)


def residual(net, st, prob, m, mu):
    return _ipm.kkt_residual(net, st, replace(prob, mu=mu), m)


def subproblem(net, st: _ipm.State, prob: _ipm.Problem, o: Opts, rep: Report, factor: Factor):
    """Inner iterations at fixed (y_n, rho); prob.mu is the starting barrier
    parameter.  Returns (state, mu, inner iterations, converged)."""
    m = _ipm.masks(net, prob)
    mu = prob.mu
    dw_last = 0.0
    its = 0
    G = residual(net, st, prob, m, mu)
    while True:
        E0 = float(np.max(np.abs(residual(net, st, prob, m, 0.0))))
        rep.kkt_err = E0
        if E0 <= o.tol:
            return st, mu, its, True
        while float(np.max(np.abs(G))) <= o.kappa_eps * mu and mu > o.mu_min:
            mu = max(o.mu_min, min(o.kappa_mu * mu, mu ** o.theta_mu))
            G = residual(net, st, prob, m, mu)
        if its == o.max_inner:
            return st, mu, its, False
        p = replace(prob, mu=mu)
        d, dw_last, nfac = _ipm.step(net, st, p, dw_last, factor)
        rep.factorizations += nfac
        tau = max(o.tau_min, 1.0 - mu)
        ap, ad = max_steps(st, d, p, m, tau)
        st = take_step(st, d, m, ap, ad)
        G = residual(net, st, prob, m, mu)
        its += 1


def solve(net, prob: _ipm.Problem, st: _ipm.State, o: Opts = None):
    """The NCL outer loop from the interior point st (prob.y_n the first
    multiplier estimates, prob.rho the first penalty, prob.mu ignored: the
    first subproblem starts at o.mu0).  Returns (state, y_n, Report)."""
    o = o or Opts()
    rep = Report()
    factor = Factor.from_network(net)
    m = _ipm.masks(net, prob)
    prob = replace(prob, y_n=np.array(prob.y_n, np.float64), mu=o.mu0)
    eta = o.eta0
    st = st.copy()
    for n in range(o.max_outer):
        st, mu, its, ok = subproblem(net, st, prob, o, rep, factor)
        rep.inner += its
        rep.outer = n + 1
        rep.mu = mu
        rep.rho = prob.rho
        r_inf = float(np.max(np.abs(st.rt[m.dual]))) if m.dual.any() else 0.0
        rep.r_inf = r_inf
        if not ok:
            rep.status = 2
            rep.history.append((its, r_inf, prob.rho, False))
            return st, prob.y_n, rep
        if r_inf <= o.tol:
            rep.history.append((its, r_inf, prob.rho, False))
            rep.status = 0
            return st, prob.y_n, rep
        if r_inf <= eta:
            y_n = prob.y_n.copy()
            y_n[m.dual] = st.z[m.dual]
            prob = replace(prob, y_n=y_n)
            eta = max(eta / o.eta_shrink, o.tol)
            rep.history.append((its, r_inf, prob.rho, True))
        else:
            prob = replace(prob, rho=min(o.rho_grow * prob.rho, o.rho_max))
            rep.history.append((its, r_inf, prob.rho, False))
        prob = replace(prob, mu=o.mu_warm)
    rep.status = 1
    return st, prob.y_n, rep
