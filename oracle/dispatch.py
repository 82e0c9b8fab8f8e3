"""Oracle: the differentiable dispatch map (TEST INFRASTRUCTURE ONLY).

Plain FP64 numpy/scipy.  Only tests/, the smoke check and the benchmark's
CPU baseline may import this module; the product path never does.

The map pd -> (phi*, pg*) is defined by the stationarity F(z; pd) = 0 of the
NCL subproblem (Section III: the augmented-Lagrangian subproblem with the
residuals r as free variables, here at fixed rho, multiplier estimate 0
and barrier parameter mu) of the corrective SCOPF of Section II-B without
PV/PQ switching, with r eliminated through its optimality y = -rho r (rho of the network):

    minimise  phi(pg) + beta_mu(w) + (eps/2) sum_k va_{k,0}^2 + (rho/2)|r|^2
    s.t.      c_k(w; pd) + r_k = 0                 (P and Q balance rows)
              h_k(w) + r_F,k <= smax2              (flow rows; slack t > 0
                                                    with barrier -mu log t)

phi = sum_g c2_g pg_g^2; beta_mu is the log barrier of vm in [vmin, vmax],
qg in [-qmax, qmax], pg in [0, pmax]; the eps term pins each block's
reference angle (bus 0), which removes the angle-shift null space.  The
loads enter the balance rows as + pd (P) and + qd_ratio * pd (Q) in every
block.  With t = mu / y_F and r = -y/rho eliminated:

    F_w   = grad phi + grad beta + eps e_ref va_ref + sum_rows y grad c_row
    F_PQ  = c(w; pd) - y / rho
    F_F   = h(w) - smax2 - y_F / rho + mu / y_F

and dF/dz is exactly the KKT matrix of the assembly (no diagonal shift)
with Sigma = Hess beta (+ eps on the reference angles) at the primal rows
and the extra dual diagonal mu / y_F^2 on the flow rows (block C for an
eliminated inequality slack).  The residual is written out independently of
the assembly, so a finite-difference Jacobian of it pins both.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import assemble as _asm


# barrier continuation from the default start: a factor ~3 per stage keeps
# each stage's start inside the region where the barrier Newton converges
MU_SCHEDULE = (10.0, 3.0, 1.0, 0.3, 0.1, 0.03)


@dataclass
class NLP:
    mu: float = 0.3
    vmin: float = 0.9
    vmax: float = 1.1
    qmax: float = 3.0
    pmax: float = 8.0
    smax2: float = 100.0
    eps: float = 1.0
    qd_ratio: float = 0.3


def residual(net, z, pd, p: NLP):
    """F(z; pd) and the diagonal Sigma (primal barrier Hessian + eps, dual
    flow-row mu/y^2) of the NCL subproblem, both in layout order."""
    if net.pvpq or getattr(net, "agc", False):
        raise ValueError("the dispatch map is defined for networks without PV/PQ or AGC rows")
    pos = _asm.Positions(net)
    z = np.asarray(z)
    if not np.iscomplexobj(z):
        z = z.astype(np.float64)
    N = pos.N
    F = np.zeros(N, z.dtype)       # complex z allowed (complex-step derivatives)
    sig = np.zeros(N, z.dtype)
    den = net.br_r ** 2 + net.br_x ** 2
    gser, bser = net.br_r / den, -net.br_x / den
    f, t = net.br_from.astype(np.int64), net.br_to.astype(np.int64)
    gb = net.gen_bus.astype(np.int64)
    pg = z[pos.pg]
    qd = p.qd_ratio * pd
    F[pos.pg] += 2.0 * net.gen_c2 * pg
    for k in range(net.nblk):
        st = _asm.branch_status(net, k)
        g, b = st * gser, st * bser
        vm_p, va_p = pos.vm[k], pos.va[k]
        v, th = z[vm_p], z[va_p]
        yP, yQ = z[pos.rowP[k]], z[pos.rowQ[k]]
        Pinj = np.zeros(net.nb, z.dtype)
        Qinj = np.zeros(net.nb, z.dtype)
        for s_bus, o_bus, rowF in ((f, t, pos.rowFf[k]), (t, f, pos.rowFt[k])):
            P, Q, dP, dQ, _, _ = _asm._end_derivs(g, b, v[s_bus], v[o_bus], th[s_bus] - th[o_bus])
            np.add.at(Pinj, s_bus, P)
            np.add.at(Qinj, s_bus, Q)
            yF = z[rowF]
            F[rowF] = P * P + Q * Q - p.smax2 - yF / net.rho + p.mu / yF
            sig[rowF] = p.mu / (yF * yF)
            dh = 2.0 * P[:, None] * dP + 2.0 * Q[:, None] * dQ
            var = np.stack([vm_p[s_bus], vm_p[o_bus], va_p[s_bus], va_p[o_bus]], 1)
            contrib = yP[s_bus][:, None] * dP + yQ[s_bus][:, None] * dQ + yF[:, None] * dh
            np.add.at(F, var, contrib)
        np.add.at(Pinj, gb, -pg)
        np.add.at(Qinj, gb, -z[pos.qg[k]])
        F[pos.rowP[k]] = Pinj + pd - yP / net.rho
        F[pos.rowQ[k]] = Qinj + qd - yQ / net.rho
        F[pos.qg[k]] += -yQ[gb]
        np.add.at(F, pos.pg, -yP[gb])
        lo, hi = v - p.vmin, p.vmax - v
        F[vm_p] += -p.mu / lo + p.mu / hi
        sig[vm_p] += p.mu / lo ** 2 + p.mu / hi ** 2
        q = z[pos.qg[k]]
        lo, hi = q + p.qmax, p.qmax - q
        F[pos.qg[k]] += -p.mu / lo + p.mu / hi
        sig[pos.qg[k]] += p.mu / lo ** 2 + p.mu / hi ** 2
        F[va_p[0]] += p.eps * th[0]
        sig[va_p[0]] += p.eps
    lo, hi = pg, p.pmax - pg
    F[pos.pg] += -p.mu / lo + p.mu / hi
    sig[pos.pg] += p.mu / lo ** 2 + p.mu / hi ** 2
    return F, sig


def kkt_exact(net, z, sig, p: NLP):
    """dF/dz: the assembled KKT (no shift) at z with this Sigma (lower CSC)."""
    from . import kkt
    return kkt(net, z, sig, diag_shift=False)


def full_matrix(cp, ri, v):
    import scipy.sparse as sp
    N = cp.shape[0] - 1
    Lw = sp.csc_matrix((v, ri, cp), shape=(N, N))
    return (Lw + Lw.T - sp.diags(Lw.diagonal())).tocsc()


def initial_point(net, pd, p: NLP):
    pos = _asm.Positions(net)
    z = np.zeros(pos.N)
    for k in range(net.nblk):
        z[pos.vm[k]] = 1.0
        z[pos.rowFf[k]] = p.mu / p.smax2
        z[pos.rowFt[k]] = p.mu / p.smax2
    z[pos.pg] = 0.5 * p.pmax
    return z


def max_step(net, z, dz, p: NLP, tau=0.995):
    """Largest alpha <= 1 keeping every barrier argument positive (fraction to boundary)."""
    pos = _asm.Positions(net)
    alpha = 1.0

    def lim(x, dx, lo=None, hi=None):
        nonlocal alpha
        if lo is not None:
            m = dx < 0
            if m.any():
                alpha = min(alpha, float(np.min(tau * (x[m] - lo) / -dx[m])))
        if hi is not None:
            m = dx > 0
            if m.any():
                alpha = min(alpha, float(np.min(tau * (hi - x[m]) / dx[m])))
    for k in range(net.nblk):
        lim(z[pos.vm[k]], dz[pos.vm[k]], p.vmin, p.vmax)
        lim(z[pos.qg[k]], dz[pos.qg[k]], -p.qmax, p.qmax)
        for rows in (pos.rowFf[k], pos.rowFt[k]):
            lim(z[rows], dz[rows], 0.0)
    lim(z[pos.pg], dz[pos.pg], 0.0, p.pmax)
    return alpha


def newton(net, pd, p: NLP, z0=None, step_tol=1e-10, maxit=100, verbose=False):
    """Solve F(z; pd) = 0 by Newton's method with fraction-to-boundary and
    backtracking on |F|_2.  The step uses the exact dF/dz (sparse LU with
    pivoting).  Converged when the full Newton step is below step_tol
    relative to z: near an active bound the barrier Hessian is so large
    that |F| itself bottoms out at (barrier curvature) x (one ulp of z).
    From the default start the barrier parameter is continued down from 10
    to p.mu through MU_SCHEDULE (each stage warm-starts the next); from a given z0 only the
    target mu is solved.  Returns z and the total iteration count."""
    import scipy.sparse.linalg as spl
    from dataclasses import replace
    if z0 is None:
        z = initial_point(net, pd, p)
        mus = [m for m in MU_SCHEDULE if m > p.mu] + [p.mu]
    else:
        z = np.array(z0, np.float64)
        mus = [p.mu]
    total = 0
    for mu in mus:
        q = replace(p, mu=mu)
        tol = step_tol if mu == p.mu else 1e-6
        F, sig = residual(net, z, pd, q)
        nrm = np.linalg.norm(F)
        for it in range(maxit):
            cp, ri, v, _ = kkt_exact(net, z, sig, q)
            dz = spl.spsolve(full_matrix(cp, ri, v), -F)
            if np.all(np.abs(dz) <= tol * (1.0 + np.abs(z))):
                if max_step(net, z, dz, q) >= 1.0:     # take the last (tiny) step
                    z = z + dz
                break
            alpha = max_step(net, z, dz, q)
            while True:
                zt = z + alpha * dz
                Ft, sigt = residual(net, zt, pd, q)
                nt = np.linalg.norm(Ft)
                if nt <= (1.0 - 1e-4 * alpha) * nrm or alpha < 1e-10:
                    break
                alpha *= 0.5
            if alpha < 1e-10 and np.all(np.abs(dz) <= 1e-6 * (1.0 + np.abs(z))):
                break                 # at the rounding floor of |F| with a tiny remaining step
            z, F, sig, nrm = zt, Ft, sigt, nt
            total += 1
            if verbose:
                print(f"  mu {mu:g} it {it}: |F|inf {np.abs(F).max():.3e} alpha {alpha:.3g}")
        else:
            raise RuntimeError(f"Newton did not converge at mu = {mu:g}: |F|inf = {np.abs(F).max():.3e}")
    return z, total


def outputs(net, z):
    """phi(pg) and pg at a state."""
    pos = _asm.Positions(net)
    pg = z[pos.pg]
    return float(np.sum(net.gen_c2 * pg * pg)), pg.copy()


def gradients(net, z, pd, p: NLP, method="splu", cotangent=None):
    """d phi*/d pd and d pg*/d pd (ng x nb) at a solution z, from the exact
    KKT: a = K^{-1} g for each output gradient g, then d/dpd_i =
    -sum_k (a[P_k,i] + qd_ratio a[Q_k,i]).  method: "dense" (numpy solve
    of the dense K), "splu" (scipy sparse LU) or "ldlt" (the oracle's
    pivot-free LDL^T, for large K; then only phi* and, if given, one pg
    cotangent are differentiated and the pg Jacobian is None)."""
    _, sig = residual(net, z, pd, p)
    cp, ri, v, pos = kkt_exact(net, z, sig, p)
    ng = net.ng
    pg = z[pos.pg]
    rowP, rowQ = pos.rowP, pos.rowQ
    if method == "ldlt":
        from . import Factor
        F = Factor(pos.N, cp, ri, np.array(pos.block_off))
        rc = F.factor(cp, ri, v, nthreads=8)
        if rc != 0:
            raise RuntimeError(f"oracle LDL^T of the dispatch KKT failed: {rc}")
        G = np.zeros((2, pos.N))
        G[0, pos.pg] = 2.0 * net.gen_c2 * pg
        if cotangent is not None:
            G[1, pos.pg] = cotangent
        A = F.solve(G)
        D = -(A[:, rowP].sum(axis=1) + p.qd_ratio * A[:, rowQ].sum(axis=1))   # (2, nb)
        return D[0].copy(), (D[1].copy() if cotangent is not None else None)
    Kf = full_matrix(cp, ri, v)
    G = np.zeros((pos.N, ng + 1))
    G[pos.pg, 0] = 2.0 * net.gen_c2 * pg
    G[pos.pg, 1 + np.arange(ng)] = 1.0
    if method == "dense":
        A = np.linalg.solve(Kf.toarray(), G)
    else:
        import scipy.sparse.linalg as spl
        A = spl.splu(Kf).solve(G)
    D = -(A[rowP].sum(axis=0) + p.qd_ratio * A[rowQ].sum(axis=0))   # (nb, ng+1)
    return D[:, 0].copy(), D[:, 1:].T.copy()
