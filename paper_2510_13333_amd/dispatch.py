"""Differentiable dispatch: loads pd -> (optimal cost phi*, dispatch pg*).

The map is defined by the stationarity F(z; pd) = 0 of the NCL subproblem
(Section III: the augmented-Lagrangian subproblem, here at fixed rho,
multiplier estimate 0 and barrier parameter mu) of the corrective SCOPF
(Section II-B) without PV/PQ rows.  Its Jacobian dF/dz is the KKT matrix
of the Newton system (Section IV-B) assembled without the diagonal shift,
so that

    d phi*/d pd = -(K^{-1} grad phi)[P rows] - qd_ratio (K^{-1} grad phi)[Q rows]

summed over the blocks (every block sees the same loads), and likewise for
any cotangent of pg*.  The forward pass is a Newton solve on the library:
F and Sigma from ncl_kkt_residual, K from ncl_kkt_assemble, the LDL^T
factor and solve, the fraction-to-boundary step from ncl_kkt_max_step.
The backward pass is one ncl_kkt_solve_adjoint on the factors the forward
pass left (the exact K at the solution).  PyTorch holds the vectors and
orders the calls; the arithmetic of every step runs in the library.
"""
from __future__ import annotations

import numpy as np
import torch

from .ncl import KKT, NclError

DEFAULTS = dict(qd_ratio=0.3, mu=0.3, vmin=0.9, vmax=1.1, qmax=3.0, pmax=8.0, smax2=100.0, eps=1.0)
MU_SCHEDULE = (10.0, 3.0, 1.0, 0.3, 0.1, 0.03)
FLOOR_TOL = 1e-6      # step accepted as converged when backtracking stalls at the rounding floor
L_VM, L_VA, L_QG, L_PG, L_ROWP, L_ROWQ, L_FLOW = 1, 2, 3, 4, 5, 6, 7


class DispatchSolver:
    """Newton solver of the dispatch map on one network (one GPU handle)."""

    def __init__(self, net, params=None, device="cuda"):
        self.net = net
        self.p = dict(DEFAULTS)
        self.p.update(params or {})
        self.p["rho"] = float(net.rho)
        self.k = KKT(net).bind(nrhs_max=1, device=device)
        kinds = self.k.layout_kinds()
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.kinds = dev(kinds)
        self.pg_idx = dev(np.flatnonzero(kinds == L_PG))
        self.c2 = dev(np.asarray(net.gen_c2, np.float64))
        nb = int(net.nb)
        rowP = np.flatnonzero(kinds == L_ROWP).reshape(-1, nb)    # [blocks, nb], layout order
        rowQ = np.flatnonzero(kinds == L_ROWQ).reshape(-1, nb)
        self.rowP, self.rowQ = dev(rowP), dev(rowQ)
        self.device = device
        self.alpha = torch.empty(1, dtype=torch.float64, device=device)
        self.primal = ((self.kinds >= L_VM) & (self.kinds <= L_PG)).to(torch.float64)
        self.dw_last = 0.0
        self.z_warm = None
        self.factored_at = None      # the state whose exact K is in the handle's factors
        self.iterations = 0

    # -------------------------------------------------------------- pieces
    def initial_point(self):
        z = torch.zeros(self.k.N, dtype=torch.float64, device=self.device)
        z[self.kinds == L_VM] = 1.0
        z[self.kinds == L_PG] = 0.5 * self.p["pmax"]
        z[self.kinds == L_FLOW] = self.p["mu"] / self.p["smax2"]
        return z

    def _params(self, mu):
        q = dict(self.p)
        q["mu"] = mu
        return q

    def _factor(self, z, sig, exact):
        """Assemble and factor; True when the factorisation has the inertia of
        a strict local minimum, (n, m) with no zero or non-finite pivot.
        (Single pivots may carry the other sign when K11 is not definite:
        the inertia, not each sign, is what a minimum fixes.)"""
        self.k.assemble(z, sig, self.p["rho"], shift=not exact)
        self.k.factor()
        r = self.k.info()
        return (r["status"] in (0, -6) and r["nzero"] == 0 and r["npos"] == self.k.nprimal
                and r["nneg"] == self.k.N - self.k.nprimal)

    def _factor_corrected(self, z, sig):
        """Factor the exact Newton matrix; if its pivot signs (inertia) are
        wrong, add dw on the primal diagonal, dw growing from a fraction of
        the last accepted value (or 1e-4) by x8 until they are right (the
        inertia correction of Section V-C, as a primal shift dw I)."""
        if self._factor(z, sig, exact=True):
            self.dw_last = 0.0
            return 0.0
        dw = self.dw_last / 3.0 if self.dw_last > 0 else 1e-4
        while dw < 1e12:
            if self._factor(z, sig + dw * self.primal, exact=True):
                self.dw_last = dw
                return dw
            dw *= 8.0
        raise NclError("dispatch Newton matrix: inertia correction failed", self.k.info()["status"])

    def newton(self, pd, z0=None, step_tol=1e-10, maxit=100):
        """Solve F(z; pd) = 0: Newton steps with the exact K (inertia-corrected
        when its pivot signs are wrong), a fraction-to-boundary step,
        backtracking on |F|_2; converged when the full step is below
        step_tol relative to z.  From the default start the barrier
        parameter is continued down to mu."""
        if z0 is None:
            z = self.initial_point()
            mus = [m for m in MU_SCHEDULE if m > self.p["mu"]] + [self.p["mu"]]
        else:
            z = z0.clone()
            mus = [self.p["mu"]]
        total = 0
        for mu in mus:
            q = self._params(mu)
            tol = step_tol if mu == self.p["mu"] else 1e-6
            F, sig = self.k.residual(z, pd, q)
            nrm = float(torch.linalg.vector_norm(F))
            for _ in range(maxit):
                self._factor_corrected(z, sig)
                dz = self.k.solve(-F)
                if bool(torch.all(dz.abs() <= tol * (1.0 + z.abs()))):
                    # take the (tiny, quadratically accurate) last step
                    self.k.max_step(z, dz, pd, q, 0.995, self.alpha)
                    if float(self.alpha) >= 1.0:
                        z = z + dz
                        F, sig = self.k.residual(z, pd, q)
                    break
                self.k.max_step(z, dz, pd, q, 0.995, self.alpha)
                a = float(self.alpha)
                while True:
                    zt = z + a * dz
                    Ft, sigt = self.k.residual(zt, pd, q)
                    nt = float(torch.linalg.vector_norm(Ft))
                    if nt <= (1.0 - 1e-4 * a) * nrm or a < 1e-10:
                        break
                    a *= 0.5
                if a < 1e-10 and bool(torch.all(dz.abs() <= FLOOR_TOL * (1.0 + z.abs()))):
                    # |F| is at its rounding floor (variables pressed against
                    # their bounds make the barrier curvature huge) and the
                    # remaining step is tiny: converged as far as FP64 resolves
                    break
                z, F, sig, nrm = zt, Ft, sigt, nt
                total += 1
            else:
                raise RuntimeError(f"dispatch Newton did not converge at mu = {mu:g}")
        # leave the exact K at the solution factored for the backward pass
        if not self._factor(z, sig, exact=True):
            raise NclError("dispatch KKT at the solution (not a strict local minimum)", self.k.info()["status"])
        self.factored_at = z
        self.iterations = total
        return z

    def outputs(self, z):
        pg = z[self.pg_idx]
        return torch.sum(self.c2 * pg * pg), pg

    def vjp(self, z, gphi, gpg):
        """Cotangent of (phi*, pg*) -> cotangent of pd, by one adjoint solve."""
        if self.factored_at is None or not torch.equal(self.factored_at, z):
            _, sig = self.k.residual(z, self._pd_of[0], self.p)
            if not self._factor(z, sig, exact=True):
                raise NclError("dispatch KKT at the solution", self.k.info()["status"])
            self.factored_at = z
        pg = z[self.pg_idx]
        g = torch.zeros_like(z)
        g[self.pg_idx] = gphi * 2.0 * self.c2 * pg + gpg
        a = self.k.solve_adjoint(g)
        return -(a[self.rowP].sum(0) + self.p["qd_ratio"] * a[self.rowQ].sum(0))

    def __call__(self, pd):
        return NCLDispatch.apply(pd, self)


class NCLDispatch(torch.autograd.Function):
    """pd (nb,) float64 on the device -> (phi*, pg*); backward = adjoint solve."""

    @staticmethod
    def forward(ctx, pd, solver: DispatchSolver):
        pd_ = pd.detach().contiguous()
        z = solver.newton(pd_, z0=solver.z_warm)
        solver.z_warm = z
        solver._pd_of = (pd_,)
        phi, pg = solver.outputs(z)
        ctx.solver = solver
        ctx.save_for_backward(z)
        return phi, pg

    @staticmethod
    def backward(ctx, gphi, gpg):
        (z,) = ctx.saved_tensors
        s = ctx.solver
        gphi = torch.zeros((), dtype=torch.float64, device=z.device) if gphi is None else gphi
        gpg = torch.zeros_like(z[s.pg_idx]) if gpg is None else gpg
        return s.vjp(z, gphi, gpg), None
