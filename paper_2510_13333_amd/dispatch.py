"""Differentiable dispatch: loads pd -> (optimal cost phi*, dispatch pg*).

The map is defined by the stationarity F(z; pd) = 0 of the NCL subproblem
(Section III: the augmented-Lagrangian subproblem, here at fixed rho,
multiplier estimate 0 and barrier parameter mu) of the corrective SCOPF
(Section II-B) without PV/PQ rows.  Its Jacobian dF/dz is the KKT matrix
of the Newton system (Section IV-B) assembled without the diagonal shift,
so that

    d phi*/d pd = -(K^{-1} grad phi)[P rows] - qd_ratio (K^{-1} grad phi)[Q rows]

summed over the blocks (every block sees the same loads), and likewise for
any cotangent of pg*.  The forward pass is the library's Newton solve
(ncl_kkt_dispatch_newton: residual, exact K, inertia correction, LDL^T
factor and solve, fraction-to-boundary step, backtracking), the outputs
come from ncl_kkt_dispatch_outputs, and the backward pass is
ncl_kkt_dispatch_vjp: one ncl_kkt_solve_adjoint on the factors the
forward pass left (the exact K at the solution) and the reduction to the
loads.  PyTorch holds the vectors and orders the calls; every arithmetic
step runs in the library.
"""
from __future__ import annotations

import torch

from .ncl import KKT, NclError, NewtonOpts

DEFAULTS = dict(qd_ratio=0.3, mu=0.3, vmin=0.9, vmax=1.1, qmax=3.0, pmax=8.0, smax2=100.0, eps=1.0)
FLOOR_TOL = 1e-6      # step accepted as converged when backtracking stalls at the rounding floor


class DispatchSolver:
    """The dispatch map on one network (one GPU handle): the Newton solve
    (ncl_kkt_dispatch_newton), the outputs (ncl_kkt_dispatch_outputs) and
    the adjoint (ncl_kkt_dispatch_vjp) all run in the library; this class
    holds the device vectors and orders the calls."""

    def __init__(self, net, params=None, device="cuda"):
        self.net = net
        self.p = dict(DEFAULTS)
        self.p.update(params or {})
        self.p["rho"] = float(net.rho)
        self.k = KKT(net).bind(nrhs_max=1, device=device)
        self.device = device
        n = self.k.N
        self.work = torch.empty(7 * n + 8, dtype=torch.float64, device=device)
        self.vwork = torch.empty(2 * n, dtype=torch.float64, device=device)
        self.opts = NewtonOpts(1e-10, FLOOR_TOL, 100, 1, 0, 0, 0.0)
        self.z_warm = None
        self.factored_at = None      # the state whose exact K is in the handle's factors
        self.iterations = 0

    def newton(self, pd, z0=None, step_tol=1e-10, maxit=100):
        """Solve F(z; pd) = 0 in the library: from the default start with
        barrier continuation, or from z0 at the target barrier value."""
        z = torch.empty(self.k.N, dtype=torch.float64, device=self.device) if z0 is None else z0.clone()
        self.opts.step_tol = step_tol
        self.opts.maxit = maxit
        self.opts.from_default = 1 if z0 is None else 0
        self.k.dispatch_newton(pd, self.p, z, self.work, self.opts)
        self.factored_at = z
        self.iterations = self.opts.iterations
        return z

    def outputs(self, z):
        phi = torch.empty((), dtype=torch.float64, device=self.device)
        pg = torch.empty(self.net.ng, dtype=torch.float64, device=self.device)
        self.k.dispatch_outputs(z, phi, pg)
        return phi, pg

    def vjp(self, z, gphi, gpg):
        """Cotangent of (phi*, pg*) -> cotangent of pd, by one adjoint solve."""
        pd = self._pd_of[0]
        if self.factored_at is None or not torch.equal(self.factored_at, z):
            F, sig = self.k.residual(z, pd, self.p)
            self.k.assemble(z, sig, self.p["rho"], shift=False)
            self.k.factor()
            r = self.k.info()
            if not (r["solvable"] and r["npos"] == self.k.nprimal and r["nneg"] == self.k.N - self.k.nprimal):
                raise NclError("dispatch KKT at the solution", r["status"])
            self.factored_at = z
        gpd = torch.empty(self.net.nb, dtype=torch.float64, device=self.device)
        return self.k.dispatch_vjp(pd, self.p, z, gphi.contiguous(), None if gpg is None else gpg.contiguous(),
                                   gpd, self.vwork)

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
        if gphi is None:
            gphi = torch.zeros((), dtype=torch.float64, device=z.device)
        return s.vjp(z, gphi, gpg), None
