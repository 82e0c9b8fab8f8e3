"""GPU parity of the NCL solve (ncl_kkt_ncl_solve) against the oracle's NCL
loop (oracle/ncl.py) on the same seeded problems: the same status and
outer iterations, the same final point to the tolerance, and the oracle's
barrier KKT residual at the GPU's final point (mu = 0) within the
tolerance.  Where the penalty stays at its first value the inner iteration
counts are equal too; on the 9-bus network without PV/PQ rows the problem
is nearly infeasible (r stalls near 5e-6), rho climbs to 1e6, and the
subproblems there follow rounding (91 GPU against 205 oracle iterations in
total, both converged), so only the converged primal point is compared and
the multipliers are checked by the residual (those of biactive
complementarity pairs are not unique there).  Loads are
the NCL workload's (a fraction of the seeded pd)."""
import numpy as np
import pytest

import gridgen as G
from oracle import ipm as I
from oracle import ncl as NC

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2510_13333_amd import KKT  # noqa: E402
from paper_2510_13333_amd.ncl import NclError, SolveOpts  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda")


def host(t):
    return t.cpu().numpy()


NETS = {
    "single7": lambda: (G.make_network(7, 6, 8, 2, 0, rho=1e3), 7, 0.3),
    "c1": lambda: (G.config_network(1), 1, 0.3),
    "agc9": lambda: (G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True), 99, 0.1),
    "agc9_plain": lambda: (G.make_network(99, 9, 12, 3, 2, rho=1e3, agc=True), 99, 0.1),
    "agc30x3": lambda: (G.make_network(1, 30, 41, 6, 3, pvpq=True, rho=1e5, agc=True), 1, 0.2),
    # contingency screening (eq. (screening)): six contingencies at a fixed
    # first stage, their feasibility problems solved together
    "screen_agc60x6": lambda: (G.make_network(43, 60, 84, 9, 6, pvpq=True, rho=1e5, screen=True, agc=True), 43, 0.1),
    # the smallest AGC networks: one generator and one contingency, and one
    # generator with two contingencies (three outer iterations)
    "agc4x1_g1": lambda: (G.make_network(61, 4, 5, 1, 1, rho=1e5, agc=True), 61, 0.1),
    "agc6x2_g1": lambda: (G.make_network(62, 6, 8, 1, 2, rho=1e5, agc=True), 62, 0.1),
}
EXACT_COUNTS = {"single7", "c1", "agc9", "agc30x3", "screen_agc60x6", "agc4x1_g1", "agc6x2_g1"}


def setup(net, cfg, scale):
    st0 = G.ncl_start(net)
    pd = scale * G.draw_loads(net, cfg)
    N = st0["z"].shape[0]
    prob = I.Problem(pd=pd, lo=st0["lo"], hi=st0["hi"], y_n=np.zeros(N), mu=0.1, rho=net.rho)
    st = I.State(st0["z"], st0["rt"], st0["s"], st0["zl"], st0["zu"])
    gprob = dict(pd=dev(pd), lo=dev(st0["lo"]), hi=dev(st0["hi"]), qd_ratio=prob.qd_ratio, qmax=prob.qmax,
                 pmax=prob.pmax, smax2=prob.smax2, eps=prob.eps, rho=prob.rho)
    if net.screen:
        g = np.random.default_rng(2510)
        prob.pg0, prob.vm0 = g.uniform(1.0, 3.0, net.ng), g.uniform(0.95, 1.05, net.ng)
        gprob["pg0"], gprob["vm0"] = dev(prob.pg0), dev(prob.vm0)
    gst = {k: dev(st0[k]) for k in ("z", "rt", "s", "zl", "zu")}
    gst["y_n"] = dev(np.zeros(N))
    return prob, st, gprob, gst


@pytest.mark.parametrize("which", list(NETS))
def test_ncl_solve_matches_oracle(which):
    net, cfg, scale = NETS[which]()
    prob, st, gprob, gst = setup(net, cfg, scale)
    print(f"[ncl] {which} N={st.z.shape[0]}", flush=True)
    o = NC.Opts()
    st_o, y_o, rep_o = NC.solve(net, prob, st, o)
    assert rep_o.status == 0
    k = KKT(net).bind(nrhs_max=1)
    rep = k.ncl_solve(gprob, gst)
    assert rep["status"] == 0, rep
    assert rep["outer"] == rep_o.outer and rep["rho"] == rep_o.rho, (rep, rep_o)
    exact = which in EXACT_COUNTS
    if exact:
        assert rep["inner"] == rep_o.inner, (rep, rep_o)
    assert rep["r_inf"] <= o.tol and rep["kkt_err"] <= o.tol
    m = I.masks(net, prob)
    z, z_o = host(gst["z"]), st_o.z
    pm = m.primal
    tp = 1e-5 if exact else 1e-4
    assert np.abs(z[pm] - z_o[pm]).max() <= tp * max(1.0, np.abs(z_o[pm]).max())
    if exact:
        # off the exact path the multipliers of biactive complementarity
        # pairs are not unique; the residual check below validates them
        assert np.abs(z[~pm] - z_o[~pm]).max() <= 1e-4 * max(1.0, np.abs(z_o[~pm]).max())
    # the GPU's point is a solution by the oracle's own residual
    sg = I.State(z, host(gst["rt"]), host(gst["s"]), host(gst["zl"]), host(gst["zu"]))
    pfin = I.Problem(pd=prob.pd, lo=prob.lo, hi=prob.hi, y_n=host(gst["y_n"]), mu=0.0, rho=rep["rho"],
                     pg0=prob.pg0, vm0=prob.vm0)
    G0 = I.kkt_residual(net, sg, pfin, m)
    assert np.abs(G0).max() <= o.tol


def test_ncl_solve_bitwise_repeatable():
    net, cfg, scale = NETS["agc9"]()
    _, _, gprob, gst = setup(net, cfg, scale)
    _, _, _, gst2 = setup(net, cfg, scale)
    k = KKT(net).bind(nrhs_max=1)
    r1 = k.ncl_solve(gprob, gst)
    r2 = k.ncl_solve(gprob, gst2)
    assert r1 == r2
    for n in gst:
        assert torch.equal(gst[n], gst2[n]), n


def test_ncl_solve_limits_and_bad_options():
    net, cfg, scale = NETS["agc9"]()
    _, _, gprob, gst = setup(net, cfg, scale)
    k = KKT(net).bind(nrhs_max=1)
    rep = k.ncl_solve(gprob, gst, SolveOpts(max_inner=3))
    assert rep["status"] == 2 and rep["inner"] == 3 and rep["outer"] == 1
    with pytest.raises(NclError):
        k.ncl_solve(gprob, gst, SolveOpts(kappa_mu=1.5))
    with pytest.raises(NclError):
        k.ncl_solve(gprob, gst, SolveOpts(rho_max=1.0))
    # a start that is not strictly interior is refused before any iteration
    net, cfg, scale = NETS["agc9"]()
    _, st, gprob, gst = setup(net, cfg, scale)
    m = I.masks(net, I.Problem(pd=np.zeros(net.nb), lo=G.ncl_bounds(net)[0], hi=G.ncl_bounds(net)[1],
                               y_n=np.zeros(st.z.shape[0])))
    for name, idx, val in (("z", int(np.flatnonzero(m.has_lo)[0]), -1.0), ("s", int(np.flatnonzero(m.ineq)[0]), 0.0),
                           ("zu", int(np.flatnonzero(m.has_hi)[0]), 0.0), ("rt", int(np.flatnonzero(m.dual)[0]), np.nan)):
        bad = {n: t.clone() for n, t in gst.items()}
        bad[name][idx] = val
        before = bad["z"].clone()
        with pytest.raises(NclError):
            k.ncl_solve(gprob, bad)
        assert torch.equal(bad["z"], before)


def test_ncl_solve_500bus_256_contingencies_agc():
    """The NCL workload at full size: the 500-bus x 256 grid with PV/PQ and
    AGC droop rows.  The oracle's loop is too slow here, so the GPU's final
    point is checked by what holds at any size: converged, and the oracle's
    barrier KKT residual at mu = 0 (at the final y_n and rho) within the
    tolerance; every generator of every contingency on its droop rule."""
    net = G.config_network(7)
    prob, st, gprob, gst = setup(net, 7, 0.1)
    print(f"[ncl] 500x256 agc N={st.z.shape[0]}", flush=True)
    k = KKT(net).bind(nrhs_max=1)
    rep = k.ncl_solve(gprob, gst)
    assert rep["status"] == 0 and rep["r_inf"] <= 1e-6 and rep["kkt_err"] <= 1e-6, rep
    m = I.masks(net, prob)
    sg = I.State(host(gst["z"]), host(gst["rt"]), host(gst["s"]), host(gst["zl"]), host(gst["zu"]))
    pfin = I.Problem(pd=prob.pd, lo=prob.lo, hi=prob.hi, y_n=host(gst["y_n"]), mu=0.0, rho=rep["rho"])
    assert np.abs(I.kkt_residual(net, sg, pfin, m)).max() <= 1e-6
    from oracle.assemble import Positions
    pos = Positions(net)
    z = sg.z
    target = z[pos.pg][None, :] + net.gen_alpha[None, :] * z[pos.delta[1:]][:, None]
    assert np.abs(z[pos.pgk[1:]] - np.clip(target, 0.0, prob.pmax)).max() <= 1e-3


def test_ncl_solve_iteration_log():
    """The optional iteration log: one record per inner iteration, the outer
    index of each matching the oracle's iterations per subproblem, the
    barrier parameter non-increasing inside a subproblem, step lengths in
    (0, 1], and the penalty of the record its subproblem's."""
    from paper_2510_13333_amd.ncl import NCL_TRACE_W
    net, cfg, scale = NETS["agc9"]()
    prob, st, gprob, gst = setup(net, cfg, scale)
    _, _, rep_o = NC.solve(net, prob, st)
    k = KKT(net).bind(nrhs_max=1)
    tr = np.full((200, NCL_TRACE_W), np.nan)
    rep = k.ncl_solve(gprob, gst, SolveOpts(trace=tr))
    n = rep["inner"]
    assert np.isfinite(tr[:n]).all() and np.isnan(tr[n:]).all()
    per_outer = np.bincount(tr[:n, 0].astype(int), minlength=rep["outer"])
    assert list(per_outer) == [h[0] for h in rep_o.history]
    for o in range(rep["outer"]):
        mu = tr[:n][tr[:n, 0] == o, 1]
        assert (np.diff(mu) <= 0).all()
    assert ((tr[:n, 6] > 0) & (tr[:n, 6] <= 1) & (tr[:n, 7] > 0) & (tr[:n, 7] <= 1)).all()
    assert (tr[:n, 8] == net.rho).all()
    # a log shorter than the run keeps its first records only
    _, _, gprob2, gst2 = setup(net, cfg, scale)
    short = np.full((5, NCL_TRACE_W), np.nan)
    k.ncl_solve(gprob2, gst2, SolveOpts(trace=short))
    np.testing.assert_array_equal(short, tr[:5])
