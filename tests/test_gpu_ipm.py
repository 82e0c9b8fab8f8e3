"""GPU parity of the IPM step of the NCL subproblem (Section IV-A eq.
(nclsubpb), eq. (kktncl) in barrier form, eq. (newtonsystem) and the
recovery of the eliminated directions; the inertia correction of Section
V-C) against the oracle, through the C ABI, on the same seeded points.

Bars (FP64):
* sigma: within 4 ulp of the oracle's (divisions and at most three adds);
* right-hand side: each entry within 1e-12 of its own magnitude scale
  (1 + |r_i| + the sum of |terms| that form it, the Jacobian terms taken
  as sum_j |J_ij| |y_j| on primal rows and sum_j |J_ij| on dual rows);
* recovery, from the same dz: within 1e-14 of each formula's term scale;
* inertia correction: the same shift and number of factorisations as the
  oracle's loop (both decide on FP64 pivot signs of the same matrix), and
  at the 500-bus x 256 size: the oracle's inertia of the accepted matrix
  is (n, m) and that of the previous shift is not;
* the step: dz within 1e-8 of max |dz| and with normwise backward error
  <= 1e-12 against the oracle-assembled shifted matrix; the recovered
  directions within 1e-8 of their max.
"""
import numpy as np
import pytest

import gridgen as G
import oracle as O
from oracle import ipm as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2510_13333_amd import KKT  # noqa: E402
from paper_2510_13333_amd.ncl import InertiaOpts  # noqa: E402

EPS = np.finfo(float).eps

NETS = {
    "pvpq9": lambda: (G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5), 99),
    "plain5": lambda: (G.make_network(8, 5, 6, 2, 1, rho=1e3), 8),
    "single30": lambda: (G.make_network(6, 30, 41, 6, 0, rho=1e3), 6),
    "pvpq200x8": lambda: (G.make_network(13, 200, 280, 36, 8, pvpq=True, rho=1e5), 13),
    "agc9": lambda: (G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True), 99),
    "agc118x8": lambda: (G.make_network(5, 118, 165, 21, 8, pvpq=True, rho=1e5, agc=True), 5),
    "screen60x6": lambda: (G.make_network(43, 60, 84, 9, 6, pvpq=True, rho=1e5, screen=True), 43),
    "screen_agc60x6": lambda: (G.make_network(43, 60, 84, 9, 6, pvpq=True, rho=1e5, screen=True, agc=True), 43),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda")


def host(t):
    return t.cpu().numpy()


def setup(net, cfg, iteration=0):
    d, pd = G.draw_ipm_point(net, cfg, iteration=iteration)
    prob = I.Problem(pd=pd, lo=d["lo"], hi=d["hi"], y_n=d["y_n"], mu=0.1, rho=net.rho)
    st = I.State(d["z"], d["rt"], d["s"], d["zl"], d["zu"])
    gprob = dict(pd=dev(pd), lo=dev(d["lo"]), hi=dev(d["hi"]), y_n=dev(d["y_n"]), qd_ratio=prob.qd_ratio,
                 qmax=prob.qmax, pmax=prob.pmax, smax2=prob.smax2, eps=prob.eps, mu=prob.mu, rho=prob.rho)
    if net.screen:
        # the fixed first stage of a screening network (seeded)
        g = np.random.default_rng(2510)
        prob.pg0, prob.vm0 = g.uniform(1.0, 3.0, net.ng), g.uniform(0.95, 1.05, net.ng)
        gprob["pg0"], gprob["vm0"] = dev(prob.pg0), dev(prob.vm0)
    gst = {k: dev(d[k]) for k in ("z", "rt", "s", "zl", "zu")}
    return prob, st, gprob, gst


def empty(n):
    return torch.empty(n, dtype=torch.float64, device="cuda")


def full_abs(cp, ri, v):
    import scipy.sparse as sp
    N = cp.shape[0] - 1
    Lw = sp.csc_matrix((np.abs(v), ri, cp), shape=(N, N))
    return (Lw + Lw.T - sp.diags(Lw.diagonal())).tocsr()


def rhs_scale(net, st, prob, m, cp, ri, v):
    """Magnitude scale of every right-hand-side entry (see the module doc)."""
    A = full_abs(cp, ri, v)
    z = st.z
    lo, hi = prob.lo, prob.hi
    y = np.where(m.dual, np.abs(z), 0.0)
    onep = np.where(m.primal, 1.0, 0.0)
    s = np.where(m.primal, A @ y, A @ onep)
    s += np.abs(I.grad_lagrangian(net, z, prob, m)) + np.abs(I.constraints(net, z, prob, m))
    with np.errstate(divide="ignore", invalid="ignore"):
        s += np.where(m.has_lo, prob.mu / np.abs(z - lo), 0.0) + np.where(m.has_hi, prob.mu / np.abs(hi - z), 0.0)
        s += np.where(m.dual, np.abs(z - prob.y_n) / prob.rho, 0.0)
        s += np.where(m.ineq, prob.mu / np.abs(z), 0.0)
        s += np.where(m.flow, prob.smax2, 0.0)
    return s


def check_pieces(net, cfg, iteration=0):
    prob, st, gprob, gst = setup(net, cfg, iteration)
    m = I.masks(net, prob)
    k = KKT(net).bind(nrhs_max=1)
    N = k.N
    sg = host(k.ipm_sigma(gprob, gst, empty(N)))
    sg_o = I.sigma(net, st, prob, m)
    assert np.all(np.abs(sg - sg_o) <= 4 * EPS * np.abs(sg_o)), np.abs(sg - sg_o).max()
    # right-hand side, J'y from K assembled at this z
    k.assemble(gst["z"], dev(sg_o), prob.rho, shift=False)
    r = host(k.ipm_rhs(gprob, gst, empty(N), empty(2 * N)))
    r_o = I.reduced_rhs(net, st, prob, m)
    cp, ri, v = I.newton_matrix(net, st, prob, 0.0, m)
    scale = 1.0 + np.abs(r_o) + rhs_scale(net, st, prob, m, cp, ri, v)
    err = np.abs(r - r_o) / scale
    assert err.max() <= 1e-12, (err.max(), int(err.argmax()))
    # recovery from one seeded dz
    dz = np.random.default_rng(cfg).standard_normal(N)
    out = {n: empty(N) for n in ("drt", "ds", "dzl", "dzu")}
    k.ipm_recover(gprob, gst, dev(dz), out)
    d_o = I.recover(net, st, prob, dz, m)
    z, lo, hi = st.z, prob.lo, prob.hi
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        sc = {
            "drt": np.where(m.dual, (np.abs(dz) + np.abs(z) + np.abs(prob.y_n) + prob.rho * np.abs(st.rt)) / prob.rho,
                            0.0),
            "ds": np.where(m.ineq, prob.mu / np.abs(z) + st.s + st.s / np.abs(z) * np.abs(dz), 0.0),
            "dzl": np.where(m.has_lo, (prob.mu + np.abs(z - lo) * st.zl + st.zl * np.abs(dz)) / np.abs(z - lo), 0.0),
            "dzu": np.where(m.has_hi, (prob.mu + np.abs(hi - z) * st.zu + st.zu * np.abs(dz)) / np.abs(hi - z), 0.0),
        }
    for name, ref in (("drt", d_o.rt), ("ds", d_o.s), ("dzl", d_o.zl), ("dzu", d_o.zu)):
        got = host(out[name])
        assert np.all(np.abs(got - ref) <= 1e-14 * sc[name]), (name, np.abs(got - ref).max())
    return k, prob, st, gprob, gst, m


@pytest.mark.parametrize("which", list(NETS))
def test_sigma_rhs_recovery_match_oracle(which):
    net, cfg = NETS[which]()
    check_pieces(net, cfg)


@pytest.mark.parametrize("which,iteration", [("pvpq9", 0), ("pvpq9", 1), ("pvpq9", 2), ("plain5", 0),
                                             ("single30", 0), ("pvpq200x8", 0), ("pvpq200x8", 1), ("agc9", 0),
                                             ("agc118x8", 1)])
def test_inertia_correction_matches_oracle(which, iteration):
    net, cfg = NETS[which]()
    prob, st, gprob, gst = setup(net, cfg, iteration)
    m = I.masks(net, prob)
    k = KKT(net).bind(nrhs_max=1)
    sg = k.ipm_sigma(gprob, gst, empty(k.N))
    opts = InertiaOpts(0.0, 0, 0)
    k.factor_inertia(gst["z"], sg, prob.rho, opts, empty(k.N))
    dw_o, nfac_o, _, _ = I.inertia_correction(net, st, prob, 0.0, m)
    assert (opts.dw_last, opts.nfactor) == (dw_o, nfac_o)
    rep = k.info()
    assert rep["npos"] == int(m.primal.sum()) and rep["nneg"] == int(m.dual.sum()) and rep["solvable"] == 1
    # restarting from the accepted shift: the sequence starts at a third of it
    if dw_o > 0:
        opts2 = InertiaOpts(dw_o, 0, 0)
        k.factor_inertia(gst["z"], sg, prob.rho, opts2, empty(k.N))
        dw2, nfac2, _, _ = I.inertia_correction(net, st, prob, dw_o, m)
        assert (opts2.dw_last, opts2.nfactor) == (dw2, nfac2)


def step_direction(k, gprob, gst, dw_last=0.0):
    N = k.N
    d = {n: empty(N) for n in ("dz", "drt", "ds", "dzl", "dzu")}
    opts = InertiaOpts(dw_last, 0, 0)
    k.ipm_step(gprob, gst, d, opts, empty(3 * N))
    return {n: host(t) for n, t in d.items()}, opts


@pytest.mark.parametrize("which", list(NETS))
def test_ipm_step_matches_oracle_step(which):
    net, cfg = NETS[which]()
    prob, st, gprob, gst = setup(net, cfg, 1)
    k = KKT(net).bind(nrhs_max=1)
    d, opts = step_direction(k, gprob, gst)
    d_o, dw_o, nfac_o = I.step(net, st, prob)
    assert (opts.dw_last, opts.nfactor) == (dw_o, nfac_o)
    m = I.masks(net, prob)
    cp, ri, v = I.newton_matrix(net, st, prob, dw_o, m)
    r_o = I.reduced_rhs(net, st, prob, m)
    assert O.backward_error(cp, ri, v, d["dz"], r_o) <= 1e-12
    assert np.abs(d["dz"] - d_o.z).max() <= 1e-8 * np.abs(d_o.z).max()
    for name, ref in (("drt", d_o.rt), ("ds", d_o.s), ("dzl", d_o.zl), ("dzu", d_o.zu)):
        if np.abs(ref).max() > 0:
            assert np.abs(d[name] - ref).max() <= 1e-8 * np.abs(ref).max(), name
    # bitwise repeatable
    d2, _ = step_direction(k, gprob, gst)
    assert all(np.array_equal(d[n], d2[n]) for n in d)


def test_ipm_step_500bus_256_contingencies():
    """The full-size step: sigma, right-hand side and recovery against the
    oracle entry by entry; the accepted shift checked by the oracle's own
    factorisation (inertia (n, m) there, not at the previous shift); dz by
    its backward error against the oracle-assembled shifted matrix."""
    net, cfg = G.config_network(3), 3
    k, prob, st, gprob, gst, m = check_pieces(net, cfg)
    d, opts = step_direction(k, gprob, gst)
    nprim, N = int(m.primal.sum()), m.primal.shape[0]
    F = O.Factor.from_network(net)
    cp, ri, v = I.newton_matrix(net, st, prob, opts.dw_last, m)
    F.factor(cp, ri, v, nthreads=8)
    assert I.inertia_ok(F.inertia, nprim, N)
    seq = list(I.shift_sequence(0.0))
    assert seq[opts.nfactor - 1] == opts.dw_last
    if opts.nfactor > 1:
        F.factor(*I.newton_matrix(net, st, prob, seq[opts.nfactor - 2], m), nthreads=8)
        assert not I.inertia_ok(F.inertia, nprim, N)
    r_o = I.reduced_rhs(net, st, prob, m)
    assert O.backward_error(cp, ri, v, d["dz"], r_o) <= 1e-12
    d_o = I.recover(net, st, prob, d["dz"], m)
    for name, ref in (("drt", d_o.rt), ("ds", d_o.s), ("dzl", d_o.zl), ("dzu", d_o.zu)):
        assert np.abs(d[name] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), name


def test_ipm_rejects_screening_without_first_stage_and_bad_arguments():
    net = G.make_network(43, 60, 84, 9, 6, pvpq=True, rho=1e5, screen=True)
    k = KKT(net).bind(nrhs_max=1)
    N = k.N
    z = empty(N).fill_(1.0)
    gprob = dict(pd=empty(net.nb), lo=z, hi=z, y_n=z, qd_ratio=0.3, qmax=3.0, smax2=100.0, eps=1.0, mu=0.1, rho=1e5)
    gst = dict(z=z, rt=z, s=z, zl=z, zu=z)
    from paper_2510_13333_amd.ncl import NclError
    with pytest.raises(NclError):
        k.ipm_sigma(gprob, gst, empty(N))
    gprob["pg0"] = empty(net.ng).fill_(1.0)          # PV/PQ rows need vm0 too
    with pytest.raises(NclError):
        k.ipm_sigma(gprob, gst, empty(N))
    net2, cfg = NETS["pvpq9"]()
    prob, st, gprob2, gst2 = setup(net2, cfg)
    k2 = KKT(net2).bind(nrhs_max=1)
    gprob2["mu"] = 0.0
    with pytest.raises(NclError):
        k2.ipm_sigma(gprob2, gst2, empty(k2.N))
