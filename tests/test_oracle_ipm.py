"""Pins of the IPM-step oracle (CPU).

* The gradient of the Lagrangian, written from the derivative formulas,
  equals the complex-step gradient of phi + y'c(w) (c from its value
  formulas); the balance and flow rows agree with the dispatch map's
  residual, an independent writing of the same functions.
* The unreduced Newton matrix is the complex-step Jacobian of the barrier
  KKT residual G (exact to rounding, h = 1e-30).  Eliminating zl, zu, s
  and rt from it gives the assembled K (no shift) at the step's sigma, and
  the reduced solve plus the recovery formulas gives the full Newton step
  -M^{-1} G.  A dropped term or a wrong sign in sigma, the right-hand side
  or any recovery formula fails one of these.
* Along the step, the complex-step directional derivative of G is -G.
* The inertia correction takes the first shift of its sequence at which the
  matrix has n positive and m negative eigenvalues (eigvalsh, dense).
"""
import warnings

import numpy as np
import pytest

import gridgen as G
from oracle import assemble as A
from oracle import dispatch as D
from oracle import ipm as I


def first_stage(net):
    """Fixed first-stage values of a screening network (seeded)."""
    g = np.random.default_rng(2510)
    return g.uniform(1.0, 3.0, net.ng), g.uniform(0.95, 1.05, net.ng)


def setup(net, cfg, iteration=0, mu=0.1):
    d, pd = G.draw_ipm_point(net, cfg, iteration=iteration)
    prob = I.Problem(pd=pd, lo=d["lo"], hi=d["hi"], y_n=d["y_n"], mu=mu, rho=net.rho)
    if net.screen:
        prob.pg0, prob.vm0 = first_stage(net)
    st = I.State(d["z"], d["rt"], d["s"], d["zl"], d["zu"])
    return prob, st


NETS = {
    "pvpq": lambda: (G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5), 99),
    "plain": lambda: (G.make_network(8, 5, 6, 2, 1, rho=1e3), 8),
    "single": lambda: (G.make_network(7, 6, 8, 2, 0, rho=1e3), 7),
    "agc": lambda: (G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True), 99),
    "screen": lambda: (G.make_network(41, 24, 33, 5, 3, pvpq=True, rho=1e5, screen=True), 41),
    "screen_agc": lambda: (G.make_network(41, 24, 33, 5, 3, pvpq=True, rho=1e5, screen=True, agc=True), 41),
}


def cstep(fun, x, h=1e-30):
    """Complex-step Jacobian columns of fun at x (fun real-analytic)."""
    cols = []
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for j in range(x.size):
            xc = x.astype(complex)
            xc[j] += 1j * h
            cols.append(np.imag(fun(xc)) / h)
    return np.array(cols).T


@pytest.mark.parametrize("which", list(NETS))
def test_grad_lagrangian_is_complex_step_gradient(which):
    net, cfg = NETS[which]()
    prob, st = setup(net, cfg)
    m = I.masks(net, prob)
    z = st.z
    ip = np.flatnonzero(m.primal)
    y = np.where(m.dual, z, 0.0)

    def lag(w):
        zz = z.astype(complex)
        zz[ip] = w
        return np.atleast_1d(I.objective(net, zz, prob, m) + np.sum(y * I.constraints(net, zz, prob, m)))

    g_cs = cstep(lag, z[ip])[0]
    g = I.grad_lagrangian(net, z, prob, m)[ip]
    assert np.abs(g - g_cs).max() <= 1e-12 * max(1.0, np.abs(g_cs).max())


def test_balance_and_flow_rows_match_dispatch_residual():
    net, cfg = NETS["plain"]()
    prob, st = setup(net, cfg)
    p = D.NLP(mu=0.1, qd_ratio=prob.qd_ratio, smax2=prob.smax2)
    z = st.z.copy()
    F, _ = D.residual(net, z, prob.pd, p)
    c = I.constraints(net, z, prob)
    pos = A.Positions(net)
    for k in range(net.nblk):
        for rows in (pos.rowP[k], pos.rowQ[k]):
            np.testing.assert_allclose(c[rows], F[rows] + z[rows] / net.rho, rtol=0, atol=1e-12)
        for rows in (pos.rowFf[k], pos.rowFt[k]):
            np.testing.assert_allclose(c[rows], F[rows] + z[rows] / net.rho - p.mu / z[rows], rtol=0, atol=1e-11)


def unreduced(net, st, prob):
    m = I.masks(net, prob)
    U = I.Unknowns(m)
    N = st.z.shape[0]
    u0 = U.pack(st)
    M = cstep(lambda u: I.kkt_residual(net, U.unpack(u, N), prob, m), u0)
    G0 = I.kkt_residual(net, st, prob, m)
    return m, U, M, G0


@pytest.mark.parametrize("which", list(NETS))
def test_reduced_matrix_is_schur_complement_of_the_jacobian(which):
    net, cfg = NETS[which]()
    prob, st = setup(net, cfg)
    m, U, M, _ = unreduced(net, st, prob)
    nk = U.off[2]                       # (w, y) come first
    # the Newton equations are M du = -G; the reduced matrix acts on (dw, dy)
    # after the last four unknown groups are eliminated
    A11, A12, A21, A22 = M[:nk, :nk], M[:nk, nk:], M[nk:, :nk], M[nk:, nk:]
    S = A11 - A12 @ np.linalg.solve(A22, A21)
    cp, ri, v = I.newton_matrix(net, st, prob, 0.0, m)
    K = D.full_matrix(cp, ri, v).toarray()
    idx = np.concatenate([U.iw, U.iy])
    Kr = K[np.ix_(idx, idx)]
    scale = np.abs(Kr).max()
    assert np.abs(S - Kr).max() <= 1e-10 * scale, np.abs(S - Kr).max() / scale


@pytest.mark.parametrize("which", list(NETS))
def test_reduced_step_equals_full_newton_step(which):
    net, cfg = NETS[which]()
    prob, st = setup(net, cfg)
    m, U, M, G0 = unreduced(net, st, prob)
    du_full = -np.linalg.solve(M, G0)
    cp, ri, v = I.newton_matrix(net, st, prob, 0.0, m)
    K = D.full_matrix(cp, ri, v).toarray()
    r = I.reduced_rhs(net, st, prob, m)
    dz = np.linalg.solve(K, r)
    d = I.recover(net, st, prob, dz, m)
    du = U.pack(d)
    for a, b, name in zip(np.split(du, U.off[1:-1]), np.split(du_full, U.off[1:-1]),
                          ("dw", "dy", "drt", "ds", "dzl", "dzu")):
        if a.size:
            err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
            assert err <= 1e-8, (name, err)


@pytest.mark.parametrize("which", ["pvpq", "plain", "agc"])
def test_step_is_a_newton_direction(which):
    """d/da G(u + a du) at a = 0 is -G(u), by complex step in a (no matrix)."""
    net, cfg = NETS[which]()
    prob, st = setup(net, cfg, iteration=3)
    m = I.masks(net, prob)
    U = I.Unknowns(m)
    N = st.z.shape[0]
    cp, ri, v = I.newton_matrix(net, st, prob, 0.0, m)
    K = D.full_matrix(cp, ri, v).toarray()
    d = I.recover(net, st, prob, np.linalg.solve(K, I.reduced_rhs(net, st, prob, m)), m)
    u0, du = U.pack(st), U.pack(d)
    h = 1e-30
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        Gd = np.imag(I.kkt_residual(net, U.unpack(u0 + 1j * h * du, N), prob, m)) / h
    G0 = I.kkt_residual(net, st, prob, m)
    assert np.abs(Gd + G0).max() <= 1e-9 * np.abs(G0).max()


def test_recovery_sign_against_printed_form():
    """The printed recovery (opposite signs on the mu term and on d lam) is
    not a Newton step: it fails the full-step comparison on the same point,
    so the pin above distinguishes the two readings."""
    net, cfg = NETS["pvpq"]()
    prob, st = setup(net, cfg)
    m, U, M, G0 = unreduced(net, st, prob)
    du_full = -np.linalg.solve(M, G0)
    cp, ri, v = I.newton_matrix(net, st, prob, 0.0, m)
    K = D.full_matrix(cp, ri, v).toarray()
    dz = np.linalg.solve(K, I.reduced_rhs(net, st, prob, m))
    d = I.recover(net, st, prob, dz, m)
    printed = d.copy()
    dd = m.dual
    printed.rt[dd] = (st.z[dd] + prob.rho * st.rt[dd] - prob.y_n[dd] - dz[dd]) / prob.rho
    b = U.off
    full_rt = du_full[b[2]:b[3]]
    assert np.abs(U.pack(d)[b[2]:b[3]] - full_rt).max() <= 1e-8 * np.abs(full_rt).max()
    assert np.abs(U.pack(printed)[b[2]:b[3]] - full_rt).max() > 1e-3 * np.abs(full_rt).max()


def eig_inertia(cp, ri, v):
    ev = np.linalg.eigvalsh(D.full_matrix(cp, ri, v).toarray())
    return int((ev > 0).sum()), int((ev < 0).sum()), int((ev == 0).sum())


@pytest.mark.parametrize("iteration", [0, 1, 2, 3])
def test_inertia_correction_takes_the_first_good_shift(iteration):
    net, cfg = NETS["pvpq"]()
    prob, st = setup(net, cfg, iteration=iteration)
    m = I.masks(net, prob)
    nprim, N = int(m.primal.sum()), m.primal.shape[0]
    dw, nfac, F, (cp, ri, v) = I.inertia_correction(net, st, prob, 0.0, m)
    assert I.inertia_ok(eig_inertia(cp, ri, v), nprim, N)
    seq = list(I.shift_sequence(0.0))
    assert seq[nfac - 1] == dw
    for prev in seq[:nfac - 1]:
        assert not I.inertia_ok(eig_inertia(*I.newton_matrix(net, st, prob, prev, m)), nprim, N)


def test_inertia_correction_exact_when_already_right():
    """At a point with large bound multipliers (Sigma dominates H) the exact
    matrix has the inertia: no shift, one factorisation."""
    net, cfg = NETS["pvpq"]()
    prob, st = setup(net, cfg)
    m = I.masks(net, prob)
    st.zl[m.has_lo] *= 1e4
    st.zu[m.has_hi] *= 1e4
    # the angles have no bound: pin them with a large reference term and
    # check whether the rest already has the inertia
    prob.eps = 1.0
    cp, ri, v = I.newton_matrix(net, st, prob, 0.0, m)
    good = I.inertia_ok(eig_inertia(cp, ri, v), int(m.primal.sum()), m.primal.shape[0])
    dw, nfac, _, _ = I.inertia_correction(net, st, prob, 0.0, m)
    assert (dw == 0.0 and nfac == 1) == good


def test_shift_sequence_restarts_from_the_last_shift():
    seq = list(I.shift_sequence(3e-2))
    assert seq[0] == 0.0 and seq[1] == pytest.approx(1e-2) and seq[2] == pytest.approx(8e-2)
    seq = list(I.shift_sequence(0.0))
    assert seq[1] == 1e-4 and seq[-1] < 1e12 <= seq[-1] * 8


def test_agc_rows_vanish_on_the_clipped_recourse():
    """eq. (agc): p^k = min(max(p^0 + alpha Delta, pmin), pmax).  With pi+ and
    pi- the parts of p^k - (p^0 + alpha Delta) above and below zero and the
    slacks pmax - p^k, p^k - pmin, the five AGC rows of eq. (droopmpec)
    vanish; pairing pi+ with the upper slack instead does not.  The point
    puts generators on both bounds and inside."""
    net, cfg = NETS["agc"]()
    prob, st = setup(net, cfg)
    pos = A.Positions(net)
    z = st.z.copy()
    ng = net.ng
    z[pos.pg] = np.array([7.5, 0.2, 4.0])[:ng]
    for k in range(1, net.nblk):
        dk = [3.0, -2.0][k - 1]
        z[pos.delta[k]] = dk
        target = z[pos.pg] + net.gen_alpha * dk
        pk = np.clip(target, 0.0, prob.pmax)
        z[pos.pgk[k]] = pk
        pip, pim, spu, spl = pos.acomp[k]
        z[pip] = np.maximum(pk - target, 0.0)
        z[pim] = np.maximum(target - pk, 0.0)
        z[spu] = prob.pmax - pk
        z[spl] = pk
    c = I.constraints(net, z, prob)
    rows = pos.rowA[1:].ravel()
    assert np.abs(c[rows]).max() <= 1e-14
    # the point has generators at pmax, at pmin and inside
    pk = z[pos.pgk[1:].ravel()]
    assert (pk == prob.pmax).any() and (pk == 0.0).any() and ((pk > 0) & (pk < prob.pmax)).any()
    # the other pairing leaves a product nonzero
    for k in range(1, net.nblk):
        pip, pim, spu, spl = pos.acomp[k]
        assert np.abs(z[pip] * z[spu]).max() + np.abs(z[pim] * z[spl]).max() > 0


@pytest.mark.parametrize("agc", [False, True])
def test_screening_blocks_are_the_corrective_contingency_blocks(agc):
    """eq. (screening): with pg0 and vm0 fixed at a corrective state's first
    stage, the screening network's constraint values and Lagrangian
    gradient equal those of the corrective network's contingency blocks at
    the same block states."""
    full = G.make_network(41, 24, 33, 5, 3, pvpq=True, rho=1e5, agc=agc)
    scr = G.make_network(41, 24, 33, 5, 3, pvpq=True, rho=1e5, agc=agc, screen=True)
    prob_f, st_f = setup(full, 41)
    pf, ps = A.Positions(full), A.Positions(scr)
    a, b = pf.block_off[1], pf.block_off[-1]
    prob_s = I.Problem(pd=prob_f.pd, lo=prob_f.lo[a:b], hi=prob_f.hi[a:b], y_n=prob_f.y_n[a:b], mu=prob_f.mu,
                       rho=prob_f.rho, pg0=st_f.z[pf.pg], vm0=st_f.z[pf.vm0])
    zs = st_f.z[a:b]
    c_f = I.constraints(full, st_f.z, prob_f)
    c_s = I.constraints(scr, zs, prob_s)
    np.testing.assert_array_equal(c_s, c_f[a:b])
    g_f = I.grad_lagrangian(full, st_f.z, prob_f)
    g_s = I.grad_lagrangian(scr, zs, prob_s)
    # the contingency blocks' own positions (the corrective gradient also
    # collects the blocks' terms on the border pg and vm0, absent here)
    np.testing.assert_allclose(g_s, g_f[a:b], rtol=1e-14, atol=1e-14)
