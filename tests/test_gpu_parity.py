"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars (FP64 throughout):
* assembly: every K entry within 1e-12 * (|K_ij| + max_{j' != i} |K_ij'|);
* factors: the oracle factors the K values the GPU assembled (so that
  assembly rounding, bounded above relative to each row's largest entry,
  does not count against the factorisation), and every entry of D
  (relative) and of L (of max(1, |L|)) agrees within 1e-8 plus ten times
  its own rounding sensitivity: the largest change of that entry in the
  oracle's factors when every K value is perturbed by one ulp (two random
  perturbations) or when the oracle is built with FMA contraction.  The
  pivot-free LDL^T is unique but some entries are ill-conditioned: at the
  500-bus x 256 state 49 one ulp of K moves 43 pivots by more than 1e-8
  (up to 8e-7), and two pivots formed by a 2e9-fold cancellation carry a
  3e-8 rounding error in the FP64 oracle itself (against an extended-
  precision factorisation of the same K);
* solve: relative solution error <= 1e-8 and normwise backward error
  <= 1e-12, the residual taken with the oracle-assembled K;
* inertia (n, m) and status NCL_OK; run-to-run results bitwise equal;
  solve_adjoint bitwise equal to solve.
"""
import numpy as np
import pytest

import gridgen as G
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2510_13333_amd import KKT  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def small_pvpq():
    return G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5)


def check_assembly(kv, cp, ri, v):
    N = cp.shape[0] - 1
    col = np.repeat(np.arange(N), np.diff(cp))
    off = ri != col
    rowmax = np.zeros(N)
    np.maximum.at(rowmax, ri[off], np.abs(v[off]))
    np.maximum.at(rowmax, col[off], np.abs(v[off]))
    tol = 1e-12 * (np.abs(v) + np.maximum(rowmax[ri], rowmax[col]))
    err = np.abs(kv - v)
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, f"{bad.size} entries off, first at {bad[:5]}: {kv[bad[:5]]} vs {v[bad[:5]]}"


def factor_sensitivity(F, cp, ri, v, perm=None):
    """Per-entry rounding sensitivity of the oracle's (L, D): the largest
    change of each entry under one-ulp random-sign perturbations of K (two
    of them) and under the oracle's FMA build (same arithmetic, other
    rounding: it shows the entries formed by exact cancellation of large
    terms, which a perturbation of K leaves alone); d relative, L of
    max(1, |L|)."""
    d0, l0 = F.d.copy(), F.lx.copy()
    sd, sl = np.zeros_like(d0), np.zeros_like(l0)
    P = O.Factor(F.N, cp, ri, F.block_off, perm=perm)
    runs = [(P, v * (1.0 + 2.0 ** -52 * np.random.default_rng(seed).choice([-1.0, 1.0], size=v.shape)))
            for seed in (1, 2)]
    if O.host_has_fma():
        runs.append((O.Factor(F.N, cp, ri, F.block_off, perm=perm, fma=True), v))
    for Q, vals in runs:
        assert Q.factor(cp, ri, vals, nthreads=8) == 0
        sd = np.maximum(sd, np.abs(Q.d - d0) / np.abs(d0))
        sl = np.maximum(sl, np.abs(Q.lx - l0) / np.maximum(1.0, np.abs(l0)))
    return sd, sl


def check_factors(k, F, cp, ri, v, perm=None):
    """The handle's factors against the oracle's factorisation of the
    handle's own K values (F: an oracle Factor of the same pattern and
    order; refactored here)."""
    v = k.get_values().cpu().numpy()
    assert F.factor(cp, ri, v, nthreads=8) == 0
    lx, d = k.get_factors()
    sd, sl = factor_sensitivity(F, cp, ri, v, perm)
    ed = np.abs(d - F.d) / np.abs(F.d)
    el = np.abs(lx - F.lx) / np.maximum(1.0, np.abs(F.lx))
    bd, bl = np.flatnonzero(ed > 1e-8 + 10 * sd), np.flatnonzero(el > 1e-8 + 10 * sl)
    assert bd.size == 0, f"{bd.size} pivots off, first {bd[:5]}: err {ed[bd[:5]]} sensitivity {sd[bd[:5]]}"
    assert bl.size == 0, f"{bl.size} L entries off, first {bl[:5]}: err {el[bl[:5]]} sensitivity {sl[bl[:5]]}"
    return lx, d


def run_case(net, cfg, nrhs=1, iteration=0, factors=True, k=None, state=None):
    z, s = G.draw_point(net, cfg, iteration=iteration) if state is None else state
    if k is None:
        k = KKT(net).bind(nrhs_max=nrhs)
    k.assemble(dev(z), dev(s), net.rho)
    cp, ri, v, pos = O.kkt(net, z, s)
    kv = k.get_values().cpu().numpy()
    check_assembly(kv, cp, ri, v)
    k.factor()
    info = k.info()
    assert info["status"] == 0, info
    assert info["npos"] == pos.is_primal.sum() and info["nneg"] == (~pos.is_primal).sum()
    F = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
    assert F.factor(cp, ri, v, nthreads=8) == 0
    if factors:
        check_factors(k, F, cp, ri, v)
        assert F.factor(cp, ri, v, nthreads=8) == 0
    B = G.draw_rhs(pos.N, nrhs, cfg, iteration=iteration)
    X = k.solve(dev(B)).cpu().numpy()
    Xo = F.solve(B)
    rel = np.abs(X - Xo).max() / np.abs(Xo).max()
    eta = O.backward_error(cp, ri, v, X, B)
    assert rel <= 1e-8, rel
    assert eta <= 1e-12, eta
    return k, (z, s, B, X)


def test_c1_four_rhs():
    run_case(G.config_network(1), 1, nrhs=4)


def test_pvpq_border_small():
    run_case(small_pvpq(), 99, nrhs=2)


def test_tiny_networks():
    run_case(G.make_network(7, 2, 1, 1, 0), 7)
    run_case(G.make_network(8, 5, 6, 2, 1), 8)           # one contingency, border of 2
    run_case(G.make_network(9, 6, 8, 2, 1, pvpq=True, rho=1e5), 9)


def test_c2_refactor_same_pattern():
    net = G.config_network(2)
    k = None
    for it in range(3):
        k, _ = run_case(net, 2, iteration=it, factors=(it == 0), k=k)


def test_c3_full_size():
    run_case(G.config_network(3), 3, factors=False)


def test_c3_trajectory_states_four_rhs():
    """500-bus x 256 with PV/PQ rows at trajectory states 0, 24 and 49 (the
    last), four right-hand sides each; the factors compared at state 49."""
    net = G.config_network(3)
    z0, s0 = G.draw_point(net, 3)
    k = None
    for it in (0, 24, 49):
        st = G.draw_trajectory_point(net, 3, it, z0, s0)
        k, _ = run_case(net, 3, nrhs=4, iteration=it, factors=(it == 49), k=k, state=st)


def test_border_over_216_factors():
    """A 230-generator border takes the blocked border factor (panel and
    trailing-update launches) and the border solve from global memory."""
    net = G.make_network(31, 1300, 1820, 230, 3, rho=1e4)
    k, _ = run_case(net, 31, nrhs=2)
    assert k.instances[0]["nbd"] == 230


def test_c5_shift_on_factors():
    run_case(G.config_network(5), 5, factors=True)


@pytest.mark.parametrize("pvpq", [True, False])
def test_agc_small(pvpq):
    """AGC droop rows (eq. droopmpec) in the contingency blocks: the block's
    own generation, pi+-, the two slacks and the adjustment column delta
    (one entry per generator), with and without the PV/PQ rows."""
    net = G.make_network(99, 9, 12, 3, 2, pvpq=pvpq, rho=1e5, agc=True)
    run_case(net, 99, nrhs=2)


@pytest.mark.parametrize("pvpq", [False, True])
def test_agc_degenerate_sizes(pvpq):
    """One generator (delta's column has one entry), one or two contingencies."""
    for nb, nl, ng, K, seed in ((4, 5, 1, 1, 61), (6, 8, 1, 2, 62), (5, 7, 2, 1, 63)):
        run_case(G.make_network(seed, nb, nl, ng, K, pvpq=pvpq, rho=1e5, agc=True), seed, nrhs=2)


def test_agc_screening():
    """Screening with AGC rows: no pg0 column in ALIN, no border."""
    net = G.make_network(43, 60, 84, 9, 6, pvpq=True, rho=1e5, screen=True, agc=True)
    k, _ = run_case(net, 43, nrhs=2)
    assert k.instances[0]["nbd"] == 0


def test_agc_full_size():
    """The 500-bus x 256 grid with PV/PQ and AGC rows (5201-column
    contingency blocks), two states, factors compared at the second."""
    net = G.config_network(7)
    k, _ = run_case(net, 7, factors=False)
    run_case(net, 7, iteration=1, factors=True, k=k)


def test_uniform_topology():
    net = G.make_network(32, 300, 420, 54, 12, pvpq=True, rho=1e5, topology="uniform")
    run_case(net, 32, nrhs=2)


def test_determinism_and_adjoint():
    net = G.config_network(2)
    k, (z, s, B, X) = run_case(net, 2, nrhs=2, factors=False)
    lx1, d1 = k.get_factors()
    Bd = dev(B)
    X1 = k.solve(Bd).cpu().numpy()
    k.assemble(dev(z), dev(s), net.rho)
    k.factor()
    lx2, d2 = k.get_factors()
    X2 = k.solve(Bd).cpu().numpy()
    Xa = k.solve_adjoint(Bd).cpu().numpy()
    assert np.array_equal(lx1, lx2) and np.array_equal(d1, d2)
    assert np.array_equal(X1, X2) and np.array_equal(X1, Xa)
    # in-place solve (dx aliases db)
    Bi = dev(B)
    k.solve(Bi, out=Bi)
    assert np.array_equal(Bi.cpu().numpy(), X1)


@pytest.mark.parametrize("cfg", [2, 3])
def test_multi_rhs_bitwise_equals_single(cfg):
    """Every launch of a solve covers all right-hand sides; each column's
    arithmetic is the single-column solve's, bit for bit (also the adjoint
    solve and a leading dimension above N)."""
    net = G.config_network(cfg)
    z, s = G.draw_point(net, cfg)
    k = KKT(net).bind(nrhs_max=4)
    k.assemble(dev(z), dev(s), net.rho)
    k.factor()
    B = G.draw_rhs(k.N, 4, cfg, iteration=3)
    Bp = np.zeros((4, k.N + 7))
    Bp[:, :k.N] = B
    Bd = dev(Bp)[:, :k.N]                      # leading dimension N + 7
    X4 = torch.empty((4, k.N + 7), dtype=torch.float64, device="cuda")
    k._solve_ld(Bd, X4, k.N + 7)
    X4 = X4[:, :k.N].cpu().numpy()
    Xa = k.solve_adjoint(dev(B)).cpu().numpy()
    for r in range(4):
        x1 = k.solve(dev(B[r])).cpu().numpy()
        assert np.array_equal(X4[r], x1), r
        assert np.array_equal(Xa[r], x1), r


def test_set_values_seam_random_quasidefinite():
    """Arbitrary quasi-definite values on a block-arrowhead pattern through
    ncl_kkt_analyze_pattern / ncl_kkt_set_values."""
    net = G.make_network(2, 30, 41, 6, 3)
    k0 = KKT(net)
    cp, ri = k0.pattern()
    z, s = G.draw_point(net, 2)
    _, _, _, pos = O.kkt(net, z, s)
    g = np.random.default_rng(3)
    v = g.standard_normal(cp[-1])
    col = np.repeat(np.arange(pos.N), np.diff(cp))
    diag = ri == col
    # make the primal block diagonally dominant and the dual diagonal negative
    rowabs = np.zeros(pos.N)
    np.add.at(rowabs, ri[~diag], np.abs(v[~diag]))
    np.add.at(rowabs, col[~diag], np.abs(v[~diag]))
    prim = pos.is_primal
    dv = np.where(prim[col[diag]], rowabs[col[diag]] + 10.0 ** g.uniform(-3, 3, diag.sum()),
                  -(10.0 ** g.uniform(-6, 0, diag.sum())))
    v[diag] = dv
    k = KKT(pattern=(pos.N, np.array(pos.block_off), cp, ri, prim.astype(np.uint8))).bind()
    k.set_values(dev(v))
    k.factor()
    info = k.info()
    assert info["status"] == 0 and info["npos"] == prim.sum()
    F = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
    assert F.factor(cp, ri, v) == 0
    lx, d = k.get_factors()
    np.testing.assert_allclose(d, F.d, rtol=1e-10)
    b = G.draw_rhs(pos.N, 1, 2)
    x = k.solve(dev(b)).cpu().numpy()
    assert O.backward_error(cp, ri, v, x, b) <= 1e-13


def test_wrong_sign_pivot_reported():
    """A primal diagonal made negative: the factorisation completes (finite
    numbers) and reports NCL_ERR_INERTIA at the first wrong-sign pivot."""
    net = G.config_network(1)
    k0 = KKT(net)
    cp, ri = k0.pattern()
    z, s = G.draw_point(net, 1)
    cpo, rio, v, pos = O.kkt(net, z, s)
    col = np.repeat(np.arange(pos.N), np.diff(cp))
    j = int(np.flatnonzero(pos.is_primal)[5])
    q = np.flatnonzero((ri == j) & (col == j))[0]
    v = v.copy()
    v[q] = -1e9
    k = KKT(pattern=(pos.N, np.array(pos.block_off), cp, ri, pos.is_primal.astype(np.uint8))).bind()
    k.set_values(dev(v))
    k.factor()
    info = k.info()
    assert info["status"] == -6
    F = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
    F.factor(cp, ri, v)
    prim_new = pos.is_primal[F.perm]
    wrong = np.flatnonzero((F.d > 0) != prim_new)
    assert info["first_bad"] == wrong[0]


@pytest.mark.parametrize("which", ["c1", "pvpq", "c2", "big_border", "c3", "agc"])
def test_factor_solve_equals_factor_then_solve(which):
    """The combined call (the border factored on a second stream while the
    blocks' forward substitution runs) gives the bits of factor + solve."""
    nets = {"c1": lambda: (G.config_network(1), 1), "pvpq": lambda: (small_pvpq(), 99),
            "c2": lambda: (G.config_network(2), 2), "c3": lambda: (G.config_network(3), 3),
            "big_border": lambda: (G.make_network(31, 1300, 1820, 230, 3, rho=1e4), 31),
            "agc": lambda: (G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True), 99)}
    net, cfg = nets[which]()
    k = KKT(net).bind(nrhs_max=2)
    for it in range(2):
        z, s = G.draw_point(net, cfg, iteration=it)
        b = dev(G.draw_rhs(k.N, 2, cfg, iteration=it))
        k.assemble(dev(z), dev(s), net.rho)
        k.factor()
        x0 = k.solve(b)
        info0 = k.info()
        x1 = k.factor_solve(b)
        info1 = k.info()
        assert torch.equal(x0, x1), which
        assert info0 == info1
        # and after the combined call the factors serve further solves
        assert torch.equal(k.solve(b), x0)


def test_factor_solve_failed_factor_gives_nan():
    net = G.config_network(1)
    k0 = KKT(net)
    cp, ri = k0.pattern()
    z, s = G.draw_point(net, 1)
    cpo, rio, v, pos = O.kkt(net, z, s)
    col = np.repeat(np.arange(pos.N), np.diff(cp))
    j = int(np.flatnonzero(pos.is_primal)[5])
    q = np.flatnonzero((ri == j) & (col == j))[0]
    v = v.copy()
    v[q] = -1e9
    k = KKT(pattern=(pos.N, np.array(pos.block_off), cp, ri, pos.is_primal.astype(np.uint8))).bind()
    k.set_values(dev(v))
    x = k.factor_solve(dev(G.draw_rhs(pos.N, 1, 1)[0]))
    assert torch.isnan(x).all()
    info = k.info()
    assert info["status"] == -6 and info["solvable"] == 0
