"""GPU: the accuracy gate, iterative refinement, the solve guard after a
failed factorisation and caller-given orderings (through the C ABI).

* ncl_kkt_backward_error against the oracle's normwise and componentwise
  backward errors on the same x and the same K values; at an exact solve
  (eta <= 1e-12) and at a perturbed one (where the residual is far above
  rounding and both sides must agree to ~1e-9).
* One refinement step brings the componentwise error to rounding level.
* After a factorisation with the wrong inertia: the device fills x with NaN
  before the status is read; after ncl_kkt_info the solves refuse
  (NCL_ERR_STATE); a good factorisation clears it.
* Every block-respecting ordering factors without pivoting with the right
  pivot signs (Section IV-B, last paragraph), and matches the oracle run on
  the same ordering.
"""
import numpy as np
import pytest

import gridgen as G
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2510_13333_amd import KKT, NclError  # noqa: E402
from tests.test_library_cpu import block_respecting_perm  # noqa: E402
from tests.test_gpu_parity import check_factors  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def small_pvpq():
    return G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5)


def setup(net, cfg, nrhs, iteration=0, perm=None):
    z, s = G.draw_point(net, cfg, iteration=iteration)
    k = KKT(net, perm=perm).bind(nrhs_max=nrhs)
    k.assemble(dev(z), dev(s), net.rho)
    k.factor()
    info = k.info()
    assert info["status"] == 0 and info["solvable"] == 1, info
    cp, ri = k.pattern()
    v = k.get_values().cpu().numpy()
    B = G.draw_rhs(k.N, nrhs, cfg, iteration=iteration)
    return k, (z, s), (cp, ri, v), B


@pytest.mark.parametrize("which", ["c1", "pvpq", "c2"])
def test_backward_error_matches_oracle(which):
    net = {"c1": G.config_network(1), "pvpq": small_pvpq(), "c2": G.config_network(2)}[which]
    cfg = {"c1": 1, "pvpq": 99, "c2": 2}[which]
    nrhs = 3
    k, _, (cp, ri, v), B = setup(net, cfg, nrhs)
    Bd = dev(B)
    X = k.solve(Bd)
    e = k.backward_error(Bd, X).cpu().numpy()
    Xh = X.cpu().numpy()
    for r in range(nrhs):
        eta = O.backward_error(cp, ri, v, Xh[r], B[r])
        assert e[r, 0] <= 1e-12 and eta <= 1e-12, (e[r], eta)
    # perturbed solutions: residuals far above rounding, both sides agree
    g = np.random.default_rng(5)
    Xp = Xh * (1.0 + 1e-7 * g.standard_normal(Xh.shape))
    e = k.backward_error(Bd, dev(Xp)).cpu().numpy()
    for r in range(nrhs):
        eta = O.backward_error(cp, ri, v, Xp[r], B[r])
        om = O.componentwise_backward_error(cp, ri, v, Xp[r], B[r])
        assert e[r, 0] == pytest.approx(eta, rel=1e-9), (r, e[r, 0], eta)
        assert e[r, 1] == pytest.approx(om, rel=1e-9), (r, e[r, 1], om)


def test_backward_error_sees_nan():
    net = G.config_network(1)
    k, _, _, B = setup(net, 1, 1)
    x = k.solve(dev(B[0]))
    x[17] = float("nan")
    e = k.backward_error(dev(B[0]), x).cpu().numpy()
    assert np.isnan(e).all()


@pytest.mark.parametrize("which", ["c2", "pvpq_border"])
def test_refinement_reaches_rounding(which):
    if which == "c2":
        net, cfg = G.config_network(2), 2
    else:
        net, cfg = G.make_network(13, 200, 280, 36, 8, pvpq=True, rho=1e5), 13
    k, _, (cp, ri, v), B = setup(net, cfg, 2)
    Bd = dev(B)
    X = k.solve(Bd)
    e0 = k.backward_error(Bd, X).cpu().numpy()
    X0 = X.clone()
    k.refine(Bd, X)
    e1 = k.backward_error(Bd, X).cpu().numpy()
    Xh = X.cpu().numpy()
    for r in range(2):
        om = O.componentwise_backward_error(cp, ri, v, Xh[r], B[r])
        assert om <= 1e-12, (r, om, e0[r], e1[r])
        assert e1[r, 1] <= 1e-12 and e1[r, 1] <= max(e0[r, 1], 1e-15), (e0[r], e1[r])
    print(f"{which}: omega before {e0[:, 1]}, after {e1[:, 1]}")
    # the correction is small: refinement does not move a backward-stable x far
    rel = (X - X0).abs().max().item() / X0.abs().max().item()
    assert rel <= 1e-6, rel


def test_solve_guard_after_failed_factor():
    """A primal diagonal made hugely negative: the inertia is wrong, so the
    factors may not be solved with."""
    net = G.config_network(1)
    k0 = KKT(net)
    cp, ri = k0.pattern()
    z, s = G.draw_point(net, 1)
    cpo, rio, v, pos = O.kkt(net, z, s)
    col = np.repeat(np.arange(pos.N), np.diff(cp))
    j = int(np.flatnonzero(pos.is_primal)[5])
    q = np.flatnonzero((ri == j) & (col == j))[0]
    vb = v.copy()
    vb[q] = -1e9
    k = KKT(pattern=(pos.N, np.array(pos.block_off), cp, ri, pos.is_primal.astype(np.uint8))).bind()
    b = dev(G.draw_rhs(pos.N, 1, 1)[0])
    k.set_values(dev(vb))
    k.factor()
    x = k.solve(b)                       # status not read yet: the device refuses
    assert torch.isnan(x).all()
    info = k.info()
    assert info["status"] == -6 and info["solvable"] == 0, info
    assert info["npos"] == pos.is_primal.sum() - 1
    for f in (lambda: k.solve(b), lambda: k.solve_adjoint(b), lambda: k.refine(b, x)):
        with pytest.raises(NclError) as ei:
            f()
        assert ei.value.code == -4
    # a good factorisation clears the state
    k.set_values(dev(v))
    k.factor()
    x = k.solve(b)
    assert k.info()["solvable"] == 1
    F = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
    F.factor(cp, ri, v)
    xo = F.solve(b.cpu().numpy())
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-8 * np.abs(xo).max()


def test_solve_refused_before_factor_and_during():
    net = G.config_network(1)
    z, s = G.draw_point(net, 1)
    k = KKT(net).bind()
    b = dev(G.draw_rhs(k.N, 1, 1)[0])
    with pytest.raises(NclError) as ei:
        k.factor()                           # no values yet
    assert ei.value.code == -4
    k.assemble(dev(z), dev(s), net.rho)
    with pytest.raises(NclError) as ei:
        k.solve(b)
    assert ei.value.code == -4
    k.factor_blocks()                        # half a factorisation: still refused
    with pytest.raises(NclError) as ei:
        k.solve(b)
    assert ei.value.code == -4
    k.factor_border()
    k.solve(b)


def run_perm_case(net, cfg, perm, nrhs=2):
    """Factors compared entry by entry within 1e-8 plus ten times each
    entry's own rounding sensitivity (under a random order L is not a
    well-conditioned function of K: on the 500-bus x 16 network with the
    order below, one ulp of K moves the oracle's own L by 1.3e-8 at
    max|L| 9.3e7); x and the backward error keep their fixed bars."""
    k, (z, s), _, B = setup(net, cfg, nrhs, perm=perm)
    cp, ri, v, pos = O.kkt(net, z, s)
    F = O.Factor(pos.N, cp, ri, np.array(pos.block_off), perm=perm)
    assert F.factor(cp, ri, v, nthreads=8) == 0
    sym = k.symbolic()
    assert np.array_equal(sym["perm"], F.perm)
    lx, d = check_factors(k, F, cp, ri, v, perm=perm)
    # quasi-definite: every pivot carries its column's sign (primal +, dual -)
    assert np.array_equal(d > 0, pos.is_primal[F.perm])
    assert F.factor(cp, ri, v, nthreads=8) == 0
    X = k.solve(dev(B)).cpu().numpy()
    Xo = F.solve(B)
    assert np.abs(X - Xo).max() <= 1e-8 * np.abs(Xo).max()
    assert O.backward_error(cp, ri, v, X, B) <= 1e-12


def test_user_orders_c1_twenty():
    net = G.config_network(1)
    for seed in range(20):
        run_perm_case(net, 1, block_respecting_perm(net, np.random.default_rng(100 + seed)))


def test_user_order_c2_and_pvpq():
    for net, cfg in ((G.config_network(2), 2), (small_pvpq(), 99)):
        run_perm_case(net, cfg, block_respecting_perm(net, np.random.default_rng(3)))
