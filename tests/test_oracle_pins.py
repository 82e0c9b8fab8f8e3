"""Pins of the oracle's smaller pieces against values fixed by hand or by
an independent derivation (CPU).

* Normwise and componentwise backward errors on a 2x2 system whose
  residual, norms and ratios are worked out below by hand.
* The fraction-to-boundary step on hand-built steps where one known bound
  binds (value tau * gap / |dz|).
* The diagonal shift delta_i = max(0, sum_{j != i} |H_ij| - H_ii) (the
  reading that makes H + delta + Sigma positive definite at non-optimal
  states, Section IV-B block A), checked for equality against the Hessian
  of the independent hyper-dual evaluation, and on the complementarity
  variables against its closed form |nu0| (the V0 term of block A is the
  only Hessian entry of those rows).

Each pin fails under a plausible slip: a dropped ||b||, tau on the wrong
side, off-diagonals counted twice or delta doubled.
"""
import numpy as np
import pytest

import gridgen as G
import oracle as O
from oracle import assemble as A
from oracle import dispatch as D
from tests.test_oracle_assembly import hd_jacobian_hessian, small_pvpq


def two_by_two():
    # K = [[4, 1], [1, -2]] as its lower CSC
    cp = np.array([0, 2, 3], np.int64)
    ri = np.array([0, 1, 1], np.int32)
    v = np.array([4.0, 1.0, -2.0])
    return cp, ri, v


def test_backward_errors_two_by_two():
    cp, ri, v = two_by_two()
    x = np.array([1.0, 2.0])
    b = np.array([7.0, -1.0])
    # Kx = [6, -3], r = b - Kx = [1, 2]; ||r|| = 2, ||K||_inf = 5, ||x|| = 2, ||b|| = 7
    assert O.backward_error(cp, ri, v, x, b) == pytest.approx(2.0 / 17.0, rel=1e-15)
    # |K||x| + |b| = [4 + 2 + 7, 1 + 4 + 1] = [13, 6]; max(1/13, 2/6) = 1/3
    assert O.componentwise_backward_error(cp, ri, v, x, b) == pytest.approx(1.0 / 3.0, rel=1e-15)
    # several columns: the max over them
    X = np.stack([x, np.array([1.0, 0.0])])
    B = np.stack([b, np.array([4.0, 1.0])])        # second column exact: errors 0
    assert O.backward_error(cp, ri, v, X, B) == pytest.approx(2.0 / 17.0, rel=1e-15)
    assert O.componentwise_backward_error(cp, ri, v, X, B) == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert O.componentwise_backward_error(cp, ri, v, X[1], B[1]) == 0.0


def test_componentwise_sees_a_small_row():
    """A wrong component in a row of small scale: the normwise error stays
    tiny, the componentwise one does not."""
    cp = np.array([0, 1, 2], np.int64)
    ri = np.array([0, 1], np.int32)
    v = np.array([1e8, 1e-8])
    x = np.array([1.0, 1.0 + 1e-6])
    b = np.array([1e8, 1e-8])
    # r = [0, -1e-14]; normwise: 1e-14 / (1e8 * (1 + 1e-6) + 1e8) ~ 5e-23
    assert O.backward_error(cp, ri, v, x, b) < 1e-22
    # componentwise row 1: 1e-14 / (1e-8 (1 + 1e-6) + 1e-8) ~ 5e-7
    assert O.componentwise_backward_error(cp, ri, v, x, b) == pytest.approx(1e-14 / (2e-8 + 1e-14), rel=1e-9)


def test_max_step_hand_values():
    net = G.make_network(11, 4, 5, 1, 0, rho=1e3)
    p = D.NLP()
    pos = A.Positions(net)
    z = D.initial_point(net, None, p)      # vm = 1, pg = pmax/2 = 4, flow multipliers mu/smax2
    dz = np.zeros_like(z)
    tau = 0.995
    # vm of bus 0 moves down by 0.5 from 1.0 (gap 0.1 to vmin): tau * 0.1 / 0.5
    dz[pos.vm[0][0]] = -0.5
    # qg moves down by 10 from 0 (gap 3): tau * 0.3, not binding
    dz[pos.qg[0][0]] = -10.0
    # pg moves up by 1 from 4 (gap 4): not binding
    dz[pos.pg[0]] = 1.0
    # a flow multiplier falls by its own value: tau, not binding
    dz[pos.rowFf[0][0]] = -z[pos.rowFf[0][0]]
    assert D.max_step(net, z, dz, p, tau) == pytest.approx(tau * 0.1 / 0.5, rel=1e-14)
    # with the voltage step smaller, the reactive bound binds
    dz[pos.vm[0][0]] = -0.1
    assert D.max_step(net, z, dz, p, tau) == pytest.approx(tau * 3.0 / 10.0, rel=1e-14)
    # an upper bound binding: vm up by 0.5 (gap 0.1 to vmax)
    dz[:] = 0.0
    dz[pos.vm[0][1]] = 0.5
    assert D.max_step(net, z, dz, p, tau) == pytest.approx(tau * 0.1 / 0.5, rel=1e-14)
    # nothing binding: the full step
    dz[:] = 0.0
    dz[pos.va[0]] = 5.0                    # angles carry no bound
    assert D.max_step(net, z, dz, p, tau) == 1.0


def max_step_case():
    """The network, state and steps of the hand-value test (for the GPU
    library's own check) with their expected step lengths."""
    net = G.make_network(11, 4, 5, 1, 0, rho=1e3)
    p = D.NLP()
    pos = A.Positions(net)
    z = D.initial_point(net, None, p)
    tau = 0.995
    cases = []
    dz = np.zeros_like(z)
    dz[pos.vm[0][0]] = -0.5
    dz[pos.qg[0][0]] = -10.0
    dz[pos.pg[0]] = 1.0
    dz[pos.rowFf[0][0]] = -z[pos.rowFf[0][0]]
    cases.append((dz.copy(), tau * 0.1 / 0.5))
    dz[pos.vm[0][0]] = -0.1
    cases.append((dz.copy(), tau * 3.0 / 10.0))
    return net, p, z, tau, cases


@pytest.mark.parametrize("which", ["single", "pvpq"])
def test_delta_shift_exact(which):
    net = G.config_network(1) if which == "single" else small_pvpq()
    z, _ = G.draw_point(net, 1 if which == "single" else 99)
    delta = A.delta_shift(net, z, np.zeros_like(z))
    _, H, prim = hd_jacobian_hessian(net, z)
    Hp = H[np.ix_(prim, prim)]
    off = np.abs(Hp).sum(axis=1) - np.abs(np.diag(Hp))
    want = np.maximum(0.0, off - np.diag(Hp))
    scale = np.abs(Hp).sum(axis=1) + 1.0
    assert np.all(np.abs(delta[prim] - want) <= 1e-13 * scale)
    # dual rows carry no shift
    dual = np.setdiff1d(np.arange(z.shape[0]), prim)
    assert np.all(delta[dual] == 0.0)
    assert np.count_nonzero(want) > 0
    if which == "pvpq":
        pos = A.Positions(net)
        for k in range(1, net.nblk):
            nup, num, sup, slo = pos.comp[k]
            lin, dup, dlo, cup, clo = pos.rowC[k]
            # each complementarity variable's only Hessian entry is nu0 (block A)
            np.testing.assert_array_equal(delta[num], np.abs(z[cup]))
            np.testing.assert_array_equal(delta[sup], np.abs(z[cup]))
            np.testing.assert_array_equal(delta[nup], np.abs(z[clo]))
            np.testing.assert_array_equal(delta[slo], np.abs(z[clo]))
            # reactive outputs have no Hessian at all
            assert np.all(delta[pos.qg[k]] == 0.0)
