"""Pins of the dispatch-map oracle (CPU).

* The residual F and the assembled KKT (no shift, with the residual's
  Sigma) are written independently; the complex-step Jacobian of F (exact
  to rounding, h = 1e-30) must equal K entry by entry.  A dropped term or a
  wrong sign in either fails it.
* Newton converges to a point where the exact K has inertia (n, m): a
  strict local minimum of the barrier problem.
* The implicit-function gradients (one solve with K) match central finite
  differences of the converged map (h = 1e-6) in random load directions.
"""
import warnings

import numpy as np
import pytest

import gridgen as G
from oracle import assemble as A
from oracle import dispatch as D


@pytest.fixture(scope="module")
def small():
    net = G.make_network(5, 40, 56, 7, 3, rho=1e4)
    return net, D.NLP(), G.draw_loads(net, 5)


def interior_point(net, p, seed=0):
    pos = A.Positions(net)
    rng = np.random.default_rng(seed)
    z = D.initial_point(net, None, p) + 0.01 * rng.standard_normal(pos.N)
    for k in range(net.nblk):
        z[pos.rowP[k]] = rng.standard_normal(net.nb)
        z[pos.rowQ[k]] = rng.standard_normal(net.nb)
        z[pos.rowFf[k]] = 10 ** rng.uniform(-3, 0, net.nl)
        z[pos.rowFt[k]] = 10 ** rng.uniform(-3, 0, net.nl)
    return z


def test_complex_step_jacobian_is_kkt(small):
    net, p, pd = small
    z = interior_point(net, p)
    F, sig = D.residual(net, z, pd, p)
    cp, ri, v, _ = D.kkt_exact(net, z, sig, p)
    K = D.full_matrix(cp, ri, v).toarray()
    J = np.zeros_like(K)
    h = 1e-30
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for j in range(z.size):
            e = np.zeros(z.size, complex)
            e[j] = 1j * h
            J[:, j] = D.residual(net, z + e, pd, p)[0].imag / h
    scale = np.maximum(np.abs(K), 1.0)
    assert (np.abs(J - K) <= 1e-12 * scale).all(), np.abs(J - K).max()


def test_newton_reaches_strict_local_minimum(small):
    net, p, pd = small
    z, its = D.newton(net, pd, p)
    F, sig = D.residual(net, z, pd, p)
    cp, ri, v, pos = D.kkt_exact(net, z, sig, p)
    w = np.linalg.eigvalsh(D.full_matrix(cp, ri, v).toarray())
    n = int(pos.is_primal.sum())
    assert (w > 0).sum() == n and (w < 0).sum() == pos.N - n
    # the full Newton step at the returned point is at rounding level
    import scipy.sparse.linalg as spl
    dz = spl.spsolve(D.full_matrix(cp, ri, v), -F)
    assert np.all(np.abs(dz) <= 1e-10 * (1 + np.abs(z)))


def test_gradients_match_central_differences(small):
    net, p, pd = small
    z, _ = D.newton(net, pd, p)
    g, Jpg = D.gradients(net, z, pd, p, method="dense")
    g2, _ = D.gradients(net, z, pd, p, method="ldlt")
    np.testing.assert_allclose(g2, g, rtol=1e-8, atol=1e-12)
    h = 1e-6
    for d in G.draw_directions(net.nb, 3, 5):
        zp, _ = D.newton(net, pd + h * d, p, z0=z)
        zm, _ = D.newton(net, pd - h * d, p, z0=z)
        fp, pgp = D.outputs(net, zp)
        fm, pgm = D.outputs(net, zm)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * abs(g @ d), (fd, g @ d)
        fdp = (pgp - pgm) / (2 * h)
        assert np.abs(fdp - Jpg @ d).max() <= 1e-6 * np.abs(Jpg @ d).max()
