"""Pins for the oracle's numeric LDL^T and solve.

* a textbook dense pivot-free LDL^T (numpy) of the permuted matrix gives the
  same L and D (pivots to rounding relative to (|L||D||L|^T)_jj);
* numpy.linalg.solve and SciPy SuperLU (partial pivoting, an unrelated
  method) give the same solution;
* inertia equals the signs of the eigenvalues, and d_j > 0 exactly for the
  primal columns (quasi-definite Schur complements stay quasi-definite);
* any symmetric permutation of a quasi-definite K has an LDL^T without
  pivoting (dense check over random permutations);
* with no dual rows (m = 0) the factorisation is a Cholesky factorisation:
  d_j = l_jj^2 of numpy.linalg.cholesky;
* the border Schur complement equals K_bb - sum_k K_bk K_kk^{-1} K_kb
  computed densely (block-arrowhead structure, Section II-B);
* the reconstruction ||P K P^T - L D L^T|| is at rounding level.
"""
import numpy as np
import pytest

import gridgen as G
import oracle as O


def dense_ldlt(M):
    n = M.shape[0]
    L = np.eye(n)
    d = np.zeros(n)
    W = M.copy()
    for j in range(n):
        d[j] = W[j, j]
        L[j + 1:, j] = W[j + 1:, j] / d[j]
        W[j + 1:, j + 1:] -= np.outer(L[j + 1:, j], L[j + 1:, j]) * d[j]
    return L, d


def setup(net, cfg, it=0):
    z, sig = G.draw_point(net, cfg, iteration=it)
    cp, ri, v, pos = O.kkt(net, z, sig)
    f = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
    rc = f.factor(cp, ri, v)
    assert rc == 0
    from oracle.assemble import to_dense
    import scipy.sparse as sp
    Lw = sp.csc_matrix((v, ri, cp), shape=(pos.N, pos.N)).toarray()
    K = Lw + Lw.T - np.diag(np.diag(Lw))
    return f, K, pos, (cp, ri, v)


def small_nets():
    return [("c1", G.config_network(1), 1),
            ("c2small", G.make_network(2, 30, 41, 6, 4, rho=1e4), 2),
            ("pvpq", G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5), 3),
            ("agc", G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True), 7)]


@pytest.mark.parametrize("name,net,cfg", small_nets())
def test_dense_ldlt_equal(name, net, cfg):
    f, K, pos, _ = setup(net, cfg)
    PK = K[np.ix_(f.perm, f.perm)]
    L, d = dense_ldlt(PK)
    # two rounding orders of one elimination: each pivot agrees to rounding
    # relative to the terms summed into it, (|L| |D| |L|^T)_jj
    scale_d = np.einsum("ij,j,ij->i", np.abs(L), np.abs(d), np.abs(L))
    assert (np.abs(f.d - d) <= 1e-10 * scale_d).all()
    Ls = f.L_csc().toarray() + np.eye(pos.N)
    scale = np.abs(L).max()
    assert np.abs(Ls - L).max() <= 1e-9 * scale
    # the dense factor has no entries outside the symbolic pattern
    assert np.abs(L[(Ls == 0) & ~np.eye(pos.N, dtype=bool)]).max(initial=0) <= 1e-9 * scale


@pytest.mark.parametrize("name,net,cfg", small_nets())
def test_solve_and_inertia(name, net, cfg):
    f, K, pos, (cp, ri, v) = setup(net, cfg)
    B = G.draw_rhs(pos.N, 4, cfg)
    X = f.solve(B)
    Xr = np.linalg.solve(K, B.T).T
    assert np.abs(X - Xr).max() <= 1e-8 * np.abs(Xr).max()
    assert O.backward_error(cp, ri, v, X, B) <= 1e-14
    ev = np.linalg.eigvalsh(K)
    assert f.inertia == (int((ev > 0).sum()), int((ev < 0).sum()), 0)
    prim_new = pos.is_primal[f.perm]
    assert ((f.d > 0) == prim_new).all()


def test_random_permutations_exist():
    """Quasi-definite: 100 random symmetric permutations all factor without
    pivoting, with d_j > 0 exactly on primal columns."""
    net = G.config_network(1)
    f, K, pos, _ = setup(net, 1)
    g = np.random.default_rng(5)
    for _ in range(100):
        p = g.permutation(pos.N)
        L, d = dense_ldlt(K[np.ix_(p, p)])
        assert np.isfinite(d).all()
        assert ((d > 0) == pos.is_primal[p]).all()


def test_m0_is_cholesky():
    """The primal block alone (m = 0) is SPD: LDL^T = Cholesky."""
    net = G.config_network(1)
    z, sig = G.draw_point(net, 1)
    from oracle.assemble import assemble
    r, c, v, pos = assemble(net, z, sig)
    keep = pos.is_primal[r] & pos.is_primal[c]
    n = int(pos.is_primal.sum())
    assert pos.is_primal[:n].all()
    cp, ri, vals = O.lower_csc(r[keep], c[keep], v[keep], n)
    f = O.Factor(n, cp, ri, np.array([0, n]))
    assert f.factor(cp, ri, vals) == 0
    import scipy.sparse as sp
    Lw = sp.csc_matrix((vals, ri, cp), shape=(n, n)).toarray()
    A11 = Lw + Lw.T - np.diag(np.diag(Lw))
    C = np.linalg.cholesky(A11[np.ix_(f.perm, f.perm)])
    np.testing.assert_allclose(f.d, np.diag(C) ** 2, rtol=1e-10)


def test_border_schur_complement():
    net = G.make_network(2, 30, 41, 6, 4, rho=1e4)
    f, K, pos, _ = setup(net, 2)
    bs = pos.block_off[-1]
    S = K[bs:, bs:].copy()
    for k in range(pos.nblk):
        a, b = pos.block_off[k], pos.block_off[k + 1]
        S -= K[bs:, a:b] @ np.linalg.solve(K[a:b, a:b], K[a:b, bs:])
    # border columns come last in the oracle order, in layout order
    Ls = f.L_csc().toarray() + np.eye(pos.N)
    Lbb = Ls[bs:, bs:]
    Db = f.d[bs:]
    np.testing.assert_allclose(Lbb @ np.diag(Db) @ Lbb.T, S, rtol=1e-9, atol=1e-9 * np.abs(S).max())


def test_c2_superlu_and_reconstruction():
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    net = G.config_network(2)
    z, sig = G.draw_point(net, 2)
    cp, ri, v, pos = O.kkt(net, z, sig)
    f = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
    assert f.factor(cp, ri, v, nthreads=4) == 0
    Lw = sp.csc_matrix((v, ri, cp), shape=(pos.N, pos.N))
    K = (Lw + Lw.T - sp.diags(Lw.diagonal())).tocsc()
    b = G.draw_rhs(pos.N, 1, 2)[0]
    x = f.solve(b)
    xs = sla.spsolve(K, b)
    assert np.abs(x - xs).max() <= 1e-8 * np.abs(xs).max()
    assert O.backward_error(cp, ri, v, x, b) <= 1e-15
    assert f.inertia == (int(pos.is_primal.sum()), int((~pos.is_primal).sum()), 0)
    # reconstruction, relative to | |L| |D| |L^T| |
    P = sp.csc_matrix((np.ones(pos.N), (np.arange(pos.N), f.perm)), shape=(pos.N, pos.N))
    PKP = P @ K @ P.T
    Lu = f.L_csc() + sp.eye(pos.N)
    R = PKP - Lu @ sp.diags(f.d) @ Lu.T
    absLDL = abs(Lu) @ sp.diags(np.abs(f.d)) @ abs(Lu).T
    assert abs(R).max() <= 64 * np.finfo(float).eps * abs(absLDL).max()
