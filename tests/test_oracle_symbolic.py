"""Pins for the oracle's symbolic analysis, by brute force on small inputs:

* ordering: an O(n^3) dense-boolean minimum-degree elimination written from
  the ordering rule (smallest current degree, ties to the smallest layout
  index, neighbours become a clique, border vertices never eliminated,
  postorder of the elimination forest), block by block;
* elimination tree and fill: dense boolean elimination of the permuted
  pattern, parent(j) = min{i > j : L_ij != 0};
* supernodes: the fundamental and relaxed-amalgamation rules re-evaluated
  from the brute-force fill.
"""
import numpy as np
import pytest

import gridgen as G
import oracle as O
from oracle import assemble as A


def small_pvpq():
    return G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5)


def nets():
    return [("c1", G.config_network(1)), ("pvpq", small_pvpq()),
            ("c2small", G.make_network(2, 30, 41, 6, 4, rho=1e4)),
            ("agc", G.make_network(99, 9, 12, 3, 2, pvpq=False, rho=1e5, agc=True))]


def _pattern(net):
    z = np.ones(A.Positions(net).N)
    r, c, v, pos = A.assemble(net, z, z)
    N = pos.N
    adj = np.zeros((N, N), bool)
    adj[r, c] = True
    adj[c, r] = True
    np.fill_diagonal(adj, False)
    return adj, pos


def brute_order(adj, pos):
    N = pos.N
    bstart = pos.block_off[-1]
    perm = []
    for k in range(pos.nblk):
        a, b = pos.block_off[k], pos.block_off[k + 1]
        loc = list(range(a, b)) + list(range(bstart, N))
        g = adj[np.ix_(loc, loc)].copy()
        nv = b - a
        alive = np.ones(len(loc), bool)
        seq, nbrs = [], {}
        for _ in range(nv):
            deg = np.where(alive[:nv], (g[:nv] & alive).sum(axis=1), 10 ** 9)
            v = int(np.argmin(deg))            # argmin takes the first (smallest index) on ties
            nb = np.flatnonzero(g[v] & alive)
            nbrs[v] = nb
            seq.append(v)
            alive[v] = False
            for x in nb:
                g[x, nb] = True
            g[nb, nb] = False
            g[v, :] = False
            g[:, v] = False
        epos = {v: i for i, v in enumerate(seq)}
        par = {}
        for v in seq:
            bl = [x for x in nbrs[v] if x < nv]
            par[v] = min(bl, key=lambda x: epos[x]) if bl else -1
        children = {v: [] for v in seq}
        for v in seq:                          # increasing position
            if par[v] >= 0:
                children[par[v]].append(v)
        out = []

        def dfs(u):
            for c in children[u]:
                dfs(c)
            out.append(u)

        for v in seq:
            if par[v] < 0:
                dfs(v)
        perm.extend(a + np.array(out, int))
    perm.extend(range(bstart, N))
    return np.array(perm)


def brute_fill(adj, perm):
    N = adj.shape[0]
    P = adj[np.ix_(perm, perm)]
    L = np.tril(P, -1)
    for j in range(N):
        rows = np.flatnonzero(L[:, j])
        if rows.size:
            L[np.ix_(rows, rows)] |= np.tril(np.ones((rows.size, rows.size), bool), -1)
    return L


@pytest.mark.parametrize("name,net", nets())
def test_order_matches_brute_force(name, net):
    adj, pos = _pattern(net)
    f = O.Factor.from_network(net)
    assert np.array_equal(f.perm, brute_order(adj, pos))


@pytest.mark.parametrize("name,net", nets())
def test_etree_fill_colcount(name, net):
    adj, pos = _pattern(net)
    f = O.Factor.from_network(net)
    L = brute_fill(adj, f.perm)
    N = pos.N
    for j in range(N):
        rows = np.flatnonzero(L[:, j])
        assert np.array_equal(f.li[f.lp[j]:f.lp[j + 1]], rows)
        assert f.parent[j] == (rows[0] if rows.size else -1)
        assert f.colcount[j] == rows.size + 1


@pytest.mark.parametrize("name,net", nets())
def test_supernode_rules(name, net):
    adj, pos = _pattern(net)
    f = O.Factor.from_network(net)
    L = brute_fill(adj, f.perm)
    N = pos.N
    region = np.full(N, pos.nblk)
    for k in range(pos.nblk):
        region[pos.block_off[k]:pos.block_off[k + 1]] = k
    parent = np.array([np.flatnonzero(L[:, j])[0] if L[:, j].any() else -1 for j in range(N)])
    cc = L.sum(axis=0) + 1
    nchild = np.bincount(parent[parent >= 0], minlength=N)
    # fundamental partition, by definition (with the 32-column cap)
    fund = [0]
    run = 1
    for j in range(N - 1):
        join = (parent[j] == j + 1 and cc[j] == cc[j + 1] + 1 and nchild[j + 1] == 1
                and region[j] == region[j + 1] and run < 32)
        if join:
            run += 1
        else:
            fund.append(j + 1)
            run = 1
    fund.append(N)
    # relaxed amalgamation, by definition
    sup = []
    cf, cl = fund[0], fund[1] - 1
    for q in range(1, len(fund) - 1):
        pf, pl = fund[q], fund[q + 1] - 1
        ok = parent[cl] == pf and region[cl] == region[pf] and (pl - cf + 1) <= 16
        if ok:
            w = pl - cf + 1
            off = np.flatnonzero(L[pl + 1:, cf:pl + 1].any(axis=1)).size
            entries = w * (w + 1) // 2 + w * off
            zeros = entries - cc[cf:pl + 1].sum()
            ok = 4 * zeros <= entries
        if ok:
            cl = pl
        else:
            sup.append(cf)
            cf, cl = pf, pl
    sup.append(cf)
    sup.append(N)
    assert np.array_equal(f.sup, np.array(sup))
    # panel rows: the supernode's columns then the union of their structures below it
    for s in range(f.nsuper):
        a, b = f.sup[s], f.sup[s + 1]
        rows = list(range(a, b)) + list(b + np.flatnonzero(L[b:, a:b].any(axis=1)))
        assert np.array_equal(f.sri[f.srp[s]:f.srp[s + 1]], np.array(rows))


def test_block_templates_share_order():
    """Contingency blocks have identical graphs, so identical block orders."""
    net = G.make_network(2, 30, 41, 6, 4, rho=1e4)
    f = O.Factor.from_network(net)
    bo = f.pos.block_off
    base = f.perm[bo[1]:bo[2]] - bo[1]
    for k in range(2, net.nblk):
        assert np.array_equal(f.perm[bo[k]:bo[k + 1]] - bo[k], base)
