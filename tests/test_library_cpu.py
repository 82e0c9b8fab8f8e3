"""Host-side tests of libnclkkt (no GPU): the C ABI loads and exports every
declared symbol, the symbolic analysis equals the oracle's bit for bit, the
K pattern equals the oracle assembly's pattern, and bad inputs are
rejected with NCL_ERR_ARG."""
import ctypes
import os
import re

import numpy as np
import pytest

import gridgen as G
import oracle as O
from paper_2510_13333_amd import KKT, NclError, library_path, load

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "ncl_kkt.h")).read()
    names = set(re.findall(r"\b(ncl_[a-z_]+)\s*\(", hdr))
    assert len(names) >= 17
    lib = ctypes.CDLL(library_path())
    for n in sorted(names):
        assert hasattr(lib, n), n


def _compare(k, F):
    s = k.symbolic()
    for key, ref in [("perm", F.perm), ("etree", F.parent), ("colcount", F.colcount), ("lcolptr", F.lp),
                     ("lrowind", F.li), ("super_ptr", F.sup), ("srowptr", F.srp), ("srowind", F.sri)]:
        assert np.array_equal(s[key], ref), key


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_symbolic_bit_exact(cfg):
    net = G.config_network(cfg)
    _compare(KKT(net), O.Factor.from_network(net))


@pytest.mark.parametrize("seed", range(4))
def test_symbolic_bit_exact_random_small(seed):
    g = np.random.default_rng(seed)
    nb = int(g.integers(8, 40))
    ng = int(g.integers(2, max(3, nb // 4)))
    nl = int(nb - 1 + g.integers(2, nb // 2 + 3))
    pvpq = bool(seed % 2)
    net = G.make_network(50 + seed, nb, nl, ng, int(g.integers(1, 5)), pvpq=pvpq, topology="uniform" if seed >= 2 else "geo",
                         agc=seed >= 2)
    _compare(KKT(net), O.Factor.from_network(net))


@pytest.mark.parametrize("relax", [(1, 0, 1), (4, 1, 2), (32, 1, 1)])
def test_symbolic_relax_parameters(relax):
    net = G.make_network(2, 60, 84, 10, 3)
    _compare(KKT(net, relax=relax), O.Factor.from_network(net, relax=relax))


def block_respecting_perm(net, g):
    """A random elimination order that keeps every block's columns inside the
    block, the same local order for blocks that share a pattern (all blocks
    but a complementarity base block), and the border in layout order."""
    from oracle.assemble import Positions
    pos = Positions(net)
    off = pos.block_off
    perm = np.arange(pos.N, dtype=np.int32)
    local = {}
    for b in range(net.nblk):
        n = off[b + 1] - off[b]
        key = (b == 0 and net.pvpq, n)
        if key not in local:
            local[key] = g.permutation(n)
        perm[off[b]:off[b + 1]] = off[b] + local[key]
    return perm


@pytest.mark.parametrize("seed", range(20))
def test_symbolic_user_order_c1(seed):
    net = G.config_network(1)
    p = block_respecting_perm(net, np.random.default_rng(seed))
    k = KKT(net, perm=p)
    F = O.Factor.from_network(net, perm=p)
    _compare(k, F)
    # the postorder relabels the given elimination: the etree of the final
    # order is a topological order, and the fill is that of the given order
    assert (F.parent[F.parent >= 0] > np.flatnonzero(F.parent >= 0)).all()


@pytest.mark.parametrize("which", ["c2", "pvpq"])
def test_symbolic_user_order_blocks(which):
    net = G.config_network(2) if which == "c2" else G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5)
    p = block_respecting_perm(net, np.random.default_rng(7))
    _compare(KKT(net, perm=p), O.Factor.from_network(net, perm=p))


def test_user_order_rejected_unless_block_respecting():
    net = G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5)
    from oracle.assemble import Positions
    pos = Positions(net)
    g = np.random.default_rng(1)
    good = block_respecting_perm(net, g)
    # two columns of different blocks swapped
    bad = good.copy()
    a, b = pos.block_off[1], pos.block_off[2]
    bad[a], bad[b] = bad[b], bad[a]
    # two contingency blocks (one template) in different local orders
    mixed = good.copy()
    s, e = pos.block_off[2], pos.block_off[3]
    mixed[s:e] = s + g.permutation(e - s)
    # the border permuted
    bord = good.copy()
    bord[-2], bord[-1] = bord[-1], bord[-2]
    for p in (bad, mixed, bord):
        with pytest.raises(NclError) as ei:
            KKT(net, perm=p)
        assert ei.value.code == -1
    for p in (bad, bord):
        with pytest.raises(RuntimeError):
            O.Factor.from_network(net, perm=p)


@pytest.mark.slow
def test_symbolic_bit_exact_c5():
    net = G.config_network(5)
    _compare(KKT(net), O.Factor.from_network(net))


SMALL = {
    1: lambda: G.config_network(1),
    3: lambda: G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5),
    7: lambda: G.make_network(99, 9, 12, 3, 2, pvpq=True, rho=1e5, agc=True),
    8: lambda: G.make_network(99, 9, 12, 3, 2, pvpq=False, rho=1e5, agc=True),
}


@pytest.mark.parametrize("cfg", list(SMALL))
def test_pattern_matches_oracle(cfg):
    net = SMALL[cfg]()
    k = KKT(net)
    z, s = G.draw_point(net, cfg)
    cp, ri, _, pos = O.kkt(net, z, s)
    kcp, kri = k.pattern()
    assert k.N == pos.N and k.nnzK == cp[-1]
    assert np.array_equal(kcp, cp) and np.array_equal(kri, ri)
    assert k.nprimal == int(pos.is_primal.sum())


def test_analyze_pattern_seam_matches_network_analysis():
    net = G.make_network(2, 30, 41, 6, 3)
    k1 = KKT(net)
    cp, ri = k1.pattern()
    z, s = G.draw_point(net, 2)
    _, _, _, pos = O.kkt(net, z, s)
    k2 = KKT(pattern=(k1.N, np.array(pos.block_off), cp, ri, pos.is_primal.astype(np.uint8)))
    a, b = k1.symbolic(), k2.symbolic()
    for key in a:
        assert np.array_equal(a[key], b[key]), key


def test_bad_inputs_rejected():
    net = G.config_network(1)
    bad = G.make_network(1, 30, 41, 6, 0)
    bad.br_to = bad.br_to.copy()
    bad.br_to[0] = 999
    with pytest.raises(NclError) as e:
        KKT(bad)
    assert e.value.code == -1
    dup = G.make_network(1, 30, 41, 6, 0)
    dup.gen_bus = dup.gen_bus.copy()
    dup.gen_bus[1] = dup.gen_bus[0]
    with pytest.raises(NclError):
        KKT(dup)
    two = G.make_network(2, 30, 41, 6, 2)
    two.outage = np.array([3, 3], np.int32)
    with pytest.raises(NclError):
        KKT(two)
    # calls out of order: no workspace bound
    k = KKT(net)
    L = load()
    assert L.ncl_kkt_factor(k._h, None) == -4
    assert L.ncl_kkt_solve(k._h, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, k.N, None) == -4
    assert L.ncl_kkt_workspace_bytes(k._h, 0, ctypes.byref(ctypes.c_size_t())) == -1
    assert L.ncl_status_string(-6) == b"pivot of the wrong sign (inertia)"


def test_pattern_seam_rejects_block_coupling():
    N = 6
    # blocks [0,2), [2,4), border [4,6); entry (2,1) couples two blocks
    cols = {0: [0, 1], 1: [1, 2], 2: [2, 3], 3: [3], 4: [4, 5], 5: [5]}
    cp = np.zeros(N + 1, np.int64)
    ri = []
    for c in range(N):
        ri += cols[c]
        cp[c + 1] = len(ri)
    with pytest.raises(NclError):
        KKT(pattern=(N, np.array([0, 2, 4]), cp, np.array(ri, np.int32), np.ones(N, np.uint8)))


def test_batch_symbolic_is_per_instance_symbolic():
    """A batched handle's symbolic result is the concatenation of each
    network's own analysis (global indices offset by the instance's first
    column), also with per-instance amalgamation parameters."""
    nets = [G.make_network(41, 30, 41, 6, 0, instance=0), G.make_network(41, 60, 84, 11, 5, instance=1),
            G.make_network(41, 24, 33, 4, 3, pvpq=True, instance=2),
            G.make_network(41, 36, 50, 7, 4, pvpq=True, instance=5, agc=True)]
    relax = [(8, 1, 4), (16, 1, 2), (4, 1, 4), (16, 1, 4)]
    kb = KKT(nets=nets, relax=relax)
    sb = kb.symbolic()
    cpb, rib = kb.pattern()
    assert [i["N"] for i in kb.instances] == [KKT(n).N for n in nets]
    nz = sp = 0
    for i, (n, r) in enumerate(zip(nets, relax)):
        k1 = KKT(n, relax=r)
        s1 = k1.symbolic()
        c0, N1 = kb.instances[i]["col0"], kb.instances[i]["N"]
        sl = slice(c0, c0 + N1)
        assert np.array_equal(sb["perm"][sl], s1["perm"] + c0)
        e1 = np.where(s1["etree"] >= 0, s1["etree"] + c0, -1)
        assert np.array_equal(sb["etree"][sl], e1)
        assert np.array_equal(sb["colcount"][sl], s1["colcount"])
        lo, hi = sb["lcolptr"][c0], sb["lcolptr"][c0 + N1]
        assert np.array_equal(sb["lcolptr"][c0:c0 + N1 + 1] - lo, s1["lcolptr"])
        assert np.array_equal(sb["lrowind"][lo:hi], s1["lrowind"] + c0)
        ns = k1.nsuper
        assert np.array_equal(sb["super_ptr"][sp:sp + ns], s1["super_ptr"][:ns] + c0)
        sp += ns
        cp1, ri1 = k1.pattern()
        assert np.array_equal(cpb[c0:c0 + N1 + 1] - cpb[c0], cp1)
        assert np.array_equal(rib[cpb[c0]:cpb[c0 + N1]], ri1 + c0)
        nz += k1.nnzL
    assert nz == kb.nnzL and sp == kb.nsuper


def test_kernel_model_counts():
    """Per-kernel launches per step follow the schedule: one launch per
    non-empty level list, one for every once-per-step kernel."""
    from paper_2510_13333_amd.ncl import KERNELS
    k = KKT(G.config_network(2))
    m = {n: k.kernel_model(i) for i, n in enumerate(KERNELS)}
    assert m["values"] == (0, 0)
    for n in ("assemble", "border_schur", "border_sum", "status", "sol_load", "sol_bpart",
              "sol_border", "sol_store"):
        assert m[n][0] == 1 and m[n][1] > 0, n
    # the dense border factor: the register launch, plus one launch per
    # 32-column block for borders over 216 rows
    nbd = k.instances[0]["nbd"]
    assert m["border_factor"][0] == 1 + ((nbd + 31) // 32 if nbd > 216 else 0) and m["border_factor"][1] > 0
    for n in ("fac_gather", "fac_rows", "sol_fwd_gather", "sol_bwd"):
        assert m[n][0] >= 5
    # the backward pass: one launch per level, plus one border step
    assert m["sol_bwd"][0] == m["fac_diag"][0] and m["sol_bwd_border"][0] == 1
    # assembly reads z and sigma and writes every K value
    assert m["assemble"][1] == 8 * (2 * k.N + k.nnzK)


def test_profile_stride_arguments():
    """The profiling stride is checked on the host (no GPU needed)."""
    k = KKT(G.config_network(1))
    k.profile_stride(3)
    with pytest.raises(NclError):
        k.profile_stride(0)


@pytest.mark.parametrize("pvpq,agc", [(False, False), (True, False), (True, True)])
def test_screening_symbolic_matches_oracle(pvpq, agc):
    """Screening networks (NCL_SCREEN): no border, the contingency blocks
    alone; pattern and symbolic analysis bit-exact with the oracle's."""
    net = G.make_network(43, 60, 84, 9, 6, pvpq=pvpq, rho=1e5, screen=True, agc=agc)
    z, s = G.draw_point(net, 43)
    cp, ri, v, pos = O.kkt(net, z, s)
    k = KKT(net)
    assert k.N == pos.N and k.instances[0]["nbd"] == 0 and k.instances[0]["nblk"] == 6
    cpl, ril = k.pattern()
    assert np.array_equal(cpl, cp) and np.array_equal(ril, ri)
    F = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
    sym = k.symbolic()
    assert np.array_equal(sym["perm"], F.perm) and np.array_equal(sym["etree"], F.parent)
    assert np.array_equal(sym["lcolptr"], F.lp) and np.array_equal(sym["lrowind"], F.li)
    assert np.array_equal(sym["super_ptr"], F.sup)


@pytest.mark.parametrize("pvpq,agc", [(False, False), (True, False), (True, True), (False, True)])
def test_layout_kinds_match_the_layout(pvpq, agc):
    """The kind codes the IPM kernels read (NCL_L_*) name every column as the
    documented layout does: balance and flow rows, the complementarity
    variables and rows, the border pg and vm0, the AGC variables and rows."""
    net = G.make_network(99, 9, 12, 3, 2, pvpq=pvpq, rho=1e5, agc=agc)
    k = KKT(net)
    kinds = k.layout_kinds()
    gk, _, _, _ = G.layout(net)
    code = {G.VM: 1, G.VA: 2, G.QG: 3, G.PG: 4, G.ROW_P: 5, G.ROW_Q: 6, G.ROW_FF: 7, G.ROW_FT: 7,
            G.NUP: 8, G.NUM: 9, G.SUP: 10, G.SLO: 11, G.ROW_LIN: 12, G.ROW_DUP: 13, G.ROW_DLO: 14,
            G.ROW_CUP: 15, G.ROW_CLO: 16, G.VM0: 17, G.PGK: 18, G.PIP: 19, G.PIM: 20, G.SPU: 21, G.SPL: 22,
            G.DELTA: 23, G.ROW_ALIN: 24, G.ROW_ADUP: 25, G.ROW_ADLO: 26, G.ROW_ACUP: 27, G.ROW_ACLO: 28}
    assert np.array_equal(kinds, np.array([code[int(x)] for x in gk], np.uint8))


def test_agc_network_checks():
    """NCL_AGC needs contingencies and finite participation factors."""
    bad = G.make_network(99, 9, 12, 3, 2, pvpq=False, rho=1e5, agc=True)
    bad.gen_alpha = bad.gen_alpha.copy()
    bad.gen_alpha[1] = np.nan
    with pytest.raises(NclError):
        KKT(bad)
    single = G.make_network(1, 30, 41, 6, 0)
    single.agc = True
    single.gen_alpha = np.full(6, 1.0 / 6)
    with pytest.raises(NclError):
        KKT(single)


@pytest.mark.parametrize("pvpq", [False, True])
def test_agc_degenerate_sizes_match_oracle(pvpq):
    """AGC rows at their smallest: one generator (delta's column has one
    entry) and one contingency; pattern and symbolic bit-exact."""
    for nb, nl, ng, K, seed in ((4, 5, 1, 1, 61), (6, 8, 1, 2, 62), (5, 7, 2, 1, 63)):
        net = G.make_network(seed, nb, nl, ng, K, pvpq=pvpq, rho=1e5, agc=True)
        z, s = G.draw_point(net, seed)
        cp, ri, _, pos = O.kkt(net, z, s)
        k = KKT(net)
        kcp, kri = k.pattern()
        assert k.N == pos.N and np.array_equal(kcp, cp) and np.array_equal(kri, ri), (nb, ng, K)
        _compare(k, O.Factor.from_network(net))
