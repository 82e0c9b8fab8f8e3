"""GPU parity of the batched path: several independent networks analysed into
one handle (every launch covers all of them) against (a) the same networks
factored one handle at a time, bitwise, and (b) the CPU oracle at the bars
of the single-network parity tests.

Bitwise equality holds because a batched handle runs, per network, the same
templates, term order and fixed-order block reductions as a single handle.
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


def mixed_networks(rho=1e4):
    """Uneven small instances: no border, plain border, PV/PQ border, and
    AGC rows with and without PV/PQ rows."""
    return [
        G.make_network(41, 30, 41, 6, 0, rho=rho, instance=0),
        G.make_network(41, 60, 84, 11, 5, rho=rho, instance=1),
        G.make_network(41, 24, 33, 4, 3, pvpq=True, rho=rho, instance=2),
        G.make_network(41, 118, 165, 21, 9, rho=rho, instance=3),
        G.make_network(41, 45, 63, 8, 2, pvpq=True, rho=rho, instance=4),
        G.make_network(41, 36, 50, 7, 4, pvpq=True, rho=rho, instance=5, agc=True),
        G.make_network(41, 50, 70, 9, 3, rho=rho, instance=6, agc=True),
    ]


def points(nets, cfg, iteration=0):
    zs, ss = [], []
    for i, n in enumerate(nets):
        z, s = G.draw_point(n, cfg, instance=i, iteration=iteration)
        zs.append(z)
        ss.append(s)
    return zs, ss


def run_batch_vs_single(nets, cfg, nrhs, oracle_check=True, iteration=0):
    rho = nets[0].rho
    assert all(n.rho == rho for n in nets)
    kb = KKT(nets=nets).bind(nrhs_max=nrhs)
    assert len(kb.instances) == len(nets)
    zs, ss = points(nets, cfg, iteration)
    kb.assemble(dev(np.concatenate(zs)), dev(np.concatenate(ss)), rho)
    kb.factor()
    info = kb.info()
    assert info["status"] == 0, info
    B = G.draw_rhs(kb.N, nrhs, cfg, iteration=iteration)
    Xb = kb.solve(dev(B)).cpu().numpy()
    Xa = kb.solve_adjoint(dev(B)).cpu().numpy()
    assert np.array_equal(Xa, Xb)
    vb = kb.get_values().cpu().numpy()
    npos = nneg = 0
    voff = 0
    for i, net in enumerate(nets):
        I = kb.instances[i]
        c0, n = I["col0"], I["N"]
        k1 = KKT(net).bind(nrhs_max=nrhs)
        assert k1.N == n
        k1.assemble(dev(zs[i]), dev(ss[i]), rho)
        k1.factor()
        i1 = k1.info()
        npos += i1["npos"]
        nneg += i1["nneg"]
        v1 = k1.get_values().cpu().numpy()
        assert np.array_equal(vb[voff:voff + v1.size], v1), f"instance {i}: K values differ"
        voff += v1.size
        X1 = k1.solve(dev(np.ascontiguousarray(B[:, c0:c0 + n]))).cpu().numpy()
        assert np.array_equal(Xb[:, c0:c0 + n], X1), f"instance {i}: batched and single solves differ"
        if oracle_check:
            cp, ri, v, pos = O.kkt(net, zs[i], ss[i])
            F = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
            assert F.factor(cp, ri, v, nthreads=8) == 0
            Xo = F.solve(B[:, c0:c0 + n])
            rel = np.abs(X1 - Xo).max() / np.abs(Xo).max()
            eta = O.backward_error(cp, ri, v, X1, B[:, c0:c0 + n])
            assert rel <= 1e-8, (i, rel)
            assert eta <= 1e-12, (i, eta)
    assert voff == vb.size
    assert info["npos"] == npos and info["nneg"] == nneg
    return kb


def test_batch_mixed_small():
    run_batch_vs_single(mixed_networks(), 41, nrhs=2)


def test_batch_refactor_iterations():
    nets = mixed_networks()
    kb = KKT(nets=nets).bind(nrhs_max=1)
    for it in range(3):
        zs, ss = points(nets, 41, iteration=it)
        kb.assemble(dev(np.concatenate(zs)), dev(np.concatenate(ss)), nets[0].rho)
        kb.factor()
        assert kb.info()["status"] == 0
        B = G.draw_rhs(kb.N, 1, 41, iteration=it)
        X = kb.solve(dev(B)).cpu().numpy()
        for i, net in enumerate(nets):
            I = kb.instances[i]
            c0, n = I["col0"], I["N"]
            cp, ri, v, pos = O.kkt(net, zs[i], ss[i])
            assert O.backward_error(cp, ri, v, X[:, c0:c0 + n], B[:, c0:c0 + n]) <= 1e-12


def test_batch_c4_workload():
    """The 64 uneven instances of the batched workload: batched == one handle
    per instance bitwise; the first 16 instances' backward error <= 1e-12
    against the oracle-assembled K; and every instance whose border exceeds
    216 rows (the blocked border factor and the border solve from global
    memory) solved by the oracle too and compared element by element."""
    nets = G.batched_networks(64)
    kb = run_batch_vs_single(nets, 4, nrhs=1, oracle_check=False)
    zs, ss = points(nets, 4)
    B = G.draw_rhs(kb.N, 1, 4)
    X = kb.solve(dev(B)).cpu().numpy()
    large = [i for i, I in enumerate(kb.instances) if I["nbd"] > 216]
    assert len(large) >= 4
    for i, net in enumerate(nets):
        if i >= 16 and i not in large:
            continue
        I = kb.instances[i]
        c0, n = I["col0"], I["N"]
        cp, ri, v, pos = O.kkt(net, zs[i], ss[i])
        assert O.backward_error(cp, ri, v, X[:, c0:c0 + n], B[:, c0:c0 + n]) <= 1e-12, i
        if i in large:
            F = O.Factor(pos.N, cp, ri, np.array(pos.block_off))
            assert F.factor(cp, ri, v, nthreads=8) == 0
            Xo = F.solve(B[:, c0:c0 + n])
            assert np.abs(X[:, c0:c0 + n] - Xo).max() <= 1e-8 * np.abs(Xo).max(), i


def test_graph_replay_matches_eager():
    """The batched step captured once in a hipGraph: every replay (new state
    copied into the captured inputs, eager work and synchronisation between
    replays) is bitwise equal to the eager step on the same state."""
    nets = mixed_networks()
    rho = nets[0].rho
    kb = KKT(nets=nets).bind(nrhs_max=1)
    states = []
    for it in range(3):
        zs, ss = points(nets, 41, iteration=it)
        states.append((dev(np.concatenate(zs)), dev(np.concatenate(ss)), dev(G.draw_rhs(kb.N, 1, 41, iteration=it)[0])))
    zb, sb, bb = (t.clone() for t in states[0])
    xb = torch.empty_like(bb)
    kb.assemble(zb, sb, rho)                     # warm up outside the capture
    kb.factor()
    kb.solve(bb, out=xb)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        kb.assemble(zb, sb, rho)
        kb.factor()
        kb.solve(bb, out=xb)
    torch.cuda.synchronize()
    for rep in range(2):
        for it, (z, s, b) in enumerate(states):
            zb.copy_(z)
            sb.copy_(s)
            bb.copy_(b)
            g.replay()
            torch.cuda.synchronize()
            xr = xb.clone()
            kb.assemble(z, s, rho)
            kb.factor()
            xe = kb.solve(b)
            torch.cuda.synchronize()
            assert kb.info()["status"] == 0
            assert torch.equal(xr, xe), (rep, it)


def test_profiling_brackets_each_kind():
    """ncl_kkt_profile brackets exactly the launches the per-kernel model
    counts for one step, with non-negative event times."""
    from paper_2510_13333_amd.ncl import KERNELS
    nets = mixed_networks()
    kb = KKT(nets=nets).bind(nrhs_max=1)
    zs, ss = points(nets, 41)
    z, s, b = dev(np.concatenate(zs)), dev(np.concatenate(ss)), dev(G.draw_rhs(kb.N, 1, 41)[0])
    x = torch.empty_like(b)
    for kind, name in enumerate(KERNELS):
        if name == "values":
            continue
        kb.profile(kind)
        kb.assemble(z, s, nets[0].rho)
        kb.factor()
        kb.solve(b, out=x)
        n, ms = kb.profile_read()
        launches, nbytes = kb.kernel_model(kind)
        assert n == launches, (name, n, launches)
        assert ms >= 0.0 and nbytes >= 0
    # a stride brackets every stride-th launch only (levels sampled in turn)
    gather = KERNELS.index("fac_gather")
    kb.profile(gather)
    kb.profile_stride(2)
    kb.assemble(z, s, nets[0].rho)
    kb.factor()
    kb.solve(b, out=x)
    n, ms = kb.profile_read()
    assert n == (kb.kernel_model(gather)[0] + 1) // 2 and ms > 0.0
    kb.profile(-1)
    assert kb.profile_read() == (0, 0.0)
