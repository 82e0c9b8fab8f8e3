"""GPU parity of the differentiable dispatch map against its oracle.

* ncl_kkt_residual (F and Sigma) against the oracle residual at a random
  interior state: every entry within 1e-12 of its scale;
* the exact Newton matrix (assembly without the shift, dual-row Sigma)
  against the oracle's, at the assembly bar of the KKT parity tests;
* ncl_kkt_max_step against the oracle's fraction-to-boundary step;
* the forward Newton solve against the oracle Newton solution, and the
  autograd gradients (one adjoint solve on the stored factors) against the
  oracle dense-KKT gradients and central finite differences (h = 1e-6) of
  the GPU map itself, on a small network and on the 2000-bus x 64
  contingency workload (there the oracle gradient uses the oracle's own
  LDL^T on the oracle-assembled K at the GPU solution, and 32 directions).
"""
import numpy as np
import pytest

import gridgen as G
from oracle import assemble as A
from oracle import dispatch as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2510_13333_amd import KKT  # noqa: E402
from paper_2510_13333_amd.dispatch import DispatchSolver  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def small_net():
    return G.make_network(5, 40, 56, 7, 3, rho=1e4)


def nlp_dict(p, net):
    return dict(qd_ratio=p.qd_ratio, mu=p.mu, rho=net.rho, vmin=p.vmin, vmax=p.vmax, qmax=p.qmax, pmax=p.pmax,
                smax2=p.smax2, eps=p.eps)


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


@pytest.mark.parametrize("which", ["small", "single_block"])
def test_residual_sigma_and_exact_kkt(which):
    net = small_net() if which == "small" else G.make_network(6, 30, 41, 6, 0, rho=1e3)
    p = D.NLP()
    pd = G.draw_loads(net, 5)
    z = interior_point(net, p)
    k = KKT(net).bind()
    F, sig = k.residual(dev(z), dev(pd), nlp_dict(p, net))
    Fo, so = D.residual(net, z, pd, p)
    F, sig = F.cpu().numpy(), sig.cpu().numpy()
    scale = 1.0 + np.abs(Fo) + np.abs(so)
    assert (np.abs(F - Fo) <= 1e-12 * scale).all(), np.abs(F - Fo).max()
    assert (np.abs(sig - so) <= 1e-12 * (1.0 + np.abs(so))).all()
    # exact Newton matrix: no shift, flow rows -(1/rho + mu/y^2)
    k.assemble(dev(z), dev(so), net.rho, shift=False)
    kv = k.get_values().cpu().numpy()
    cp, ri, v, _ = D.kkt_exact(net, z, so, p)
    cpl, ril = k.pattern()
    assert np.array_equal(cpl, cp) and np.array_equal(ril, ri)
    assert (np.abs(kv - v) <= 1e-12 * (1.0 + np.abs(v))).all(), np.abs(kv - v).max()


def test_max_step_matches_oracle():
    net = small_net()
    p = D.NLP()
    pd = G.draw_loads(net, 5)
    z = interior_point(net, p)
    rng = np.random.default_rng(3)
    k = KKT(net).bind()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    for scale in (1e-3, 0.1, 10.0):
        dz = scale * rng.standard_normal(z.size)
        k.max_step(dev(z), dev(dz), dev(pd), nlp_dict(p, net), 0.995, out)
        assert abs(float(out) - D.max_step(net, z, dz, p)) <= 1e-15 * 1.0


def test_small_forward_and_gradients():
    net = small_net()
    p = D.NLP()
    pd = G.draw_loads(net, 5)
    zo, _ = D.newton(net, pd, p)
    go, Jo = D.gradients(net, zo, pd, p, method="dense")
    s = DispatchSolver(net)
    pdt = dev(pd).requires_grad_(True)
    phi, pg = s(pdt)
    zg = s.z_warm.cpu().numpy()
    assert np.abs(zg - zo).max() <= 1e-7 * np.abs(zo).max()
    phi_o, pg_o = D.outputs(net, zo)
    assert abs(float(phi.detach()) - phi_o) <= 1e-9 * abs(phi_o)
    (g,) = torch.autograd.grad(phi, pdt, retain_graph=True)
    g = g.cpu().numpy()
    assert np.abs(g - go).max() <= 1e-7 * np.abs(go).max()
    w = np.random.default_rng(1).standard_normal(net.ng)
    (gw,) = torch.autograd.grad(pg, pdt, grad_outputs=dev(w))
    assert np.abs(gw.cpu().numpy() - Jo.T @ w).max() <= 1e-7 * np.abs(Jo.T @ w).max()
    # central differences of the GPU map itself
    h = 1e-6
    for d in G.draw_directions(net.nb, 4, 5):
        fp = float(s(dev(pd + h * d))[0])
        fm = float(s(dev(pd - h * d))[0])
        assert abs((fp - fm) / (2 * h) - g @ d) <= 1e-5 * abs(g @ d)


def test_c5_gradients_vs_oracle_and_fd():
    """2000-bus x 64 contingencies: forward Newton on the GPU, gradient by
    one adjoint solve, against the oracle gradient at the GPU solution and
    central differences in 32 random load directions."""
    net = G.config_network(5)
    p = D.NLP()
    pd = G.draw_loads(net, 5)
    s = DispatchSolver(net)
    pdt = dev(pd).requires_grad_(True)
    phi, pg = s(pdt)
    print(f"[c5] Newton iterations {s.iterations}, phi {float(phi.detach()):.6f}", flush=True)
    w = np.random.default_rng(2).standard_normal(net.ng)
    (g,) = torch.autograd.grad(phi, pdt, retain_graph=True)
    (gw,) = torch.autograd.grad(pg, pdt, grad_outputs=dev(w))
    g, gw = g.cpu().numpy(), gw.cpu().numpy()
    z = s.z_warm.cpu().numpy()
    F, _ = D.residual(net, z, pd, p)
    go, gwo = D.gradients(net, z, pd, p, method="ldlt", cotangent=w)
    assert np.abs(g - go).max() <= 1e-8 * np.abs(go).max(), np.abs(g - go).max() / np.abs(go).max()
    assert np.abs(gw - gwo).max() <= 1e-8 * np.abs(gwo).max()
    h = 1e-6
    worst = 0.0
    for d in G.draw_directions(net.nb, 32, 5):
        fp = float(s(dev(pd + h * d))[0])
        fm = float(s(dev(pd - h * d))[0])
        rel = abs((fp - fm) / (2 * h) - g @ d) / abs(g @ d)
        worst = max(worst, rel)
    print(f"[c5] worst central-difference relative error {worst:.2e}", flush=True)
    assert worst <= 1e-5


def test_outputs_and_vjp_entry_points():
    """ncl_kkt_dispatch_outputs against the oracle's phi and pg at the
    solution; ncl_kkt_dispatch_vjp against the oracle's pivot-free LDL^T
    gradient for a random (gphi, gpg) cotangent, and linear in it."""
    net = small_net()
    p = D.NLP()
    pd = G.draw_loads(net, 5)
    s = DispatchSolver(net)
    z = s.newton(dev(pd))
    s._pd_of = (dev(pd),)
    phi, pg = s.outputs(z)
    zh = z.cpu().numpy()
    phi_o, pg_o = D.outputs(net, zh)
    assert abs(float(phi) - phi_o) <= 1e-14 * abs(phi_o)
    assert np.array_equal(pg.cpu().numpy(), pg_o)
    w = np.random.default_rng(4).standard_normal(net.ng)
    g1 = s.vjp(z, dev(np.array(1.0)), None).cpu().numpy()
    gw = s.vjp(z, dev(np.array(0.0)), dev(w)).cpu().numpy()
    gb = s.vjp(z, dev(np.array(2.0)), dev(w)).cpu().numpy()
    go, gwo = D.gradients(net, zh, pd, p, method="ldlt", cotangent=w)
    assert np.abs(g1 - go).max() <= 1e-10 * np.abs(go).max()
    assert np.abs(gw - gwo).max() <= 1e-10 * np.abs(gwo).max()
    assert np.abs(gb - (2 * g1 + gw)).max() <= 1e-12 * np.abs(gb).max()
