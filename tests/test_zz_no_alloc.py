"""GPU: ncl_kkt_backward_error_noalloc (library-held staging, no
allocation) against ncl_kkt_backward_error through the C ABI: the same
(eta, omega) bit for bit, on two calls in a row, the second with a smaller
system, at the exact solve and at a perturbed one; and the size limit."""
import numpy as np
import pytest

import gridgen as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2510_13333_amd import KKT, NclError  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def case(net, cfg, nrhs):
    z, s = G.draw_point(net, cfg)
    k = KKT(net).bind(nrhs_max=nrhs)
    k.assemble(dev(z), dev(s), net.rho)
    k.factor()
    B = dev(G.draw_rhs(k.N, nrhs, cfg))
    X = k.solve(B)
    return k, B, X


def test_noalloc_backward_error_equals_workspace_one():
    # 500-bus x 16 first, then the 30-bus single network (smaller)
    for net, cfg, nrhs in ((G.config_network(2), 2, 3), (G.config_network(1), 1, 2)):
        k, B, X = case(net, cfg, nrhs)
        g = np.random.default_rng(cfg)
        Xp = X * (1.0 + 1e-7 * dev(g.standard_normal(tuple(X.shape))))
        for x in (X, Xp):
            ref = k.backward_error(B, x).cpu().numpy()
            na = k.backward_error(B, x, noalloc=True).cpu().numpy()
            assert np.array_equal(ref, na), (ref, na)
            assert np.isfinite(na).all()
        assert (k.backward_error(B, X, noalloc=True).cpu().numpy()[:, 0] <= 1e-12).all()


def test_noalloc_rejects_beyond_limit():
    # 64 networks in one handle (N = 6.5 million): staging over the limit
    k = KKT(nets=G.batched_networks(64))
    assert 4 * k.N > 6 * 1048576
    b = torch.zeros(k.N, dtype=torch.float64, device="cuda")
    with pytest.raises(NclError) as ei:
        k.backward_error(b, b, noalloc=True)
    assert ei.value.code == -1
