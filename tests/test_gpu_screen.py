"""GPU parity of the contingency-screening workload (NCL_SCREEN: the
first-stage variables fixed, so the K contingency blocks are independent
KKT systems with no border; eq. (screening) and Section V-B) against the
oracle, through the C ABI: assembly, factors (small networks) and solves,
at the bars of the main parity tests."""
import pytest

import gridgen as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests.test_gpu_parity import run_case  # noqa: E402


@pytest.mark.parametrize("pvpq", [False, True])
def test_screening_small(pvpq):
    net = G.make_network(43, 60, 84, 9, 6, pvpq=pvpq, rho=1e5, screen=True)
    k, _ = run_case(net, 43, nrhs=2)
    assert k.instances[0]["nbd"] == 0


def test_screening_500bus_256_contingencies():
    net = G.config_network(6)
    k, _ = run_case(net, 6, nrhs=2, factors=False)
    assert k.instances[0]["nblk"] == 256 and k.instances[0]["nbd"] == 0
