"""Parity at the largest supported sizes of every dimension (n = 32 with
degree 31 for d = 1, n = 32 for d = 2 and 3 -- 34 Legendre modes, the largest
register tier and LDS-chunked slabs --, n = 18 for d = 4, n = 10 for d = 5):
one FP64 iteration on the GPU; per-sample path values of sampled nodes against
the oracle's own walks (the oracle cannot redo every node at these sizes), and
for every node the increment equals the mean of its per-sample values."""
import numpy as np
import pytest

import oracle as O
from paper_2608_22190_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("dim,n,deg,M,nstar", [(1, 32, 31, 40, 12), (2, 32, 2, 24, 6), (3, 32, 1, 8, 4),
                                               (4, 18, 1, 8, 3), (5, 10, 1, 8, 3)])
def test_maximum_sizes_fp64(dim, n, deg, M, nstar):
    from paper_2608_22190_amd import hpsmc as H
    wl = W.small(dim=dim, n=n, M_deg=deg, M=M, T=0.5, f="sin", src="longtime", nstar=nstar)
    _say("max size", dim, n, deg, M)
    U = np.random.default_rng(dim).standard_normal((1, wl.nsp, deg + 1)) * 0.3
    with H.Plan(wl) as plan:
        plan.hpsmc_set_probe(M)
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 0)
        probe = plan.hpsmc_get_probe(0)[0]
        eps, _ = plan.hpsmc_get_increment(0)
        st = plan.hpsmc_stats()
    nodes = wl.nsp * deg
    assert probe.shape == (nodes, M) and np.all(np.isfinite(probe))
    assert np.max(np.abs(eps[0] - probe.mean(axis=1))) <= 1e-13 * (1 + np.max(np.abs(probe)))
    assert st["path_steps"] > 0
    pb = O.Problem(wl)
    Ut = O.reconstruct(dim, n, deg, U[0].reshape(-1))
    rng = np.random.default_rng(5)
    for node in rng.choice(nodes, size=3, replace=False):
        for smp in (0, M - 1):
            S, _ = pb.sample_path(Ut, 0, 0, 0, int(node), smp)
            assert abs(probe[node, smp] - S) <= TOL * (1 + abs(S)), (node, smp, probe[node, smp], S)
