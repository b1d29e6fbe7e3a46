"""The matrix-core form of the 5-D FP32 path-advancing kernel.

Its walk is the vector-unit kernel's (the same shared direction routine,
jump and exit test in FP32), so the integer count of residual evaluations is
identical and only the rounding order of the slab contraction differs: the
innermost two modes as a 32x32x2 matrix-core product over 32-row tiles of
(k0, k1, k2), the rest on the vector unit.  Mode counts P = n + 2 cover every
tiling case of the slab image: all rows in remainder tiles (P = 3, 4, 5), one
or several main tiles per k0 with a remainder (P = 6, 7, 9, 10), none (P = 8)
and the largest supported P = 12; sample counts leave ragged waves; short
rounds carry the path state over; blocks of one, two and four waves.  Rounds
with few live paths (sparse rounds) run each 64-path item on all the waves of
a block, each wave taking a share of every tile's k-steps; every case runs
with that split on and off.
"""
import numpy as np
import pytest

import oracle as O
from paper_2608_22190_amd import workloads as W

pytestmark = pytest.mark.gpu


def _hp():
    from paper_2608_22190_amd import hpsmc
    return hpsmc


def _say(*a):
    print("[case]", *a, flush=True)


def _run(wl, mma, launch, U, m_probe, tag=1, split=1):
    H = _hp()
    with H.Plan(wl) as plan:
        plan.hpsmc_set_option("sample_mfma", mma)
        plan.hpsmc_set_option("sample_split", split)
        assert plan.hpsmc_get_option("sample_split") == split
        plan.hpsmc_set_launch(*launch)
        assert plan.hpsmc_get_option("sample_mfma_active") == (2 if mma else 0)
        plan.hpsmc_set_probe(m_probe)
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, tag)
        return plan.hpsmc_get_probe(0)[0], plan.hpsmc_get_increment(0)[0], plan.hpsmc_stats()


@pytest.mark.parametrize("n,deg,M,launch", [(1, 2, 40, (1, 4, 2, 16)), (2, 2, 70, (1, 4, 2, 16)),
                                            (3, 1, 33, (1, 2, 2, 16)), (4, 1, 64, (1, 4, 2, 32)),
                                            (5, 1, 20, (1, 1, 4, 16)), (6, 1, 9, (1, 4, 2, 16)),
                                            (7, 1, 6, (1, 4, 2, 16)), (8, 1, 4, (1, 4, 2, 16)),
                                            (10, 1, 2, (1, 4, 1, 16))])
def test_mma5_kernel_walks_the_vector_kernel_paths(n, deg, M, launch):
    wl = W.small(dim=5, n=n, M_deg=deg, M=M, T=0.5, f="neg_u3", src="cos_decay", precision="fp32", nstar=40)
    _say("mma5 vs valu", n, deg, M, launch)
    U = np.random.default_rng(n).standard_normal((1, wl.nsp, deg + 1)) * 0.5
    mp = min(M, 4)
    pv, ev, sv = _run(wl, 0, launch, U, mp)
    scale = 1.0 + np.max(np.abs(pv))
    runs = {}
    for split in (1, 0):   # sparse rounds on all the block's waves, or never
        pm, em, sm = runs[split] = _run(wl, 1, launch, U, mp, split=split)
        assert sm["path_steps"] == sv["path_steps"]
        assert sm["node_samples"] == sv["node_samples"] == wl.nsp * deg * M
        dmv = np.max(np.abs(pm - pv))
        print(f"split={split}: max|S_mma - S_valu| = {dmv:.3e} (scale {scale:.3e}), path steps {sm['path_steps']}")
        assert dmv <= 1e-4 * scale
        assert np.max(np.abs(em - ev)) <= 1e-4 * scale
    if launch[1] in (2, 4):
        # these small sets leave sparse rounds: the split rounds sum u and v in another order
        assert not np.array_equal(runs[1][0], runs[0][0])
    else:
        assert np.array_equal(runs[1][0], runs[0][0])
    pm = runs[1][0]
    # sampled paths against the FP64 oracle: no less accurate than the vector-unit kernel
    pb = O.Problem(wl)
    Ut = O.reconstruct(5, n, deg, U[0].reshape(-1))
    rng = np.random.default_rng(7)
    nodes = rng.choice(pm.shape[0], size=min(5, pm.shape[0]), replace=False)
    e_m = e_v = 0.0
    for node in nodes:
        for smp in range(min(mp, 3)):
            S, _ = pb.sample_path(Ut, 0, 0, 1, int(node), smp)
            e_m = max(e_m, abs(pm[node, smp] - S))
            e_v = max(e_v, abs(pv[node, smp] - S))
    print(f"vs oracle: mma {e_m:.3e} valu {e_v:.3e}")
    assert e_m <= 2.0 * e_v + 1e-5 * scale


def test_mma5_several_intervals_and_instances():
    """Group offsets in the tile image: two intervals of different degree in a
    sweep, two instances, every group's slab sequence at its own offset."""
    wl = W.small(dim=5, n=3, M_deg=[2, 3], n_intervals=2, M=24, T=0.4, f="neg_u3", src="cos_decay",
                 precision="fp32", nstar=24, schedule="sweeps", n_instances=2)
    _say("mma5 sweep, two instances")
    H = _hp()
    res = {}
    for mma in (1, 0):
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("sample_mfma", mma)
            plan.hpsmc_set_launch(1, 4, 2, 16)
            assert plan.hpsmc_get_option("sample_mfma_active") == (2 if mma else 0)
            plan.hpsmc_set_probe(4)
            plan.hpsmc_sweep(1)
            res[mma] = ([plan.hpsmc_get_probe(iv) for iv in range(2)], plan.hpsmc_stats())
    (pm, sm), (pv, sv) = res[1], res[0]
    assert sm["path_steps"] == sv["path_steps"]
    for a, b in zip(pm, pv):
        assert a.shape == b.shape and np.max(np.abs(a - b)) <= 1e-4 * (1 + np.max(np.abs(b)))


@pytest.mark.parametrize("n", [2, 4])
def test_mma5_exact_fixed_point(n):
    """Nodal data of a solution inside the discrete space (prod (1 - x_i^2)
    times a quadratic in t): every residual vanishes, so the increment is zero
    up to FP32 rounding of the contraction."""
    H = _hp()
    wl = W.small(dim=5, n=n, M_deg=2, M=64, T=0.5, src="quad", f="neg_u3", nstar=40, precision="fp32",
                 src_param=[0.8, -0.4, 0.3, 0, 0, 0, 0, 0])
    _say("mma5 fixed point", n)
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    U = np.zeros((1, wl.nsp, 3))
    for jf in range(wl.nsp):
        X = [x[i] for i in np.unravel_index(jf, (n,) * 5)]
        for l in range(3):
            U[0, jf, l] = pb.exact(X, t[l])
    with H.Plan(wl) as plan:
        plan.hpsmc_set_launch(1, 4, 2)
        assert plan.hpsmc_get_option("sample_mfma_active") == 2
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 0)
        eps, _ = plan.hpsmc_get_increment(0)
    print(f"max|eps| = {np.max(np.abs(eps)):.3e}")
    assert np.max(np.abs(eps)) < 2e-5


def test_mma5_eligibility():
    H = _hp()
    _say("mma5 eligibility")
    wl = W.small(dim=5, n=2, M_deg=1, M=8, precision="fp32", nstar=8)
    with H.Plan(wl) as plan:
        plan.hpsmc_set_launch(2, 4, 4)           # two samples per lane: vector units
        assert plan.hpsmc_get_option("sample_mfma_active") == 0
        for w in (1, 2, 4):
            plan.hpsmc_set_launch(1, w, 2)
            assert plan.hpsmc_get_option("sample_mfma_active") == 2
        plan.hpsmc_set_option("sample_mfma", 0)
        assert plan.hpsmc_get_option("sample_mfma_active") == 0
    for other in (wl.with_(precision="fp64"), wl.with_(quad="ball"), wl.with_(estimator="picard")):
        with H.Plan(other) as plan:
            plan.hpsmc_set_launch(1, 4, 2)
            assert plan.hpsmc_get_option("sample_mfma_active") == 0
