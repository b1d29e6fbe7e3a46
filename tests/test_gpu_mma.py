"""The matrix-core form of the 2-D FP32 path-advancing kernel.

It walks exactly the paths of the vector-unit kernel (the directions, jumps
and exit tests are the same FP32 operations), so the integer count of
residual evaluations is identical, and only the rounding order of the slab
contraction differs.  Against the FP64 oracle it must be as accurate as the
vector-unit FP32 kernel on every sampled path, pass reading R24's statistical
bar, and hold the exact fixed point.  Mode counts P = n + 2 cover odd and even
P (K split into unequal halves), small P and the largest supported P = 32.
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


@pytest.mark.parametrize("n,deg,M", [(1, 2, 40), (3, 3, 96), (4, 2, 130), (5, 2, 64), (11, 2, 64),
                                     (24, 2, 33), (30, 1, 20)])
def test_mma_kernel_walks_the_vector_kernel_paths(n, deg, M):
    H = _hp()
    wl = W.small(dim=2, n=n, M_deg=deg, M=M, T=0.5, f="sin", src="longtime", precision="fp32")
    _say("mma vs valu", n, deg, M)
    U = np.random.default_rng(n).standard_normal((1, wl.nsp, deg + 1)) * 0.5
    mp = min(M, 8)
    res = {}
    for mma in (1, 0):
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("sample_mfma", mma)
            plan.hpsmc_set_launch(1, 4, 4)
            assert plan.hpsmc_get_option("sample_mfma") == mma
            assert plan.hpsmc_get_option("sample_mfma_active") == mma
            plan.hpsmc_set_probe(mp)
            plan.hpsmc_set_nodes(0, U)
            plan.hpsmc_iterate(0, 2)
            res[mma] = (plan.hpsmc_get_probe(0)[0], plan.hpsmc_get_increment(0)[0], plan.hpsmc_stats())
    (pm, em, sm), (pv, ev, sv) = res[1], res[0]
    assert sm["path_steps"] == sv["path_steps"]
    scale = 1.0 + np.max(np.abs(pv))
    dmv = np.max(np.abs(pm - pv))
    print(f"max|S_mma - S_valu| = {dmv:.3e} (scale {scale:.3e})")
    assert dmv <= 1e-4 * scale
    assert np.max(np.abs(em - ev)) <= 1e-4 * scale
    # sampled paths against the FP64 oracle: no less accurate than the vector-unit kernel
    pb = O.Problem(wl)
    Ut = O.reconstruct(2, n, deg, U[0].reshape(-1))
    rng = np.random.default_rng(7)
    nodes = rng.choice(pm.shape[0], size=min(6, pm.shape[0]), replace=False)
    e_m = e_v = 0.0
    for node in nodes:
        for smp in range(min(mp, 4)):
            S, _ = pb.sample_path(Ut, 0, 0, 2, int(node), smp)
            e_m = max(e_m, abs(pm[node, smp] - S))
            e_v = max(e_v, abs(pv[node, smp] - S))
    print(f"vs oracle: mma {e_m:.3e} valu {e_v:.3e}")
    assert e_m <= 2.0 * e_v + 1e-5 * scale


@pytest.mark.parametrize("estimator,quad,n,deg,M", [("picard", "centre", 3, 3, 96), ("picard", "centre", 24, 2, 33),
                                                     ("residual", "ball", 4, 2, 130), ("residual", "ball", 11, 2, 64),
                                                     ("picard", "ball", 5, 3, 64)])
def test_mma_modes_walk_the_vector_kernel_paths(estimator, quad, n, deg, M):
    """The Picard form (u table only, the initial data at the end point of
    paths that stay inside for all N* steps) and the ball-point rule on the
    matrix cores: the vector-unit kernel's walks, per-sample values within
    FP32 rounding of them and no less accurate against the FP64 oracle."""
    H = _hp()
    wl = W.small(dim=2, n=n, M_deg=deg, M=M, T=0.5, f="sin", src="longtime", precision="fp32",
                 estimator=estimator, quad=quad, nstar=40 if estimator == "picard" else None)
    _say("mma modes", estimator, quad, n, deg, M)
    U = np.random.default_rng(n + 1).standard_normal((1, wl.nsp, deg + 1)) * 0.5
    mp = min(M, 8)
    res = {}
    for mma in (1, 0):
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("sample_mfma", mma)
            plan.hpsmc_set_launch(1, 4, 4, 16)        # several rounds: the state is carried over
            assert plan.hpsmc_get_option("sample_mfma_active") == mma
            plan.hpsmc_set_probe(mp)
            plan.hpsmc_set_nodes(0, U)
            plan.hpsmc_iterate(0, 1)
            res[mma] = (plan.hpsmc_get_probe(0)[0], plan.hpsmc_get_nodes(0)[0], plan.hpsmc_stats())
    (pm, um, sm), (pv, uv, sv) = res[1], res[0]
    assert sm["path_steps"] == sv["path_steps"]
    scale = 1.0 + np.max(np.abs(pv))
    dmv = np.max(np.abs(pm - pv))
    print(f"max|S_mma - S_valu| = {dmv:.3e} (scale {scale:.3e})")
    assert dmv <= 1e-4 * scale
    assert np.max(np.abs(um - uv)) <= 1e-4 * scale
    pb = O.Problem(wl)
    Ut = O.reconstruct(2, n, deg, U[0].reshape(-1))
    rng = np.random.default_rng(9)
    e_m = e_v = 0.0
    for node in rng.choice(pm.shape[0], size=min(6, pm.shape[0]), replace=False):
        for smp in range(min(mp, 4)):
            S, _ = pb.sample_path(Ut, 0, 0, 1, int(node), smp)
            e_m = max(e_m, abs(pm[node, smp] - S))
            e_v = max(e_v, abs(pv[node, smp] - S))
    print(f"vs oracle: mma {e_m:.3e} valu {e_v:.3e}")
    assert e_m <= 2.0 * e_v + 1e-5 * scale


def test_mma_fp32_statistical_parity_r24():
    """Reading R24 with the matrix-core kernel: same Philox words as the FP64
    solve; e32 <= e64 + 3 sigma and |u32 - u64| <= 3 sigma + 1e-5."""
    H = _hp()
    wl = W.small(dim=2, n=5, M_deg=4, M=512, iters=4, T=0.5, f="sin", src="longtime")
    _say("mma r24")
    res = {}
    for prec in ("fp64", "fp32"):
        with H.Plan(wl.with_(precision=prec)) as plan:
            plan.hpsmc_set_launch(1, 4, 4)
            if prec == "fp32":
                assert plan.hpsmc_get_option("sample_mfma_active") == 1
            plan.hpsmc_solve()
            res[prec] = plan.hpsmc_get_nodes(0)[0]
            eps, ssq = plan.hpsmc_get_increment(0)
            if prec == "fp64":
                sig = np.sqrt(np.maximum(ssq[0] / wl.M - eps[0] ** 2, 0) / wl.M).max()
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    ex = np.zeros_like(res["fp64"])
    for jf in range(wl.nsp):
        X = [x[i] for i in np.unravel_index(jf, (wl.n,) * 2)]
        for l in range(len(t)):
            ex[jf, l] = pb.exact(X, t[l])
    Uo, _ = pb.solve()
    assert np.max(np.abs(res["fp64"] - Uo[0])) <= 1e-12 * np.max(np.abs(Uo[0]))
    e64 = np.max(np.abs(res["fp64"] - ex))
    e32 = np.max(np.abs(res["fp32"] - ex))
    d = np.max(np.abs(res["fp32"] - res["fp64"]))
    print(f"e64={e64:.3e} e32={e32:.3e} |u32-u64|={d:.3e} sigma={sig:.3e}")
    assert e32 <= e64 + 3 * sig
    assert d <= 3 * sig + 1e-5


@pytest.mark.parametrize("n", [3, 6])
def test_mma_exact_fixed_point(n):
    """Nodal data of a solution inside the discrete space: every residual
    vanishes, so the increment is zero up to FP32 rounding of the contraction."""
    H = _hp()
    wl = W.small(dim=2, n=n, M_deg=2, M=64, T=0.5, src="quad", f="sin", nstar=80, precision="fp32",
                 src_param=[0.8, -0.4, 0.3, 0, 0, 0, 0, 0])
    _say("mma fixed point", n)
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    U = np.zeros((1, wl.nsp, 3))
    for jf in range(wl.nsp):
        X = [x[i] for i in np.unravel_index(jf, (n,) * 2)]
        for l in range(3):
            U[0, jf, l] = pb.exact(X, t[l])
    with H.Plan(wl) as plan:
        plan.hpsmc_set_launch(1, 2, 6)
        assert plan.hpsmc_get_option("sample_mfma_active") == 1
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 0)
        eps, _ = plan.hpsmc_get_increment(0)
    assert np.max(np.abs(eps)) < 2e-5


def test_mma_option_and_eligibility():
    H = _hp()
    _say("mma option")
    wl = W.small(dim=2, n=4, M_deg=2, M=16, precision="fp32")
    with H.Plan(wl) as plan:
        assert plan.hpsmc_get_option("sample_mfma") == 1
        plan.hpsmc_set_launch(2, 4, 4)           # two samples per lane: vector units
        assert plan.hpsmc_get_option("sample_mfma_active") == 0
        plan.hpsmc_set_launch(1, 4, 4)
        assert plan.hpsmc_get_option("sample_mfma_active") == 1
        plan.hpsmc_set_launch(1, 2, 6)           # two-wave blocks
        assert plan.hpsmc_get_option("sample_mfma_active") == 1
        with pytest.raises(H.HpsmcError):
            plan.hpsmc_set_option("sample_mfma", 2)
        with pytest.raises(H.HpsmcError):
            plan.hpsmc_get_option("no_such_option")
    for other in (wl.with_(precision="fp64"), W.small(dim=1, n=4, M_deg=2, M=16, precision="fp32"),
                  W.small(dim=3, n=3, M_deg=2, M=16, precision="fp32")):
        with H.Plan(other) as plan:
            plan.hpsmc_set_launch(1, 4, 4)
            assert plan.hpsmc_get_option("sample_mfma_active") == 0
