"""The windowed 1-D round kernel against the general round kernel and the oracle.

On a line the windowed kernel replaces the general vector-unit kernel for the
residual form with the centre-point rule: it copies the slabs of 32 walk steps
into LDS per barrier and forms the basis values inside the two dot products,
in the Chebyshev basis (its rows converted from the Legendre tensors).  Its
walk and residual are the general kernel's, so the evaluation counts are
identical and the path values agree to rounding.  The cases cover FP64 and
FP32, one, two and four paths per lane, one-, two- and four-wave blocks, every
mode tier (P <= 12, 20, 36), rounds shorter than a window and windows cut by
the round end, and paths that outlive several rounds.
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


def _run(wl, win, launch, U, m_probe, tag=1):
    H = _hp()
    with H.Plan(wl) as plan:
        plan.hpsmc_set_option("sample_1d", win)
        plan.hpsmc_set_launch(*launch)
        assert plan.hpsmc_get_option("sample_1d_active") == win
        plan.hpsmc_set_probe(m_probe)
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, tag)
        return plan.hpsmc_get_probe(0)[0], plan.hpsmc_get_increment(0)[0], plan.hpsmc_stats()


CASES = [  # n (P = n + 2), precision, launch (samples/lane, waves/block, blocks/CU, round steps), nstar, M
    (3, "fp64", (1, 4, 2, 256), 60, 70),
    (10, "fp64", (2, 4, 4, 40), 300, 33),
    (16, "fp64", (2, 2, 8, 64), 900, 40),
    (16, "fp64", (4, 1, 4, 24), 500, 65),
    (30, "fp64", (1, 4, 2, 100), 400, 20),
    (10, "fp32", (1, 4, 4, 256), 300, 64),
    (16, "fp32", (2, 4, 8, 48), 900, 40),
    (30, "fp32", (4, 2, 2, 32), 400, 24),
]


@pytest.mark.parametrize("n,prec,launch,nstar,M", CASES)
def test_windowed_1d_kernel_matches_the_general_kernel(n, prec, launch, nstar, M):
    wl = W.small(dim=1, n=n, M_deg=3, M=M, T=0.5, precision=prec, nstar=nstar)
    _say("1d window vs general", n, prec, launch, nstar, M)
    U = np.random.default_rng(n).standard_normal((1, wl.nsp, 4)) * 0.5
    mp = min(M, 6)
    pg, eg, sg = _run(wl, 0, launch, U, mp)
    pw, ew, sw = _run(wl, 1, launch, U, mp)
    assert sw["path_steps"] == sg["path_steps"]
    assert sw["node_samples"] == sg["node_samples"] == wl.nsp * 3 * M
    scale = 1.0 + np.max(np.abs(pg))
    tol = 1e-13 if prec == "fp64" else 1e-5
    d = np.max(np.abs(pw - pg))
    print(f"max|S_window - S_general| = {d:.3e} (scale {scale:.3e}), path steps {sw['path_steps']}")
    assert d <= tol * scale
    assert np.max(np.abs(ew - eg)) <= tol * scale


def test_windowed_1d_kernel_walks_the_oracle_paths():
    """FP64 sample paths against the oracle's walks at 1e-12 relative."""
    wl = W.small(dim=1, n=12, M_deg=2, M=48, T=0.5, precision="fp64", nstar=700)
    _say("1d window vs oracle")
    U = np.random.default_rng(5).standard_normal((1, wl.nsp, 3)) * 0.5
    pw, _, _ = _run(wl, 1, (2, 4, 4, 96), U, 4)
    pb = O.Problem(wl)
    Ut = O.reconstruct(1, 12, 2, U[0].reshape(-1))
    rng = np.random.default_rng(3)
    for node in rng.choice(pw.shape[0], size=6, replace=False):
        for smp in range(4):
            S, _ = pb.sample_path(Ut, 0, 0, 1, int(node), smp)
            assert abs(pw[node, smp] - S) <= 1e-12 * (1.0 + abs(S)), (node, smp, pw[node, smp], S)


def test_windowed_1d_kernel_eligibility():
    H = _hp()
    _say("1d window eligibility")
    wl = W.small(dim=1, n=4, M_deg=1, M=8, precision="fp64", nstar=8)
    with H.Plan(wl) as plan:
        for ns in (1, 2, 4):
            plan.hpsmc_set_launch(ns, 4, 2)
            assert plan.hpsmc_get_option("sample_1d_active") == 1
        plan.hpsmc_set_option("sample_1d", 0)
        assert plan.hpsmc_get_option("sample_1d_active") == 0
    for other in (wl.with_(quad="ball"), wl.with_(estimator="picard"),
                  W.small(dim=2, n=4, M_deg=1, M=8, precision="fp64", nstar=8)):
        with H.Plan(other) as plan:
            plan.hpsmc_set_launch(1, 4, 2)
            assert plan.hpsmc_get_option("sample_1d_active") == 0
