"""The fractional form (Ex. 2-3: u_t = -(-Delta)^{alpha/2} u + f(u) + s in 1-D,
generalized Jacobi reconstruction of parameter (alpha/2, alpha/2), the
alpha-stable walk) on the GPU against the FP64 oracle on identical Philox
words: per-sample path values and iterates for several alpha, node counts,
degrees and ragged sample counts; solves over several intervals (sequential,
geometric mesh with sweeps, Aitken relaxation); the exact fixed point of the
discrete space; FP32 within the Monte Carlo noise; the full-size long-time
workload on sampled paths; the calls the fractional form does not take."""
import numpy as np
import pytest

import oracle as O
from paper_2608_22190_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _hp():
    from paper_2608_22190_amd import hpsmc
    return hpsmc


def _say(*a):
    print("[case]", *a, flush=True)


def _close(a, b, tol=TOL):
    return np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("alpha,n,deg,M,waves", [(0.4, 9, 4, 97, 4), (1.0, 5, 2, 130, 2), (1.6, 7, 3, 64, 4),
                                                 (0.4, 16, 6, 33, 1), (0.1, 6, 3, 64, 2), (1.9, 6, 3, 80, 4)])
def test_frac_iteration_matches_oracle_fp64(alpha, n, deg, M, waves):
    H = _hp()
    wl = W.small(dim=1, n=n, M_deg=deg, M=M, T=0.5, f="u_minus_u3", src="frac_longtime", alpha=alpha)
    _say("frac iteration", alpha, n, deg, M, waves)
    U = np.random.default_rng(n).standard_normal((1, n, deg + 1)) * 0.4
    with H.Plan(wl) as plan:
        plan.hpsmc_set_launch(1, waves, 4, 32)
        plan.hpsmc_set_probe(min(M, 6))
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 2)
        Ug = plan.hpsmc_get_nodes(0)[0]
        pr = plan.hpsmc_get_probe(0)[0]
        st = plan.hpsmc_stats()
        x, _ = plan.hpsmc_grid(0)
    pb = O.Problem(wl)
    xo, _ = pb.grid(0)
    assert np.max(np.abs(x - xo)) < 1e-14
    Uo, _, steps = pb.iterate(U[0].reshape(-1), iter_tag=2)
    assert _close(Ug, Uo.reshape(n, deg + 1))
    assert st["path_steps"] == steps
    Ut = O.frac_reconstruct(alpha, n, deg, U[0].reshape(-1))
    for node in np.random.default_rng(1).choice(pr.shape[0], size=5, replace=False):
        for smp in range(pr.shape[1]):
            S, _ = pb.sample_path(Ut, 0, 0, 2, int(node), smp)
            assert abs(pr[node, smp] - S) <= TOL * (1 + abs(S))


@pytest.mark.parametrize("alpha,n,deg,M", [(0.5, 7, 3, 97), (1.4, 9, 4, 64)])
def test_frac_picard_matches_oracle_fp64(alpha, n, deg, M):
    """The Picard form with the alpha-stable walk: integrand f(u*) + s, the
    initial data at the end point of paths that stay inside for all N* steps,
    the estimate replacing the iterate; short rounds carry paths over."""
    H = _hp()
    wl = W.small(dim=1, n=n, M_deg=deg, M=M, T=0.5, f="u_minus_u3", src="frac_longtime", alpha=alpha,
                 estimator="picard")
    _say("frac picard", alpha, n, deg, M)
    U = np.random.default_rng(n + 3).standard_normal((1, n, deg + 1)) * 0.4
    with H.Plan(wl) as plan:
        plan.hpsmc_set_launch(1, 4, 4, 16)
        plan.hpsmc_set_probe(min(M, 6))
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 1)
        Ug = plan.hpsmc_get_nodes(0)[0]
        pr = plan.hpsmc_get_probe(0)[0]
        st = plan.hpsmc_stats()
    pb = O.Problem(wl)
    Uo, _, steps = pb.iterate(U[0].reshape(-1), iter_tag=1)
    assert _close(Ug, Uo.reshape(n, deg + 1))
    assert np.array_equal(Ug[:, 0], U[0][:, 0])
    assert st["path_steps"] == steps
    Ut = O.frac_reconstruct(alpha, n, deg, U[0].reshape(-1))
    for node in np.random.default_rng(2).choice(pr.shape[0], size=5, replace=False):
        for smp in range(pr.shape[1]):
            S, _ = pb.sample_path(Ut, 0, 0, 1, int(node), smp)
            assert abs(pr[node, smp] - S) <= TOL * (1 + abs(S))
    # two intervals: the terminal data come from the first interval's last column
    wl2 = W.small(dim=1, n=6, M_deg=[3, 3], M=48, iters=2, T=0.8, n_intervals=2, f="u_minus_u3",
                  src="frac_longtime", alpha=alpha, estimator="picard")
    with H.Plan(wl2) as plan:
        plan.hpsmc_solve()
        got = [plan.hpsmc_get_nodes(iv)[0] for iv in range(2)]
    Uo2, _ = O.Problem(wl2).solve()
    for iv in range(2):
        assert _close(got[iv], Uo2[iv]), iv


def test_frac_solves_match_oracle_fp64():
    H = _hp()
    cases = [W.small(dim=1, n=7, M_deg=[3, 4], M=80, iters=3, T=1.0, n_intervals=2, f="u_minus_u3",
                     src="frac_longtime", alpha=0.7),
             W.frac_singular(M=40, iters=2, N=4, n=6, alpha=0.4, rho=0.51).with_(schedule="sweeps", iters=4),
             W.small(dim=1, n=6, M_deg=3, M=64, iters=4, T=0.5, f="u_minus_u3", src="frac_longtime", alpha=1.2,
                     accel="aitken")]
    for wl in cases:
        _say("frac solve", wl.name, wl.schedule, wl.accel)
        with H.Plan(wl) as plan:
            plan.hpsmc_solve()
            got = [plan.hpsmc_get_nodes(iv)[0] for iv in range(wl.n_intervals)]
        Uo, _ = O.Problem(wl).solve()
        for iv in range(wl.n_intervals):
            assert _close(got[iv], Uo[iv]), (wl.name, iv)


@pytest.mark.parametrize("alpha,prec", [(0.4, "fp64"), (1.3, "fp64"), (0.8, "fp32")])
def test_frac_exact_fixed_point(alpha, prec):
    H = _hp()
    wl = W.small(dim=1, n=5, M_deg=2, M=128, T=0.5, f="u_minus_u3", src="frac_poly", alpha=alpha, precision=prec,
                 src_param=[0.5, -0.3, 0.2, 0.7, 0, 0, 0, 0])
    _say("frac fixed point", alpha, prec)
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    U = np.array([[[pb.exact([xj], tl) for tl in t] for xj in x]])
    with H.Plan(wl) as plan:
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 0)
        eps, _ = plan.hpsmc_get_increment(0)
        st = plan.hpsmc_stats()
    assert st["path_steps"] > 0
    assert np.max(np.abs(eps)) < (1e-12 if prec == "fp64" else 2e-5)


def test_frac_fp32_within_monte_carlo_noise():
    H = _hp()
    wl = W.small(dim=1, n=9, M_deg=4, M=2048, iters=3, T=0.5, f="u_minus_u3", src="frac_longtime", alpha=0.6)
    _say("frac fp32")
    res = {}
    for prec in ("fp64", "fp32"):
        with H.Plan(wl.with_(precision=prec)) as plan:
            plan.hpsmc_solve()
            res[prec] = plan.hpsmc_get_nodes(0)[0]
            eps, ssq = plan.hpsmc_get_increment(0)
    sig = np.sqrt(np.maximum(ssq[0] / wl.M - eps[0] ** 2, 0) / wl.M).max()
    d = np.max(np.abs(res["fp32"] - res["fp64"]))
    print(f"|u32-u64|={d:.3e} sigma={sig:.3e}")
    assert d <= 3 * sig + 1e-5


def test_frac_full_size_long_time_sampled_paths():
    """Ex. 2's workload at full size (11 nodes x 6 node times per interval, M =
    8192, the launch the autotuner picks): every node's increment is the mean of
    its per-sample values; sampled paths against the oracle's walk."""
    H = _hp()
    wl = W.frac_long_time(iters=1, n_intervals=1)
    _say("frac full size")
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    U0 = np.array([[[pb.exact([xj], tl) for tl in t] for xj in x]])
    with H.Plan(wl) as plan:
        plan.hpsmc_tune(0, 256, None)
        plan.hpsmc_set_probe(wl.M)
        plan.hpsmc_set_nodes(0, U0)
        plan.hpsmc_iterate(0, 0)
        probe = plan.hpsmc_get_probe(0)[0]
        eps, _ = plan.hpsmc_get_increment(0)
    assert probe.shape == (wl.n * wl.degree[0], wl.M) and np.all(np.isfinite(probe))
    assert np.max(np.abs(eps[0] - probe.mean(axis=1))) <= 1e-13 * (1 + np.max(np.abs(probe)))
    Ut = O.frac_reconstruct(wl.alpha, wl.n, wl.degree[0], U0[0].reshape(-1))
    rng = np.random.default_rng(7)
    for _ in range(12):
        node, smp = int(rng.integers(probe.shape[0])), int(rng.integers(wl.M))
        S, _ = pb.sample_path(Ut, 0, 0, 0, node, smp)
        assert abs(probe[node, smp] - S) <= TOL * (1 + abs(S)), (node, smp)


def test_frac_rejects_what_it_does_not_take():
    H = _hp()
    wl = W.small(dim=1, n=5, M_deg=2, M=16, f="u_minus_u3", src="frac_longtime", alpha=0.5)
    with H.Plan(wl) as plan:
        for call in (lambda: plan.hpsmc_get_coeffs(0), lambda: plan.hpsmc_eval(0, 0, np.zeros((1, 2)))):
            with pytest.raises(H.HpsmcError) as ei:
                call()
            assert ei.value.status == -2
