"""The ball-point path quadrature (a walk step adds Delta * r at a point drawn
from the normalized Green's function of its ball, the representation of the
error analysis, Sec. 3) on the GPU against the FP64 oracle on identical Philox
words: per-sample path values and iterates for d = 1..5 with every
samples-per-lane setting (LDS-chunked slabs for d >= 3), the Picard form with
the ball rule, solves with several intervals and sweeps, the exact fixed
point, FP32 within the Monte Carlo noise, and ENOTSUP for the gradient."""
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


@pytest.mark.parametrize("dim,n,deg,M,ns,nstar,est", [
    (1, 6, 4, 150, 1, 40, "residual"), (1, 9, 3, 97, 2, None, "picard"), (2, 4, 3, 96, 2, 60, "residual"),
    (2, 5, 2, 65, 4, None, "residual"), (2, 4, 2, 70, 1, 30, "picard"), (3, 3, 2, 70, 1, 30, "residual"),
    (4, 2, 2, 40, 2, 20, "residual"), (5, 2, 2, 33, 1, 12, "picard")])
def test_ball_iteration_matches_oracle_fp64(dim, n, deg, M, ns, nstar, est):
    H = _hp()
    wl = W.small(dim=dim, n=n, M_deg=deg, M=M, T=0.5, f="sin", src="longtime", estimator=est, nstar=nstar,
                 quad="ball")
    _say("ball iteration", dim, n, deg, M, ns, est)
    U = np.random.default_rng(dim + 20).standard_normal((1, wl.nsp, deg + 1)) * 0.4
    with H.Plan(wl) as plan:
        plan.hpsmc_set_launch(ns, 2, 4)
        assert plan.hpsmc_get_option("sample_mfma_active") == 0
        plan.hpsmc_set_probe(min(M, 6))
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 1)
        Ug = plan.hpsmc_get_nodes(0)[0]
        pr = plan.hpsmc_get_probe(0)[0]
        st = plan.hpsmc_stats()
    pb = O.Problem(wl)
    Uo, _, steps = pb.iterate(U[0].reshape(-1), iter_tag=1)
    Uo = Uo.reshape(wl.nsp, deg + 1)
    assert np.max(np.abs(Ug - Uo)) <= TOL * max(1.0, np.max(np.abs(Uo)))
    assert st["path_steps"] == steps
    Ut = O.reconstruct(dim, n, deg, U[0].reshape(-1))
    for node in np.random.default_rng(4).choice(pr.shape[0], size=min(5, pr.shape[0]), replace=False):
        for smp in range(pr.shape[1]):
            S, _ = pb.sample_path(Ut, 0, 0, 1, int(node), smp)
            assert abs(pr[node, smp] - S) <= TOL * (1 + abs(S))


def test_ball_solves_match_oracle_fp64():
    H = _hp()
    _say("ball solves")
    for wl in [W.small(dim=1, n=6, M_deg=[3, 4], M=120, iters=3, T=0.8, n_intervals=2, quad="ball",
                       f="u_minus_u3", src="sin_decay"),
               W.small(dim=2, n=4, M_deg=[2, 3, 2], M=64, iters=3, T=0.6, n_intervals=3, quad="ball",
                       schedule="sweeps", f="sin", src="longtime", accel="aitken")]:
        with H.Plan(wl) as plan:
            plan.hpsmc_solve()
            got = [plan.hpsmc_get_nodes(iv)[0] for iv in range(wl.n_intervals)]
        Uo, _ = O.Problem(wl).solve()
        for iv in range(wl.n_intervals):
            assert np.max(np.abs(got[iv] - Uo[iv])) <= TOL * max(1.0, np.max(np.abs(Uo[iv]))), (wl.schedule, iv)


@pytest.mark.parametrize("dim,f,prec", [(1, "u_minus_u3", "fp64"), (2, "sin", "fp64"), (3, "neg_u3", "fp64"),
                                        (2, "sin", "fp32")])
def test_ball_exact_fixed_point(dim, f, prec):
    H = _hp()
    wl = W.small(dim=dim, n=3, M_deg=2, M=64, T=0.5, src="quad", f=f, nstar=60, quad="ball", precision=prec,
                 src_param=[0.8, -0.4, 0.3, 0, 0, 0, 0, 0])
    _say("ball fixed point", dim, f, prec)
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    U = np.zeros((1, wl.nsp, len(t)))
    for jf in range(wl.nsp):
        X = [x[i] for i in np.unravel_index(jf, (wl.n,) * dim)]
        for l in range(len(t)):
            U[0, jf, l] = pb.exact(X, t[l])
    with H.Plan(wl) as plan:
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 0)
        eps, _ = plan.hpsmc_get_increment(0)
    assert np.max(np.abs(eps)) < (1e-12 if prec == "fp64" else 2e-5)


def test_ball_fp32_within_monte_carlo_noise():
    H = _hp()
    wl = W.small(dim=2, n=5, M_deg=3, M=512, iters=3, T=0.5, f="sin", src="longtime", quad="ball")
    _say("ball fp32")
    res = {}
    for prec in ("fp64", "fp32"):
        with H.Plan(wl.with_(precision=prec)) as plan:
            plan.hpsmc_set_option("sample_mfma", 0)   # the vector-unit kernel (the matrix-core one: test_gpu_mma)
            plan.hpsmc_set_launch(1, 4, 4)
            assert plan.hpsmc_get_option("sample_mfma_active") == 0
            plan.hpsmc_solve()
            res[prec] = plan.hpsmc_get_nodes(0)[0]
            eps, ssq = plan.hpsmc_get_increment(0)
    sig = np.sqrt(np.maximum(ssq[0] / wl.M - eps[0] ** 2, 0) / wl.M).max()
    d = np.max(np.abs(res["fp32"] - res["fp64"]))
    print(f"|u32-u64|={d:.3e} sigma={sig:.3e}")
    assert d <= 3 * sig + 1e-5


def test_ball_has_no_gradient():
    H = _hp()
    wl = W.small(dim=2, n=3, M_deg=2, M=16, ic="phi", ic_data=np.zeros((1, 9)), src="longtime", f="sin",
                 quad="ball")
    with H.Plan(wl) as plan:
        with pytest.raises(H.HpsmcError) as ei:
            plan.hpsmc_loss_grad_c0(np.zeros((1, 9)))
        assert ei.value.status == -2
