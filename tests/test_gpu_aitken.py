"""The Aitken-relaxed iteration (the acceleration remark after Algorithm 1) on
the GPU against the FP64 oracle on identical Philox words: whole solves
(sequential intervals and sweeps, residual and Picard forms, several
instances, each with its own weight), the history carried across single
iterations, its restart after new nodal values, tuning between iterations,
graph replay, and the gradient's ENOTSUP."""
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


def _close(a, b):
    return np.max(np.abs(a - b)) <= TOL * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("schedule,estimator", [("sequential", "residual"), ("sweeps", "residual"),
                                                ("sequential", "picard")])
def test_aitken_solve_matches_oracle(schedule, estimator):
    H = _hp()
    ni = 3
    c0 = np.random.default_rng(11).standard_normal((ni, 16)) * 0.2
    wl = W.small(dim=2, n=4, M_deg=[3, 2], M=72, iters=5, T=0.6, n_intervals=2, f="sin", src="longtime",
                 ic="phi", ic_data=c0, n_instances=ni, schedule=schedule, estimator=estimator,
                 accel="aitken", omega=[0.9, 0.3, 3.0])
    _say("aitken solve", schedule, estimator)
    with H.Plan(wl) as plan:
        plan.hpsmc_solve()
        got = [plan.hpsmc_get_nodes(iv) for iv in range(2)]
    for inst in range(ni):
        Uo, _ = O.Problem(wl).solve(inst=inst)
        for iv in range(2):
            assert _close(got[iv][inst], Uo[iv]), (inst, iv)


def test_aitken_history_across_iterations_restart_and_tuning(tmp_path):
    H = _hp()
    wl = W.small(dim=1, n=7, M_deg=4, M=130, T=0.5, f="u_minus_u3", src="sin_decay", accel="aitken",
                 omega=[1.0, 0.2, 4.0])
    _say("aitken iterations")
    pb = O.Problem(wl)
    U0 = np.random.default_rng(5).standard_normal((wl.nsp, 5)) * 0.3
    with H.Plan(wl) as plan:
        plan.hpsmc_set_nodes(0, U0[None])
        Uo, rp, st = U0.reshape(-1).copy(), np.zeros(wl.nsp * 4), np.zeros(2)
        for k in range(4):
            if k == 2:      # trials of the tuner run plain iterations and restore the iterate
                plan.hpsmc_tune(0, 32, None)
            plan.hpsmc_iterate(0, k)
            Uo, _, _ = pb.iterate_aitken(Uo, rp, st, iter_tag=k)
            assert _close(plan.hpsmc_get_nodes(0)[0], Uo.reshape(wl.nsp, 5)), k
        # new nodal values restart the history: the next weight is omega[0] again
        plan.hpsmc_set_nodes(0, U0[None])
        plan.hpsmc_iterate(0, 7)
        Uo, rp, st = U0.reshape(-1).copy(), np.zeros(wl.nsp * 4), np.zeros(2)
        Uo, _, _ = pb.iterate_aitken(Uo, rp, st, iter_tag=7)
        assert _close(plan.hpsmc_get_nodes(0)[0], Uo.reshape(wl.nsp, 5))
        # start_interval restarts it too
        plan.hpsmc_start_interval(0)
        plan.hpsmc_iterate(0, 0)
        plan.hpsmc_iterate(0, 1)
        Ug = plan.hpsmc_get_nodes(0)[0]
    Up, _ = O.Problem(wl.with_(iters=2)).solve()
    assert _close(Ug, Up[0])


def test_aitken_graph_replays_equal_eager_solve():
    H = _hp()
    wl = W.small(dim=2, n=5, M_deg=3, M=64, iters=4, T=0.5, f="sin", src="longtime", accel="aitken",
                 fresh_per_iter=False)
    _say("aitken graph")
    with H.Plan(wl) as plan:
        plan.hpsmc_solve()
        ref = plan.hpsmc_get_nodes(0)
    with H.Plan(wl) as plan:
        plan.hpsmc_set_option("graph", 1)
        for rep in range(3):
            plan.hpsmc_solve()
            assert np.array_equal(plan.hpsmc_get_nodes(0), ref), rep
            plan.hpsmc_stats()            # eager work between replays


def test_aitken_fp32_within_monte_carlo_noise():
    H = _hp()
    wl = W.small(dim=2, n=5, M_deg=3, M=512, iters=4, T=0.5, f="sin", src="longtime", accel="aitken")
    _say("aitken fp32")
    res = {}
    for prec in ("fp64", "fp32"):
        with H.Plan(wl.with_(precision=prec)) as plan:
            plan.hpsmc_solve()
            res[prec] = plan.hpsmc_get_nodes(0)[0]
            _, ssq = plan.hpsmc_get_increment(0)
            eps, _ = plan.hpsmc_get_increment(0)
    sig = np.sqrt(np.maximum(ssq[0] / wl.M - eps[0] ** 2, 0) / wl.M).max()
    d = np.max(np.abs(res["fp32"] - res["fp64"]))
    print(f"|u32-u64|={d:.3e} sigma={sig:.3e}")
    assert d <= 3 * sig + 1e-5


def test_aitken_has_no_gradient():
    H = _hp()
    wl = W.small(dim=2, n=3, M_deg=2, M=16, ic="phi", ic_data=np.zeros((1, 9)), src="longtime", f="sin",
                 accel="aitken")
    with H.Plan(wl) as plan:
        with pytest.raises(H.HpsmcError) as ei:
            plan.hpsmc_loss_grad_c0(np.zeros((1, 9)))
        assert ei.value.status == -2
