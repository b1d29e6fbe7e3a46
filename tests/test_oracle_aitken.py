"""Pins of the oracle's Aitken-relaxed iteration (the acceleration remark after
Algorithm 1: Aitken extrapolation folded into the iteration as a weighted
average u <- u + w r of the iterate and its update).

- closed form: with common random numbers and an affine f the iteration map G
  is affine; on a problem with a single Monte Carlo node it is a scalar map
  u -> a u + b, and Aitken's delta-squared weight w = 1/(1 - a) lands on the
  fixed point after the second iteration exactly (to rounding), for any first
  weight.  The fixed point is obtained independently by running the plain
  iteration to convergence;
- special case: bounds [1, 1] pin the weight to 1 and reproduce the plain
  iteration (Algorithm 1, Step 3; eq. uast's replacement for the Picard form);
- invariant: on a many-node problem the relaxed iteration has the plain
  iteration's fixed point and reaches a tolerance in fewer iterations.
"""
import numpy as np
import pytest

import oracle as O
from paper_2608_22190_amd import workloads as W


def _affine_scalar(estimator="residual", **kw):
    # n = 1: the single spatial node x = 0; one node time (l = 1): one unknown
    return W.small(dim=1, n=1, M_deg=1, M=64, T=0.5, nstar=40, f="affine", f_param=[0.7, 0.2, 0, 0],
                   src="sin_decay", fresh_per_iter=False, estimator=estimator, **kw)


def _plain_fixed_point(pb, U, iters=400):
    for _ in range(iters):
        U, mx, _ = pb.iterate(U)
        if mx < 1e-15:
            break
    return U


@pytest.mark.parametrize("estimator", ["residual", "picard"])
@pytest.mark.parametrize("w0", [1.0, 0.6])
def test_scalar_affine_map_converges_in_two_steps(estimator, w0):
    wl = _affine_scalar(estimator, accel="aitken", omega=[w0, 0.01, 100.0])
    pb = O.Problem(wl)
    U0 = np.array([0.3, -0.4])                      # [column 0 (initial data), column 1]
    Ufix = _plain_fixed_point(pb, U0)
    # the plain map is a contraction but not a one-step solver (the pin has power)
    U1p, _, _ = pb.iterate(U0)
    U2p, _, _ = pb.iterate(U1p)
    a = (U2p[1] - U1p[1]) / (U1p[1] - U0[1])
    assert 0.02 < abs(a) < 0.98, a
    assert abs(U2p[1] - Ufix[1]) > 1e-3 * abs(Ufix[1] - U0[1])
    # Aitken: w0 first, then the secant weight 1/(1 - a)
    rp, st = np.zeros(1), np.zeros(2)
    U1, _, _ = pb.iterate_aitken(U0, rp, st)
    assert st[0] == w0 and st[1] == 1.0
    U2, _, _ = pb.iterate_aitken(U1, rp, st)
    assert abs(st[0] - 1.0 / (1.0 - a)) <= 1e-8 * abs(st[0])
    assert abs(U2[1] - Ufix[1]) <= 1e-12 * (1 + abs(Ufix[1]))
    assert U2[0] == U0[0]
    _, mx, _ = pb.iterate_aitken(U2, rp, st)
    assert mx <= 1e-12 * (1 + abs(Ufix[1]))


@pytest.mark.parametrize("estimator", ["residual", "picard"])
def test_unit_weight_is_the_plain_iteration(estimator):
    wl = W.small(dim=2, n=4, M_deg=3, M=48, T=0.4, f="sin", src="longtime", estimator=estimator,
                 accel="aitken", omega=[1.0, 1.0, 1.0])
    pb = O.Problem(wl)
    rng = np.random.default_rng(7)
    U = rng.standard_normal(pb.nsp * 4) * 0.3
    Ua, rp, st = U.copy(), np.zeros(pb.nsp * 3), np.zeros(2)
    for k in range(3):
        U, mx, s1 = pb.iterate(U, iter_tag=k)
        Ua, mxa, s2 = pb.iterate_aitken(Ua, rp, st, iter_tag=k)
        assert s1 == s2 and st[0] == 1.0
        assert np.max(np.abs(Ua - U)) <= 1e-15 * np.max(np.abs(U))
        assert abs(mx - mxa) <= 1e-15 * mx
    Up, _ = O.Problem(wl.with_(accel="none", iters=3)).solve()
    Uq, _ = O.Problem(wl.with_(iters=3)).solve()
    assert np.max(np.abs(Up[0] - Uq[0])) <= 1e-15 * np.max(np.abs(Up[0]))


@pytest.mark.parametrize("schedule", ["sequential", "sweeps"])
def test_relaxed_iteration_keeps_the_fixed_point_and_needs_fewer_iterations(schedule):
    """Common random numbers make the map deterministic: both iterations head for
    its fixed point; the relaxed one gets within 1e-9 of it sooner."""
    kw = dict(dim=1, n=6, M_deg=[4, 4], M=64, T=0.6, n_intervals=2, f="u_minus_u3", src="sin_decay",
              fresh_per_iter=False, schedule=schedule, nstar=60)
    ref, _ = O.Problem(W.small(iters=200, **kw)).solve()

    def iterations_to(accel, tol=1e-9):
        for k in range(1, 200):
            U, _ = O.Problem(W.small(iters=k, accel=accel, **kw)).solve()
            if max(np.max(np.abs(U[i] - ref[i])) for i in range(2)) < tol:
                return k, U
        return None, U

    kp, Up = iterations_to("none")
    ka, Ua = iterations_to("aitken")
    assert kp is not None and ka is not None and ka < kp, (kp, ka)
    print(f"{schedule}: plain {kp} iterations, Aitken {ka}")
