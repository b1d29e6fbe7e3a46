"""Pins of the oracle's ball-point path quadrature (the Green's-function
representation of a walk step's path integral used in the error analysis,
Sec. 3): the step adds Delta * r(Y_q, tau_q) with Y_q drawn in the ball
B_J(X_q) from Q_r = G_r / W.

- W: the integral of the paper's Green's functions over the ball of radius
  r = sqrt(2 d Delta) equals Delta (scipy quadrature in radial coordinates), so
  Delta is the right weight, d = 1..5;
- the law of the offsets: radial moments against the same quadrature of
  s^{d-1} G(s), isotropy (zero mean, covariance E s^2 / d times I);
- brute force in 1-D: the exact expectation of the estimator (a DP over the
  lattice walk with Gauss-Legendre quadrature over the triangular offset
  density) against the Monte Carlo mean, rejecting the centre-point rule;
- special case: a manufactured solution inside the discrete space is still an
  exact fixed point (the residual vanishes everywhere, also off the nodes).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
from paper_2608_22190_amd import workloads as W


def _green(d, rho, r=1.0):
    """Green's function of -Laplace on the ball of radius r, pole at its centre,
    as a function of the distance rho (the paper's formulas; d = 1 read with
    the sign that makes it positive)"""
    if d == 1:
        return (r - rho) * r / (2 * r)
    if d == 2:
        return math.log(r / rho) / (2 * math.pi)
    return special.gamma(d / 2 - 1) / (4 * math.pi ** (d / 2)) * (rho ** (2 - d) - r ** (2 - d))


def _sphere(d):
    return 2.0 if d == 1 else 2 * math.pi ** (d / 2) / special.gamma(d / 2)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_green_weight_is_delta(d):
    for delta in (1e-3, 0.37):
        r = math.sqrt(2 * d * delta)
        W_, _ = integrate.quad(lambda rho: _sphere(d) * rho ** (d - 1) * _green(d, rho, r), 0, r, limit=200)
        assert abs(W_ - delta) <= 1e-7 * delta   # quadrature of the log singularity


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_ball_offsets_follow_the_green_density(d):
    wl = W.small(dim=d, n=2, M_deg=2, M=8, quad="ball")
    pb = O.Problem(wl)
    off = np.array([pb.ball_offset(node, smp, q) for node in range(2) for smp in range(100) for q in range(40)])
    n = off.shape[0]
    s = np.linalg.norm(off, axis=1)
    assert np.all(s < 1.0)
    norm, _ = integrate.quad(lambda t: t ** (d - 1) * _green(d, t), 0, 1, limit=200)
    for k in (1, 2, 3):
        mk, _ = integrate.quad(lambda t: t ** (k + d - 1) * _green(d, t), 0, 1, limit=200)
        mk /= norm
        se = math.sqrt(np.var(s ** k) / n)
        assert abs(np.mean(s ** k) - mk) < 4 * se, (k, np.mean(s ** k), mk, se)
    # isotropy
    m2 = np.mean(s ** 2)
    cov = off.T @ off / n
    se_m = math.sqrt(m2 / d / n)
    assert np.all(np.abs(off.mean(axis=0)) < 4.5 * se_m)
    assert np.all(np.abs(np.diag(cov) - m2 / d) < 4.5 * math.sqrt(2.0 / n) * m2 / d + 1e-12)
    # the distribution is not the uniform one of the ball or the sphere (power of the test)
    uni = d / (d + 1.0)
    assert abs(np.mean(s) - uni) > 6 * math.sqrt(np.var(s) / n)


def _dp_ball(pb, Ut, x0, t_ell, t0, nstar, quad="ball"):
    """exact expectation of the 1-D estimator: lattice DP for the walk, and for
    each inside step Delta * E[r(X_q + J y)] with y ~ (1 - |y|) on (-1, 1)"""
    span = t_ell - t0
    delta = span / nstar
    J = math.sqrt(2 * delta)
    gx, gw = np.polynomial.legendre.leggauss(30)
    ys = np.concatenate([(gx - 1) / 2, (gx + 1) / 2])          # nodes on [-1, 0] and [0, 1]
    ws = np.concatenate([gw / 2, gw / 2]) * (1 - np.abs(ys))
    p = {0: 1.0}
    total = 0.0
    for q in range(nstar):
        tau = t0 + span - q * delta
        nxt = {}
        for k, pr in p.items():
            xq = x0 + J * k
            if quad == "ball":
                r = sum(w * pb.residual(0, Ut, [xq + J * y], tau) for y, w in zip(ys, ws))
            else:
                r = pb.residual(0, Ut, [xq], tau)
            for sg in (-1, 1):
                if abs(xq + J * sg) >= 1.0:
                    continue
                total += 0.5 * pr * delta * r
                nxt[k + sg] = nxt.get(k + sg, 0.0) + 0.5 * pr
        p = nxt
    return total


def test_ball_estimator_matches_bruteforce_expectation():
    nstar = 4   # long steps: the centre rule's expectation differs by many standard errors
    wl = W.small(dim=1, n=6, M_deg=3, M=40000, T=0.6, nstar=nstar, f="u_minus_u3", src="sin_decay", quad="ball")
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    U = np.random.default_rng(2).standard_normal((pb.nsp, 4)) * 0.5
    Ut = O.reconstruct(1, wl.n, 3, U.reshape(-1))
    rejected = 0
    for jf, ell in [(0, 3), (2, 2), (3, 1), (5, 3)]:
        node = jf + pb.nsp * (ell - 1)
        eps, ssq, _ = pb.estimate(U, nodes=[node])
        se = math.sqrt(max(ssq[0] / wl.M - eps[0] ** 2, 0.0) / wl.M)
        ref = _dp_ball(pb, Ut, x[jf], t[ell], 0.0, nstar)
        assert abs(eps[0] - ref) < 4 * se + 1e-14, (jf, ell, eps[0], ref, se)
        alt = _dp_ball(pb, Ut, x[jf], t[ell], 0.0, nstar, quad="centre")
        if abs(alt - ref) > 12 * se:
            rejected += 1
            assert abs(eps[0] - alt) > 6 * se
    assert rejected >= 2


@pytest.mark.parametrize("dim,f", [(1, "u_minus_u3"), (2, "sin"), (3, "neg_u3")])
def test_exact_fixed_point_with_ball_quadrature(dim, f):
    wl = W.small(dim=dim, n=3, M_deg=2, M=32, T=0.5, src="quad", f=f, nstar=60, quad="ball",
                 src_param=[0.8, -0.4, 0.3, 0, 0, 0, 0, 0])
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    U = np.zeros((pb.nsp, len(t)))
    for jf in range(pb.nsp):
        X = [x[i] for i in np.unravel_index(jf, (wl.n,) * dim)]
        for l in range(len(t)):
            U[jf, l] = pb.exact(X, t[l])
    eps, _, steps = pb.estimate(U)
    assert steps.sum() > 0
    assert np.max(np.abs(eps)) < 1e-12
