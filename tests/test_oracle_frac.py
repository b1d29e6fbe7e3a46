"""Pins of the oracle's fractional form (Ex. 2-3: the operator (-Delta)^{alpha/2},
generalized Jacobi functions of parameter (alpha/2, alpha/2), the alpha-stable
walk), d = 1.

- library routines: Gauss-Jacobi nodes and weights, Jacobi polynomials, the
  regularized incomplete beta function and its inverse (scipy);
- the eigen-relation (-Delta)^{alpha/2}[(1-x^2)_+^{alpha/2} P_p] = lambda_p P_p
  against a direct quadrature of the hypersingular integral (with the constant
  of the operator whose Fourier symbol is |xi|^alpha), and lambda_p at alpha = 2
  against exact calculus, (p+1)(p+2);
- the jump law against the exit-point density of a ball for the symmetric
  stable process started at its centre (integrated numerically), and its limit
  alpha -> 2 (jumps of length sqrt(2 Delta));
- the reconstruction reproduces functions of the discrete space and their time
  derivatives; the manufactured source against the hypersingular integral of
  the exact solution;
- the exact fixed point of the discrete space (eq. varepsilon_1 vanishes) and
  the geometric decrease of the iteration on Ex. 2's problem.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
from paper_2608_22190_amd import workloads as W


def _cfrac(alpha):
    """constant of (-Delta)^{alpha/2} u = C p.v. int (u(x) - u(y)) / |x-y|^{1+alpha} dy, d = 1"""
    return alpha * 2 ** (alpha - 1) * special.gamma((1 + alpha) / 2) / (math.sqrt(math.pi) * special.gamma(1 - alpha / 2))


def _frac_lap(u, x, alpha):
    """(-Delta)^{alpha/2} u at x for u supported in [-1, 1], by quadrature of
    C int_0^inf (2u(x) - u(x+z) - u(x-z)) z^{-1-alpha} dz"""
    z1, z2 = 1 - abs(x), 1 + abs(x)
    g = lambda z: (2 * u(x) - u(x + z) - u(x - z)) * z ** (-1 - alpha)
    s1, _ = integrate.quad(g, 0, z1, limit=400)
    s2, _ = integrate.quad(g, z1, z2, limit=400)
    tail = 2 * u(x) * z2 ** (-alpha) / alpha
    return _cfrac(alpha) * (s1 + s2 + tail)


@pytest.mark.parametrize("a", [0.2, 0.65, 0.95])
def test_gauss_jacobi_and_jacobi_polynomials(a):
    for n in (1, 5, 11, 24):
        x, w = O.gauss_jacobi(n, a)
        xs, ws = special.roots_jacobi(n, a, a)
        assert np.max(np.abs(x - xs)) < 1e-14 and np.max(np.abs(w - ws)) < 1e-13 * np.max(ws)
    for p in range(8):
        for xx in (-0.93, -0.2, 0.41, 0.99):
            ref = special.eval_jacobi(p, a, a, xx)
            assert abs(O.lib().or_jacobi_aa(p, a, xx) - ref) < 1e-13 * (1 + abs(ref))


def test_incomplete_beta_and_its_inverse():
    for a in (0.2, 0.5, 0.85):
        for x in (1e-30, 1e-6, 0.03, 0.4, 0.77, 0.999):
            assert abs(O.lib().or_ibeta(x, a, 1 - a) - special.betainc(a, 1 - a, x)) < 1e-14
        for y in (1e-9, 0.01, 0.3, 0.5, 0.9, 1 - 1e-7):
            ref = special.betaincinv(a, 1 - a, y)
            assert abs(O.lib().or_ibeta_inv(y, a, 1 - a) - ref) <= 1e-12 * ref


def test_fractional_eigenrelation():
    for p in range(6):
        assert abs(O.lib().or_frac_lambda(p, 2.0) - (p + 1) * (p + 2)) < 1e-12 * (p + 1) * (p + 2)
    for alpha in (0.4, 1.3):
        a = alpha / 2
        for p in (0, 1, 3):
            u = lambda y, p=p: (1 - y * y) ** a * special.eval_jacobi(p, a, a, y) if abs(y) < 1 else 0.0
            for x in (-0.55, 0.1, 0.7):
                num = _frac_lap(u, x, alpha)
                ref = O.lib().or_frac_lambda(p, alpha) * special.eval_jacobi(p, a, a, x)
                assert abs(num - ref) < 2e-6 * (1 + abs(ref)), (alpha, p, x, num, ref)


@pytest.mark.parametrize("alpha", [0.4, 1.0, 1.6])
def test_jump_law_is_the_stable_exit_law(alpha):
    delta = 0.013
    r = (delta * special.gamma(1 + alpha)) ** (1 / alpha)
    N = 4000
    J = np.array([O.lib().or_frac_jump(alpha, delta, (i + 0.5) / N) for i in range(N)])
    assert np.all(J >= r * (1 - 1e-12))
    c = math.sin(math.pi * alpha / 2) / math.pi
    dens = lambda y: c * (r * r / (y * y - r * r)) ** (alpha / 2) / y      # one side, |y| > r
    tot, _ = integrate.quad(dens, r, np.inf, limit=400)
    assert abs(2 * tot - 1) < 1e-7
    for f in (1.05, 1.5, 3.0, 10.0):
        tail, _ = integrate.quad(dens, f * r, np.inf, limit=400)
        assert abs(np.mean(J > f * r) - 2 * tail) < 2.0 / N, (f, np.mean(J > f * r), 2 * tail)
    # alpha -> 2: the walk of Lemma 2.1 (jumps of exactly sqrt(2 Delta))
    assert abs(O.lib().or_frac_jump(1.999, delta, 0.5) / math.sqrt(2 * delta) - 1) < 2e-3


def test_fractional_reconstruction_reproduces_the_discrete_space():
    rng = np.random.default_rng(3)
    for alpha, n, M in ((0.4, 7, 3), (1.3, 5, 4)):
        a = alpha / 2
        C = rng.standard_normal((n, M + 1))
        h = 0.7
        x, _ = O.gauss_jacobi(n, a)
        xi = np.zeros(M + 1)
        wts = np.zeros(M + 1)
        O.lib().or_lgl(M, O._ptr(xi), O._ptr(wts))

        def fun(xx, s, deriv=False):
            J = np.array([special.eval_jacobi(p, a, a, xx) for p in range(n)])
            L = np.polynomial.legendre.legval(s, np.eye(M + 1)) if not deriv else \
                np.array([np.polynomial.legendre.legval(s, np.polynomial.legendre.legder(np.eye(M + 1)[q])) for q in range(M + 1)])
            return (1 - xx * xx) ** a * J @ C @ L
        U = np.array([[fun(xj, s) for s in xi] for xj in x])
        Ut = O.frac_reconstruct(alpha, n, M, U.reshape(-1))
        assert np.max(np.abs(Ut.reshape(n, M + 1) - C)) < 1e-12 * np.max(np.abs(C))
        for xx, s in ((0.3, -0.2), (-0.81, 0.77)):
            out = O.frac_evaluate(alpha, n, M, h, Ut, xx, s)
            assert abs(out[0] - fun(xx, s)) < 1e-12 * (1 + abs(out[0]))
            assert abs(out[1] - 2 / h * fun(xx, s, deriv=True)) < 1e-11 * (1 + abs(out[1]))


def test_fractional_source_against_the_hypersingular_integral():
    for alpha in (0.4, 1.3):
        wl = W.small(dim=1, n=5, M_deg=2, src="frac_longtime", f="u_minus_u3", alpha=alpha)
        pb = O.Problem(wl)
        a = alpha / 2
        for t in (0.3, 1.7):
            T = math.exp(math.cos(t)) / (1 + t * t)
            Tp = T * (-math.sin(t) - 2 * t / (1 + t * t))
            u = lambda y: (1 - y * y) ** a * math.sin(y) * T if abs(y) < 1 else 0.0
            for x in (-0.6, 0.05, 0.8):
                ut = (1 - x * x) ** a * math.sin(x) * Tp
                s_num = ut + _frac_lap(u, x, alpha) - (u(x) - u(x) ** 3)
                assert abs(pb.source([x], t) - s_num) < 2e-6 * (1 + abs(s_num)), (alpha, t, x)
                assert abs(pb.exact([x], t) - u(x)) < 1e-15


@pytest.mark.parametrize("alpha", [0.4, 1.3])
def test_fractional_exact_fixed_point(alpha):
    wl = W.small(dim=1, n=5, M_deg=2, M=40, T=0.5, f="u_minus_u3", src="frac_poly", alpha=alpha,
                 src_param=[0.5, -0.3, 0.2, 0.7, 0, 0, 0, 0])
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    xs, _ = special.roots_jacobi(5, alpha / 2, alpha / 2)
    assert np.max(np.abs(x - xs)) < 1e-14
    U = np.array([[pb.exact([xj], tl) for tl in t] for xj in x])
    eps, _, steps = pb.estimate(U)
    assert steps.sum() > 0
    assert np.max(np.abs(eps)) < 1e-12


def test_fractional_iteration_decreases_geometrically():
    wl = W.small(dim=1, n=8, M_deg=4, M=64, iters=6, T=0.5, f="u_minus_u3", src="frac_longtime", alpha=1.3,
                 fresh_per_iter=False)
    pb = O.Problem(wl)
    U, mx = pb.solve()
    x, t = pb.grid(0)
    ex = np.array([[pb.exact([xj], tl) for tl in t] for xj in x])
    assert np.all(mx[1:] < 0.6 * mx[:-1]), mx
    assert np.max(np.abs(U[0] - ex)) < 0.05 * np.max(np.abs(ex))


def test_fractional_picard_form_keeps_the_noise_the_residual_form_removes():
    """The classical (Picard-form) estimator with the alpha-stable walk: its
    iterate is the Monte Carlo estimate of the solution itself, so its error
    stays at the sampling noise of |u| (and the walk's bias), while the residual
    form's increments shrink with the residual -- the paper's contrast (Ex. 2)."""
    res = {}
    for est in ("residual", "picard"):
        wl = W.small(dim=1, n=6, M_deg=3, M=300, iters=6, T=0.5, f="u_minus_u3", src="frac_longtime", alpha=1.3,
                     estimator=est)
        pb = O.Problem(wl)
        U, _ = pb.solve()
        x, t = pb.grid(0)
        ex = np.array([[pb.exact([xj], tl) for tl in t] for xj in x])
        res[est] = np.max(np.abs(U[0] - ex))
    assert res["residual"] < 1e-3, res
    assert res["picard"] > 10 * res["residual"] and res["picard"] < 0.5, res
