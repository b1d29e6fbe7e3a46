"""Pins of the oracle's quadrature, polynomials and transforms (Sec. 2.1, 2.3).

Each check ties the oracle to something other than itself: closed-form moments,
NumPy/SciPy's Legendre and Jacobi evaluators, exact polynomial calculus with
NumPy's Legendre series class, and the interpolation identities the paper
states for A (eq. spacelag) and B (eq. timeLag).
"""
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest
from scipy.special import eval_jacobi

import oracle as O


@pytest.mark.parametrize("n", [1, 2, 5, 8, 16, 24])
def test_jg11_exact_to_degree_2n_minus_1(n):
    # int_{-1}^{1} (1-x^2) x^k dx = 0 (k odd), 2/(k+1) - 2/(k+3) (k even)
    x, w = O.jg11(n)
    assert np.all(np.diff(x) > 0) and np.all(np.abs(x) < 1)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1) - 2.0 / (k + 3)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14 * max(1.0, n)
    # and not exact at degree 2n (a Gauss rule, not better); the defect of
    # x^{2n} decays like 4^{-n}, so it is resolvable only for small n
    k = 2 * n
    if n <= 8:
        assert abs(np.dot(w, x ** k) - (2.0 / (k + 1) - 2.0 / (k + 3))) > 1e-10


@pytest.mark.parametrize("M", [1, 2, 4, 6, 12, 16, 26])
def test_lgl_exact_to_degree_2M_minus_1(M):
    xi, w = O.lgl(M)
    assert xi[0] == -1.0 and xi[-1] == 1.0 and np.all(np.diff(xi) > 0)
    for k in range(2 * M):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13
    if M > 1:  # interior LGL nodes are the zeros of L'_M
        assert np.max(np.abs(npleg.legval(xi[1:-1], npleg.legder([0] * M + [1])))) < 1e-10


def test_jg11_nodes_are_interior_lgl_nodes():
    for n in (3, 8, 20):
        x, _ = O.jg11(n)
        xi, _ = O.lgl(n + 1)
        assert np.max(np.abs(x - xi[1:-1])) < 1e-15


def test_polynomials_against_numpy_scipy():
    rng = np.random.default_rng(0)
    for x in rng.uniform(-1, 1, 7):
        for k in range(0, 28):
            e = np.zeros(k + 1); e[k] = 1
            assert abs(O.legendre(k, x) - npleg.legval(x, e)) < 1e-13
            assert abs(O.legendre_deriv(k, x) - npleg.legval(x, npleg.legder(e))) < 1e-11 * (1 + k * k)
            assert abs(O.jacobi11(k, x) - eval_jacobi(k, 1, 1, x)) < 1e-11 * (1 + k)


def test_phi_identity():
    # phi_p = (1-x^2) P_p^{(1,1)} = 2(p+1)/(2p+3) (L_p - L_{p+2})  (Sec. 2.3)
    for x in np.linspace(-0.99, 0.99, 11):
        for p in range(24):
            e = np.zeros(p + 3); e[p] = 1; e[p + 2] = -1
            assert abs(O.phi(p, x) - 2 * (p + 1) / (2 * p + 3) * npleg.legval(x, e)) < 1e-13


def test_phi_second_derivative_reading_R3():
    # -phi_p'' = (p+1)(p+2) P_p^{(1,1)}: exact differentiation of the Legendre form
    for p in range(12):
        e = np.zeros(p + 3); e[p] = 1; e[p + 2] = -1
        d2 = npleg.legder(e * 2 * (p + 1) / (2 * p + 3), 2)
        for x in np.linspace(-0.9, 0.9, 7):
            assert abs(-npleg.legval(x, d2) - (p + 1) * (p + 2) * eval_jacobi(p, 1, 1, x)) < 1e-9
    # the printed factor (p+1) is not the identity for p >= 1
    x = 0.3
    e = np.array([0, 1, 0, -1.0]) * 4 / 5
    assert abs(-npleg.legval(x, npleg.legder(e, 2)) - 2 * eval_jacobi(1, 1, 1, x)) > 1e-3


@pytest.mark.parametrize("n", [1, 4, 9, 16])
def test_A_inverts_phi_collocation(n):
    x, _ = O.jg11(n)
    A = O.matrix_A(n)
    Phi = np.array([[(1 - xj * xj) * eval_jacobi(p, 1, 1, xj) for p in range(n)] for xj in x])
    assert np.max(np.abs(Phi @ A - np.eye(n))) < 1e-12


@pytest.mark.parametrize("M", [1, 2, 6, 16, 26])
def test_B_inverts_legendre_collocation_reading_R5(M):
    xi, _ = O.lgl(M)
    B = O.matrix_B(M)
    Lm = np.array([[npleg.legval(xk, np.eye(M + 1)[q]) for q in range(M + 1)] for xk in xi])
    assert np.max(np.abs(Lm @ B - np.eye(M + 1))) < 1e-12


def _poly_space_time(dim, n, M, rng):
    """random modal coefficients in span{prod phi_{p_i}} x P_M"""
    return rng.standard_normal((n,) * dim + (M + 1,))


def _eval_modal_numpy(c, X, xi, h):
    """u, u_t, Lap u of sum c[p..,q] prod phi_{p_i}(X_i) L_q(xi) by exact
    polynomial calculus in NumPy's Legendre series class (a second route)."""
    dim = c.ndim - 1
    n, T1 = c.shape[0], c.shape[-1]
    phis = []
    for p in range(n):
        e = np.zeros(p + 3); e[p] = 1; e[p + 2] = -1
        phis.append(npleg.Legendre(e * 2 * (p + 1) / (2 * p + 3)))
    u = ut = lap = 0.0
    for idx in np.ndindex(*c.shape[:-1]):
        tq = npleg.legval(xi, c[idx])
        tdq = npleg.legval(xi, npleg.legder(c[idx])) * 2 / h
        vals = [phis[idx[i]](X[i]) for i in range(dim)]
        d2 = [phis[idx[i]].deriv(2)(X[i]) for i in range(dim)]
        prod = np.prod(vals)
        u += prod * tq
        ut += prod * tdq
        for i in range(dim):
            lap += d2[i] * np.prod([vals[m] for m in range(dim) if m != i]) * tq
    return u, ut, lap


@pytest.mark.parametrize("dim,n,M", [(1, 7, 5), (2, 4, 3), (3, 3, 2)])
def test_reconstruct_and_eval_recover_polynomial(dim, n, M):
    """Nodal values of a polynomial of the discrete space reconstruct to it, and
    the oracle's evaluation of u, d_t u, Lap u at off-node points equals exact
    calculus (readings R3, R4)."""
    rng = np.random.default_rng(dim * 100 + n)
    c = _poly_space_time(dim, n, M, rng)
    x, _ = O.jg11(n)
    xi, _ = O.lgl(M)
    h = 0.7
    U = np.zeros((n,) * dim + (M + 1,))
    for idx in np.ndindex(*U.shape[:-1]):
        for k in range(M + 1):
            U[idx + (k,)] = _eval_modal_numpy(c, [x[i] for i in idx], xi[k], h)[0]
    Ut = O.reconstruct(dim, n, M, U.reshape(-1)).reshape(U.shape)
    assert np.max(np.abs(Ut - c)) < 1e-10 * np.max(np.abs(c))
    for _ in range(3):
        X = rng.uniform(-1, 1, dim)
        xq = rng.uniform(-1, 1)
        got = O.evaluate(dim, n, M, h, Ut.reshape(-1), X, xq)
        ref = _eval_modal_numpy(c, X, xq, h)
        scale = 1 + np.max(np.abs(ref))
        assert np.max(np.abs(np.array(got) - np.array(ref))) < 1e-10 * scale
