"""The polynomial source (HPSMC_SRC_POLY): per interval a tensor-Legendre
polynomial s(x, t) = sum c[k_1..k_d][q] prod_i L_{k_i}(x_i) L_q(xi).

The oracle evaluates it term by term at every path step; the library folds it
into the time contraction of the v* slab.  The oracle is pinned here against
the direct evaluation of the same polynomial written with monomials (an
asymmetric random polynomial, so that a transposed dimension, a reversed time
map or a shifted block fails), and by an exact fixed point of the iteration.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as Lg

import oracle as O
from paper_2608_22190_amd import workloads as W


def legendre_tensor(mono, P, T1):
    """tensor-Legendre coefficients [k_1..k_d][q] (P modes per dimension, T1 in
    time) of a polynomial given by monomial coefficients mono[a_1..a_d][b] in
    (x_1..x_d, xi); every axis is converted with numpy's poly2leg"""
    c = np.asarray(mono, dtype=float)
    for ax in range(c.ndim):
        c = np.apply_along_axis(Lg.poly2leg, ax, c)
    out = np.zeros((P,) * (c.ndim - 1) + (T1,))
    out[tuple(slice(0, s) for s in c.shape)] = c
    return out


def poly_problem(dim, n, degs, T=0.6, seed=0, spatial_deg=3, time_deg=2, **kw):
    """a workload with a random polynomial source per interval; returns the
    workload and the monomial coefficients of each interval's polynomial"""
    rng = np.random.default_rng(seed)
    P = n + 2
    monos, blocks = [], []
    for M in degs:
        tdeg = min(time_deg, M)
        mono = rng.standard_normal((spatial_deg + 1,) * dim + (tdeg + 1,)) * 0.3
        monos.append(mono)
        blocks.append(legendre_tensor(mono, P, M + 1).reshape(-1))
    wl = W.small(dim=dim, n=n, M_deg=list(degs), n_intervals=len(degs), T=T, f="sin", src="poly",
                 ic="nodal", ic_data=np.zeros((1, n ** dim)), **kw)
    return wl.with_(src_coeffs=np.concatenate(blocks)), monos


def _mono_eval(mono, X, xi):
    c = np.asarray(mono)
    for x in list(X) + [xi]:
        powers = x ** np.arange(c.shape[0])
        c = np.tensordot(powers, c, axes=([0], [0]))
    return float(c)


@pytest.mark.parametrize("dim,n,degs", [(1, 4, [3]), (2, 3, [2, 4]), (3, 3, [3])])
def test_oracle_poly_source_is_the_polynomial(dim, n, degs):
    wl, monos = poly_problem(dim, n, degs, seed=dim)
    pb = O.Problem(wl)
    rng = np.random.default_rng(9)
    for iv, mono in enumerate(monos):
        t0, t1 = wl.t_breaks[iv], wl.t_breaks[iv + 1]
        for _ in range(20):
            X = rng.uniform(-1, 1, dim)
            t = rng.uniform(t0, t1)
            ref = _mono_eval(mono, X, 2 * (t - t0) / (t1 - t0) - 1)
            assert abs(pb.source_iv(iv, X, t) - ref) <= 1e-12 * (1 + abs(ref))


def fixed_point_problem(precision="fp64", flip_time=False):
    """u = (1 - x^2)(1 - y^2)(c0 + c1 t) lies in the discrete space; with an
    affine f the source s = u_t - Lap u - f(u) is a polynomial of spatial degree
    4 and time degree 1, given through its Legendre coefficients.  Returns the
    workload and the exact nodal values."""
    c0, c1, a, b = 0.7, -0.4, 0.8, 0.1
    n, M, T = 4, 3, 0.5
    P = n + 2
    one_m_x2 = np.array([1.0, 0.0, -1.0])
    # t = (xi + 1) T / 2 on the single interval: g = c0 + c1 t as a polynomial in xi, g_t = c1
    g = np.array([c0 + c1 * T / 2, c1 * T / 2])
    dg = c1 * np.ones(1)
    # u = w(x) w(y) g(t), Lap u = -2 w(y) g - 2 w(x) g
    U = np.einsum("i,j,k->ijk", one_m_x2, one_m_x2, g)
    Ut = np.einsum("i,j,k->ijk", one_m_x2, one_m_x2, np.pad(dg, (0, 1)))
    lap = np.zeros_like(U)
    lap += np.einsum("i,j,k->ijk", [-2.0, 0, 0], one_m_x2, g)
    lap += np.einsum("i,j,k->ijk", one_m_x2, [-2.0, 0, 0], g)
    mono = Ut - lap - a * U
    mono[0, 0, 0] -= b
    if flip_time:
        mono = mono * np.array([1.0, -1.0])[None, None, :]
    coeffs = legendre_tensor(mono, P, M + 1).reshape(-1)
    wl = W.small(dim=2, n=n, M_deg=M, M=64, T=T, f="affine", f_param=[a, b, 0, 0], src="poly", nstar=70,
                 ic="nodal", ic_data=np.zeros((1, n * n)), precision=precision).with_(src_coeffs=coeffs)
    x, t = O.Problem(wl).grid(0)
    Un = np.zeros((n * n, M + 1))
    for j in range(n * n):
        X = x[list(np.unravel_index(j, (n, n)))]
        for l in range(M + 1):
            Un[j, l] = (1 - X[0] ** 2) * (1 - X[1] ** 2) * (c0 + c1 * t[l])
    return wl, Un


def test_oracle_poly_source_exact_fixed_point():
    """From the exact nodal values every increment vanishes to rounding, for any
    N* and M; the same source with the wrong sign of its time term does not."""
    wl, Un = fixed_point_problem()
    eps, _, _ = O.Problem(wl).estimate(Un.reshape(-1))
    assert np.max(np.abs(eps)) < 1e-13
    wlb, _ = fixed_point_problem(flip_time=True)
    eps_bad, _, _ = O.Problem(wlb).estimate(Un.reshape(-1))
    assert np.max(np.abs(eps_bad)) > 1e-3


# ---------------------------------------------------------------- GPU against the oracle
def _hp():
    from paper_2608_22190_amd import hpsmc
    return hpsmc


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.gpu
@pytest.mark.parametrize("dim,n,degs,M,schedule", [(1, 6, [4], 130, "sequential"), (2, 4, [3, 2], 70, "sequential"),
                                                   (2, 3, [2, 3, 4], 40, "sweeps"), (3, 3, [2], 33, "sequential")])
def test_poly_source_parity_fp64(dim, n, degs, M, schedule):
    H = _hp()
    wl, _ = poly_problem(dim, n, degs, seed=10 + dim, M=M, iters=2, schedule=schedule)
    wl = wl.with_(ic_data=np.random.default_rng(dim).standard_normal((1, n ** dim)) * 0.5)
    _say("poly parity", dim, n, degs, M, schedule)
    with H.Plan(wl) as plan:
        plan.hpsmc_solve()
        Ug = [plan.hpsmc_get_nodes(iv)[0] for iv in range(wl.n_intervals)]
        st = plan.hpsmc_stats()
    Uo, mx = O.Problem(wl).solve()
    scale = max(np.max(np.abs(u)) for u in Uo)
    for iv in range(wl.n_intervals):
        assert np.max(np.abs(Ug[iv] - Uo[iv].reshape(Ug[iv].shape))) <= 1e-12 * scale, iv
    assert np.allclose(st["max_eps"][:len(mx)], mx, rtol=1e-10, atol=1e-14 * scale)


@pytest.mark.gpu
def test_poly_source_exact_fixed_point_gpu():
    H = _hp()
    _say("poly fixed point")
    for prec, bar in (("fp64", 1e-13), ("fp32", 2e-5)):
        wl, Un = fixed_point_problem(prec)
        for mma in (1, 0):
            with H.Plan(wl) as plan:
                plan.hpsmc_set_option("sample_mfma", mma)
                plan.hpsmc_set_nodes(0, Un[None])
                plan.hpsmc_iterate(0, 0)
                eps, _ = plan.hpsmc_get_increment(0)
            assert np.max(np.abs(eps)) < bar, (prec, mma, np.max(np.abs(eps)))


@pytest.mark.gpu
def test_poly_source_fp32_mma_against_vector_and_oracle():
    H = _hp()
    wl, _ = poly_problem(2, 9, [3], seed=5, M=96, iters=1, precision="fp32")
    U = np.random.default_rng(3).standard_normal((1, wl.nsp, 4)) * 0.5
    _say("poly mma")
    res = {}
    for mma in (1, 0):
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("sample_mfma", mma)
            plan.hpsmc_set_launch(1, 4, 4)
            assert plan.hpsmc_get_option("sample_mfma_active") == mma
            plan.hpsmc_set_probe(8)
            plan.hpsmc_set_nodes(0, U)
            plan.hpsmc_iterate(0, 1)
            res[mma] = (plan.hpsmc_get_probe(0)[0], plan.hpsmc_stats()["path_steps"])
    (pm, sm), (pv, sv) = res[1], res[0]
    assert sm == sv
    assert np.max(np.abs(pm - pv)) <= 1e-4 * np.max(np.abs(pv))
    pb = O.Problem(wl)
    Ut = O.reconstruct(2, wl.n, 3, U[0].reshape(-1))
    for node in (0, 40, 200):
        for smp in (0, 7):
            S, _ = pb.sample_path(Ut, 0, 0, 1, node, smp)
            assert abs(pm[node, smp] - S) <= 1e-3 * (abs(S) + np.max(np.abs(pm[node])))


@pytest.mark.gpu
def test_poly_source_eval_and_gradient():
    """hpsmc_eval keeps its meaning (u*, Lap u* - d_t u*: no source); the
    gradient of the terminal misfit with a polynomial source equals the
    oracle's reverse mode."""
    H = _hp()
    n = 3
    c0 = W.c5_coefficients(2, n=n, seed=2).reshape(2, -1)
    wl, _ = poly_problem(2, n, [2], seed=8, M=24, iters=2, nstar=50)
    wl = wl.with_(ic="phi", ic_data=c0, n_instances=2)
    target = W.c5_target(2, wl.nsp, seed=1)
    _say("poly eval and gradient")
    pts = np.array([[0.2, -0.4, 0.3], [-0.7, 0.1, 0.05]])
    Un = np.random.default_rng(4).standard_normal((2, wl.nsp, 3))
    with H.Plan(wl) as plan:
        loss, grad = plan.hpsmc_loss_grad_c0(target)
        plan.hpsmc_set_nodes(0, Un)
        plan.hpsmc_iterate(0, 0)          # reconstructs Un before sampling
        got = plan.hpsmc_eval(0, 1, pts)
    pb = O.Problem(wl)
    for i in range(2):
        lo, go = pb.loss_grad(c0[i], target[i], inst=i)
        assert abs(loss[i] - lo) <= 1e-11 * (1 + abs(lo))
        assert np.max(np.abs(grad[i] - go)) <= 1e-10 * (1 + np.max(np.abs(go)))
    Ut = O.reconstruct(2, n, 2, Un[1].reshape(-1))
    for k in range(2):
        h = wl.t_breaks[1]
        u, ut, lap = O.evaluate(2, n, 2, h, Ut, pts[k, :2], 2 * pts[k, 2] / h - 1)
        assert abs(got[k, 0] - u) <= 1e-12 * (1 + abs(u))
        assert abs(got[k, 1] - (lap - ut)) <= 1e-11 * (1 + abs(lap) + abs(ut))
