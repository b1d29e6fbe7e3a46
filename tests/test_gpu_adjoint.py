"""Adjoint of the iteration (gradient of the terminal misfit with respect to
the initial phi-coefficients) under common random numbers.

FP64: the library's gradient equals the oracle's reverse mode on the same
Philox samples, and central differences (h = 1e-4) of the library's own
forward loss.  FP32: the matrix-core and vector-unit outer products agree,
and the FP32 gradient is close to the FP64 one.
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


def _problem(dim=2, n=3, deg=2, M=24, iters=2, f="sin", precision="fp64", I=2, seed=4, nstar=None):
    c0 = W.c5_coefficients(I, n=n, seed=seed).reshape(I, -1) if dim == 2 else \
        np.random.default_rng(seed).standard_normal((I, n)) / (1.0 + np.arange(n))
    wl = W.small(dim=dim, n=n, M_deg=deg, M=M, T=0.5, iters=iters, f=f, f_param=[0.7, 0.1, 0, 0],
                 src="longtime", ic="phi", ic_data=c0, n_instances=I, precision=precision, nstar=nstar)
    target = W.c5_target(I, wl.nsp, seed=1)
    return wl, c0, target


@pytest.mark.parametrize("dim,n,deg,f", [(2, 3, 2, "sin"), (2, 4, 3, "u_minus_u3"), (1, 6, 4, "sin"),
                                         (2, 3, 2, "affine")])
def test_gradient_matches_oracle_reverse_mode_fp64(dim, n, deg, f):
    H = _hp()
    wl, c0, target = _problem(dim=dim, n=n, deg=deg, f=f, nstar=60)
    _say("adjoint vs oracle", dim, n, deg, f)
    with H.Plan(wl) as plan:
        loss_g, grad_g = plan.hpsmc_loss_grad_c0(target)
    pb = O.Problem(wl)
    for i in range(wl.n_instances):
        loss_o, grad_o = pb.loss_grad(c0[i], target[i], inst=i)
        assert abs(loss_g[i] - loss_o) <= 1e-11 * (1 + abs(loss_o))
        assert np.max(np.abs(grad_g[i] - grad_o)) <= 1e-10 * (1 + np.max(np.abs(grad_o)))


def test_gradient_matches_central_differences_fp64():
    H = _hp()
    wl, c0, target = _problem(dim=2, n=3, deg=2, M=32, nstar=50)
    _say("adjoint vs FD")
    h = 1e-4
    with H.Plan(wl) as plan:
        loss, grad = plan.hpsmc_loss_grad_c0(target)
        for k in range(wl.nsp):
            cp, cm = c0.copy(), c0.copy()
            cp[:, k] += h
            cm[:, k] -= h
            plan.hpsmc_set_initial_coeffs(cp)
            lp, _ = plan.hpsmc_loss_grad_c0(target)
            plan.hpsmc_set_initial_coeffs(cm)
            lm, _ = plan.hpsmc_loss_grad_c0(target)
            fd = (lp - lm) / (2 * h)
            assert np.max(np.abs(fd - grad[:, k]) / (1 + np.abs(grad[:, k]))) <= 1e-6, (k, fd, grad[:, k])


@pytest.mark.parametrize("dim,n", [(1, 9), (2, 6), (2, 7), (2, 17), (2, 18)])
def test_fp32_mfma_and_vector_outer_products_agree(dim, n):
    H = _hp()
    wl, c0, target = _problem(dim=dim, n=n, deg=3, M=96, precision="fp32", I=3)
    _say("mfma vs valu", dim, n)
    res = {}
    for mf in (1, 0):
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("adjoint_mfma", mf)
            res[mf] = plan.hpsmc_loss_grad_c0(target)
    assert np.array_equal(res[0][0], res[1][0])            # same forward
    g1, g0 = res[1][1], res[0][1]
    print("max |g_mfma - g_vector| / max |g_vector| =", np.max(np.abs(g1 - g0)) / np.max(np.abs(g0)))
    assert np.max(np.abs(g1 - g0)) <= 1e-5 * (1 + np.max(np.abs(g0)))
    if n + 2 >= 18:   # the FP64 adjoint's slab chunks stop short of P = 18 (its accuracy there: the FD test)
        return
    with H.Plan(wl.with_(precision="fp64")) as plan:
        _, g64 = plan.hpsmc_loss_grad_c0(target)
    print("max |g32 - g64| / max |g64| =", np.max(np.abs(g1 - g64)) / np.max(np.abs(g64)))
    assert np.max(np.abs(g1 - g64)) <= 1e-3 * np.max(np.abs(g64))


def test_fp32_adjoint_past_p20_keeps_the_outer_product_form():
    """P = 21: past the range of the form that also takes u* on the matrix
    cores, the adjoint keeps u* on the vector units and the outer products on
    the matrix cores; it must agree with the all-vector form (FP32 both)."""
    H = _hp()
    wl, c0, target = _problem(dim=2, n=19, deg=2, M=64, precision="fp32", I=2, nstar=60)
    _say("adjoint p21 mfma vs valu")
    res = {}
    for mf in (1, 0):
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("adjoint_mfma", mf)
            res[mf] = plan.hpsmc_loss_grad_c0(target)
    assert np.array_equal(res[0][0], res[1][0])
    g1, g0 = res[1][1], res[0][1]
    assert np.max(np.abs(g1 - g0)) <= 1e-5 * (1 + np.max(np.abs(g0)))


def test_autograd_function_uses_the_adjoint():
    import torch
    H = _hp()
    wl, c0, target = _problem(dim=2, n=3, deg=2, M=24, nstar=40)
    _say("autograd")
    SMCLoss = H.smc_loss_function()
    dev = torch.device("cuda:0")
    c = torch.tensor(c0, dtype=torch.float64, device=dev, requires_grad=True)
    tg = torch.tensor(target, dtype=torch.float64, device=dev)
    with H.Plan(wl) as plan:
        loss = SMCLoss.apply(c, plan, tg)
        (loss * torch.tensor([1.0, 2.0], dtype=torch.float64, device=dev)).sum().backward()
        ref_loss, ref_grad = plan.hpsmc_loss_grad_c0(target)
    assert np.allclose(loss.detach().cpu().numpy(), ref_loss, rtol=1e-13)
    got = c.grad.cpu().numpy()
    assert np.allclose(got[0], ref_grad[0], rtol=1e-10, atol=1e-14)
    assert np.allclose(got[1], 2 * ref_grad[1], rtol=1e-10, atol=1e-14)
