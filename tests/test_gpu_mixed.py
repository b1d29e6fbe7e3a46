"""The precision switch (HPSMC_FP32_THEN_FP64): an interval is sampled in FP32
until max|eps| < switch_tol, then in FP64 with the counter tags running on.

* Structure: the switched solve equals, bit for bit, an FP32 plan iterated
  until its record falls below switch_tol followed by an FP64 plan that takes
  over the nodal values and iterates on with the same tags.
* Accuracy (reading R24 at the end of the solve): the switched solve reaches
  the FP64 solve's error against the exact solution within 3 sigma, where the
  FP32 solve stays at its rounding floor.
* Algorithm 1's loop condition: with tol below FP32's floor the switched solve
  converges, the FP32 solve does not.
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


def _wl(**kw):
    # the exact solution (1 - x^2)(1 - y^2)(0.8 - 0.4 t + 0.3 t^2) lies in the discrete space: the
    # residual, and with it the noise of the increments, goes to zero, down to the sampling
    # precision's rounding floor
    base = dict(dim=2, n=5, M_deg=4, M=256, iters=16, T=0.5, f="sin", src="quad",
                src_param=[0.8, -0.4, 0.3, 0, 0, 0, 0, 0])
    base.update(kw)
    return W.small(**base)


def _exact(wl):
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    ex = np.zeros((wl.nsp, len(t)))
    for j in range(wl.nsp):
        X = x[list(np.unravel_index(j, (wl.n,) * wl.dim))]
        for l in range(len(t)):
            ex[j, l] = pb.exact(X, t[l])
    return ex


def test_switch_is_fp32_then_fp64_with_the_same_tags():
    H = _hp()
    sw = 1e-5
    wl = _wl(iters=12)
    _say("switch structure")
    with H.Plan(wl.with_(precision="fp32_then_fp64", switch_tol=sw)) as plan:
        plan.hpsmc_set_probe(4)
        plan.hpsmc_solve()
        U_mix = plan.hpsmc_get_nodes(0)
        rec_mix = plan.hpsmc_stats()["max_eps"][:wl.iters]
        ns_mix = plan.hpsmc_stats()["node_samples"]
        inc_mix = plan.hpsmc_get_increment(0)
        probe_mix = plan.hpsmc_get_probe(0)
    # emulation: FP32 iterations until the record drops below sw, then FP64
    with H.Plan(wl.with_(precision="fp32")) as p32, H.Plan(wl.with_(precision="fp64")) as p64:
        p64.hpsmc_set_probe(4)
        p32.hpsmc_start_interval(0)
        k = 0
        recs = []
        while k < wl.iters:
            p32.hpsmc_iterate(0, k)
            recs.append(p32.hpsmc_stats()["max_eps"][-1])
            k += 1
            if recs[-1] < sw:
                break
        k_switch = k
        p64.hpsmc_set_nodes(0, p32.hpsmc_get_nodes(0))
        while k < wl.iters:
            p64.hpsmc_iterate(0, k)
            recs.append(p64.hpsmc_stats()["max_eps"][-1])
            k += 1
        U_emu = p64.hpsmc_get_nodes(0) if k_switch < wl.iters else p32.hpsmc_get_nodes(0)
        inc_emu = p64.hpsmc_get_increment(0)
        probe_emu = p64.hpsmc_get_probe(0)
    print("switch after iteration", k_switch, "records", rec_mix)
    assert 2 <= k_switch < wl.iters - 2
    assert np.array_equal(U_mix, U_emu)
    assert np.array_equal(rec_mix, np.array(recs))
    # the last increment and per-sample values are those of the FP64 phase
    assert np.array_equal(inc_mix[0], inc_emu[0]) and np.array_equal(inc_mix[1], inc_emu[1])
    assert np.array_equal(probe_mix, probe_emu)
    assert ns_mix == wl.iters * wl.nsp * wl.degree[0] * wl.M


def test_switch_reaches_fp64_accuracy():
    H = _hp()
    wl = _wl(iters=24)
    ex = _exact(wl)
    _say("switch accuracy")
    res = {}
    for prec in ("fp64", "fp32", "fp32_then_fp64"):
        with H.Plan(wl.with_(precision=prec, switch_tol=1e-5)) as plan:
            plan.hpsmc_solve()
            U = plan.hpsmc_get_nodes(0)[0]
            eps, ssq = plan.hpsmc_get_increment(0)
            sig = np.sqrt(np.maximum(ssq[0] / wl.M - eps[0] ** 2, 0) / wl.M).max()
        res[prec] = (np.max(np.abs(U - ex)), sig)
    print({k: f"e={v[0]:.3e} sigma={v[1]:.3e}" for k, v in res.items()})
    e64, s64 = res["fp64"]
    emix, _ = res["fp32_then_fp64"]
    e32, _ = res["fp32"]
    # both converge to the FP64 fixed point (the exact solution) within rounding; FP32 alone
    # stays at its rounding floor
    assert emix <= 10 * max(e64, 1e-13) + 3 * s64
    assert e32 > 10 * emix


def test_switch_converges_below_the_fp32_floor():
    H = _hp()
    wl = _wl(iters=30, tol=1e-11, fresh_per_iter=False)
    _say("switch tolerance")
    with H.Plan(wl.with_(precision="fp32_then_fp64", switch_tol=1e-6)) as plan:
        assert plan.hpsmc_solve() == 0
        rec = plan.hpsmc_stats()["max_eps"]
    last = np.flatnonzero(rec > 0)[-1]
    assert rec[last] < 1e-11 and last < wl.iters - 1
    # FP32 alone does not get there: its increments level off at the rounding floor, where
    # their fluctuation may also trip the divergence test (three growths in a row)
    with H.Plan(wl.with_(precision="fp32")) as plan:
        try:
            st = plan.hpsmc_solve()
        except H.HpsmcError as err:
            st = err.status
        rec32 = plan.hpsmc_stats()["max_eps"]
    assert st in (H.ENOTCONVERGED, -5)
    assert rec32[rec32 > 0].min() > 1e-11


def test_switch_rejects_what_it_does_not_cover():
    H = _hp()
    for kw, st in ((dict(switch_tol=0.0), -1), (dict(switch_tol=1e-5, accel="aitken"), -2),
                   (dict(switch_tol=1e-5, estimator="picard", nstar=30), -2)):
        with pytest.raises(H.HpsmcError) as ei:
            H.Plan(_wl().with_(precision="fp32_then_fp64", **kw))
        assert ei.value.status == st
    c0 = W.c5_coefficients(1, n=3, seed=1).reshape(1, -1)
    wl = W.small(dim=2, n=3, M_deg=2, M=16, src="longtime", f="sin", ic="phi", ic_data=c0,
                 precision="fp32_then_fp64", switch_tol=1e-5)
    with H.Plan(wl) as plan:
        with pytest.raises(H.HpsmcError) as ei:
            plan.hpsmc_loss_grad_c0(np.zeros((1, 9)))
        assert ei.value.status == -2
