"""hpsmc_eval_noalloc, the evaluation entry point for callers that cannot
allocate device memory: through the C ABI it returns exactly what hpsmc_eval
returns, on two calls in a row (the second with fewer points, so stale staging
from the first call would show), on a second plan, and it rejects a point count
beyond its static staging before any device work."""
import ctypes as C

import numpy as np
import pytest

from paper_2608_22190_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _points(rng, npts, dim, T):
    return np.concatenate([rng.uniform(-1, 1, (npts, dim)), rng.uniform(0, T, (npts, 1))], axis=1)


def _call(H, fn, plan, iv, inst, pts):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.full((pts.shape[0], 2), np.nan)
    st = getattr(H.lib(), fn)(plan.h, iv, inst, pts.ctypes.data_as(C.c_void_p), pts.shape[0],
                              out.ctypes.data_as(C.c_void_p), None)
    return st, out


@pytest.mark.parametrize("dim,n,deg,I", [(2, 6, 4, 3), (5, 3, 2, 1), (1, 9, 5, 2)])
def test_noalloc_eval_matches_eval(dim, n, deg, I):
    from paper_2608_22190_amd import hpsmc as H
    wl = W.small(dim=dim, n=n, M_deg=deg, M=8, T=0.7, nstar=4, n_instances=I)
    _say("noalloc", dim, n, deg, I)
    rng = np.random.default_rng(dim)
    U = rng.standard_normal((I, wl.nsp, deg + 1))
    with H.Plan(wl) as plan:
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 0)          # the reconstruction of U
        for npts, inst in ((5000, I - 1), (37, 0)):
            pts = _points(rng, npts, dim, 0.7)
            st0, ref = _call(H, "hpsmc_eval", plan, 0, inst, pts)
            st1, got = _call(H, "hpsmc_eval_noalloc", plan, 0, inst, pts)
            assert st0 == 0 and st1 == 0
            assert np.all(np.isfinite(ref))
            assert np.array_equal(got, ref), (npts, np.max(np.abs(got - ref)))
    # a second plan on the same GPU shares the array: its own values come back
    wl2 = wl.with_(seed=3)
    with H.Plan(wl2) as plan2:
        plan2.hpsmc_set_nodes(0, -2.0 * U)
        plan2.hpsmc_iterate(0, 1)
        pts = _points(rng, 11, dim, 0.7)
        _, ref = _call(H, "hpsmc_eval", plan2, 0, 0, pts)
        st, got = _call(H, "hpsmc_eval_noalloc", plan2, 0, 0, pts)
        assert st == 0 and np.array_equal(got, ref)


def test_noalloc_eval_rejects_too_many_points():
    from paper_2608_22190_amd import hpsmc as H
    wl = W.small(dim=2, n=3, M_deg=2, M=4, nstar=2)
    limit = (16 << 20) // 8 // (2 + 3)
    with H.Plan(wl) as plan:
        plan.hpsmc_iterate(0, 0)
        pts = np.zeros((limit + 1, 3))
        st, out = _call(H, "hpsmc_eval_noalloc", plan, 0, 0, pts)
        assert st == -1                   # HPSMC_EINVAL
        assert np.all(np.isnan(out))      # nothing was written
        st, out = _call(H, "hpsmc_eval_noalloc", plan, 0, 0, pts[:limit])
        assert st == 0 and np.all(np.isfinite(out))
