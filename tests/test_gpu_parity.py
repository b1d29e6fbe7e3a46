"""GPU hot path against the CPU FP64 oracle on identical Philox samples.

FP64 mode must match elementwise: max|u_gpu - u_oracle| <= 1e-12 max|u_oracle|
after every iteration (the increments themselves are compared absolutely on
the same scale, reading R23), and the integer count of residual evaluations
(the sum of exit indices L over all paths) must be identical.  Sizes span
several work items per node and a ragged last chunk.
"""
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


def _random_nodes(wl, seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((wl.n_instances, wl.nsp, wl.degree[0] + 1)) * scale


@pytest.mark.parametrize("dim,n,deg,M,ns", [
    (1, 6, 4, 200, 1), (1, 9, 5, 129, 2), (2, 4, 3, 96, 2), (2, 5, 2, 65, 4),
    (3, 3, 2, 70, 1), (4, 2, 2, 40, 2), (5, 2, 2, 33, 1)])
def test_one_iteration_increment_fp64(dim, n, deg, M, ns):
    H = _hp()
    wl = W.small(dim=dim, n=n, M_deg=deg, M=M, T=0.5, f="sin", src="longtime", c=0.25)
    _say("increment", dim, n, deg, M, ns)
    U = _random_nodes(wl, seed=dim)
    with H.Plan(wl) as plan:
        plan.hpsmc_set_launch(ns, 2, 4)
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 0)
        eps_g, ssq_g = plan.hpsmc_get_increment(0)
        U_g = plan.hpsmc_get_nodes(0)
        st = plan.hpsmc_stats()
    pb = O.Problem(wl)
    eps_o, ssq_o, steps_o = pb.estimate(U[0].reshape(-1), iter_tag=0)
    scale = np.max(np.abs(U))
    assert np.max(np.abs(eps_g[0] - eps_o)) <= TOL * scale
    assert np.max(np.abs(ssq_g[0] - ssq_o)) <= TOL * max(1.0, np.max(np.abs(ssq_o)))
    assert st["path_steps"] == int(np.sum(steps_o))
    U_o, _, _ = pb.iterate(U[0].reshape(-1), iter_tag=0)
    assert np.max(np.abs(U_g[0].reshape(-1) - U_o)) <= TOL * scale


def test_one_iteration_chunked_slabs_fp64():
    """Slabs larger than one LDS chunk (d = 3 with 12 modes in FP64, d = 4, 5)
    stream through LDS in chunks with the leading dimensions fixed."""
    H = _hp()
    for dim, n, deg, M, ns in [(3, 10, 2, 40, 1), (4, 4, 2, 20, 2), (5, 3, 2, 17, 1), (3, 10, 2, 40, 2)]:
        wl = W.small(dim=dim, n=n, M_deg=deg, M=M, T=0.5, f="sin", src="longtime", nstar=30)
        _say("chunked", dim, n, deg, M, ns)
        U = _random_nodes(wl, seed=dim + 10)
        with H.Plan(wl) as plan:
            plan.hpsmc_set_launch(ns, 4, 4)
            plan.hpsmc_set_nodes(0, U)
            plan.hpsmc_iterate(0, 0)
            eps_g, _ = plan.hpsmc_get_increment(0)
            st = plan.hpsmc_stats()
        eps_o, _, steps_o = O.Problem(wl).estimate(U[0].reshape(-1), iter_tag=0)
        assert np.max(np.abs(eps_g[0] - eps_o)) <= TOL * np.max(np.abs(U)), (dim, n)
        assert st["path_steps"] == int(np.sum(steps_o)), (dim, n)


@pytest.mark.parametrize("dim,n,deg,M,iters", [(1, 6, 4, 100, 3), (2, 4, 3, 64, 2)])
def test_solve_single_interval_fp64(dim, n, deg, M, iters):
    H = _hp()
    wl = W.small(dim=dim, n=n, M_deg=deg, M=M, iters=iters, T=0.5)
    _say("solve", dim, n, deg, M, iters)
    with H.Plan(wl) as plan:
        plan.hpsmc_solve()
        Ug = plan.hpsmc_get_nodes(0)[0]
        st = plan.hpsmc_stats()
    Uo, mx = O.Problem(wl).solve()
    assert np.max(np.abs(Ug - Uo[0])) <= TOL * np.max(np.abs(Uo[0]))
    assert np.allclose(st["max_eps"], mx, rtol=1e-9, atol=1e-14)


def test_solve_intervals_sequential_fp64():
    H = _hp()
    wl = W.small(dim=1, n=5, M_deg=[2, 4, 3], M=80, iters=2, T=0.9, n_intervals=3, f="u_minus_u3")
    _say("sequential intervals")
    Uo, _ = O.Problem(wl).solve()
    with H.Plan(wl) as plan:
        plan.hpsmc_solve()
        for iv in range(3):
            Ug = plan.hpsmc_get_nodes(iv)[0]
            assert np.max(np.abs(Ug - Uo[iv])) <= TOL * np.max(np.abs(Uo[iv])), iv


def test_sweeps_uneven_degrees_fp64():
    H = _hp()
    wl = W.small(dim=2, n=3, M_deg=[2, 3, 4], M=40, iters=4, n_intervals=3, f="u2_over_1pu2", src="none",
                 ic="singular", ic_param=[0.5, 0, 0, 0], schedule="sweeps")
    tb = [0.0, 0.04, 0.2, 1.0]
    wl = wl.with_(t_breaks=tb)
    _say("sweeps")
    Uo, mxo = O.Problem(wl).solve()
    with H.Plan(wl) as plan:
        plan.hpsmc_solve()
        st = plan.hpsmc_stats()
        for iv in range(3):
            Ug = plan.hpsmc_get_nodes(iv)[0]
            assert np.max(np.abs(Ug - Uo[iv])) <= TOL * np.max(np.abs(Uo[iv])), iv
    assert np.allclose(st["max_eps"], mxo, rtol=1e-9, atol=1e-14)


def test_instances_phi_initial_data_fp64():
    H = _hp()
    n, I = 4, 3
    c0 = W.c5_coefficients(I, n=n, seed=7).reshape(I, -1)
    wl = W.small(dim=2, n=n, M_deg=3, M=50, iters=2, f="sin", src="longtime", ic="phi", ic_data=c0,
                 n_instances=I)
    _say("instances")
    with H.Plan(wl) as plan:
        plan.hpsmc_solve()
        Ug = plan.hpsmc_get_nodes(0)
    pb = O.Problem(wl)
    for i in range(I):
        Uo, _ = pb.solve(inst=i)
        assert np.max(np.abs(Ug[i] - Uo[0])) <= TOL * np.max(np.abs(Uo[0])), i


@pytest.mark.parametrize("dim,n,deg", [(1, 7, 5), (2, 4, 3), (3, 3, 2), (5, 2, 2)])
def test_reconstruction_eval_matches_oracle(dim, n, deg):
    H = _hp()
    wl = W.small(dim=dim, n=n, M_deg=deg, M=1, T=0.7, nstar=1)
    _say("reconstruct", dim, n, deg)
    U = _random_nodes(wl, seed=11)
    rng = np.random.default_rng(5)
    pts = np.concatenate([rng.uniform(-1, 1, (9, dim)), rng.uniform(0, 0.7, (9, 1))], axis=1)
    with H.Plan(wl) as plan:
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 0)   # reconstructs from U before sampling
        # the reconstruction used by the iteration is that of U (before update)
        got = plan.hpsmc_eval(0, 0, pts)
    Ut = O.reconstruct(dim, n, deg, U[0].reshape(-1))
    for k in range(pts.shape[0]):
        u, ut, lap = O.evaluate(dim, n, deg, 0.7, Ut, pts[k, :dim], 2 * pts[k, dim] / 0.7 - 1)
        scale = 1 + abs(u) + abs(ut) + abs(lap)
        assert abs(got[k, 0] - u) <= 1e-12 * scale
        assert abs(got[k, 1] - (lap - ut)) <= 1e-11 * scale


@pytest.mark.parametrize("dim,f", [(1, "u_minus_u3"), (2, "sin"), (3, "neg_u3")])
def test_exact_fixed_point_gpu(dim, f):
    H = _hp()
    wl = W.small(dim=dim, n=3, M_deg=2, M=64, T=0.5, src="quad", f=f, nstar=80,
                 src_param=[0.8, -0.4, 0.3, 0, 0, 0, 0, 0])
    _say("fixed point", dim, f)
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    U = np.zeros((1, wl.nsp, 3))
    for jf in range(wl.nsp):
        X = [x[i] for i in np.unravel_index(jf, (3,) * dim)]
        for l in range(3):
            U[0, jf, l] = pb.exact(X, t[l])
    for prec in ("fp64", "fp32"):
        with H.Plan(wl.with_(precision=prec)) as plan:
            plan.hpsmc_set_nodes(0, U)
            plan.hpsmc_iterate(0, 0)
            eps, _ = plan.hpsmc_get_increment(0)
        assert np.max(np.abs(eps)) < (1e-13 if prec == "fp64" else 2e-5), prec


def test_probe_samples_match_oracle_paths():
    H = _hp()
    wl = W.small(dim=2, n=4, M_deg=3, M=300, T=0.5, f="sin", src="longtime")
    _say("probe")
    U = _random_nodes(wl, seed=3)
    with H.Plan(wl) as plan:
        plan.hpsmc_set_probe(8)
        plan.hpsmc_set_nodes(0, U)
        plan.hpsmc_iterate(0, 5)
        pr = plan.hpsmc_get_probe(0)[0]
    pb = O.Problem(wl)
    Ut = O.reconstruct(2, 4, 3, U[0].reshape(-1))
    for node in (0, 7, 21, 47):
        for smp in range(8):
            S, _ = pb.sample_path(Ut, 0, 0, 5, node, smp)
            assert abs(pr[node, smp] - S) <= 1e-12 * (1 + abs(S))


def test_edge_cases_fp64():
    H = _hp()
    _say("edges")
    for wl in [W.small(dim=1, n=1, M_deg=1, M=1, nstar=1),
               W.small(dim=1, n=2, M_deg=1, M=63, nstar=3),
               W.small(dim=2, n=1, M_deg=2, M=65, nstar=2),
               W.small(dim=1, n=3, M_deg=2, M=257, iters=1, fresh_per_iter=False)]:
        with H.Plan(wl) as plan:
            plan.hpsmc_solve()
            Ug = plan.hpsmc_get_nodes(0)[0]
        Uo, _ = O.Problem(wl).solve()
        # n = 1 puts the only node at x = 0 where the solution vanishes: the
        # scale then falls back to 1 (the nodes agree to rounding, not to 0)
        assert np.max(np.abs(Ug - Uo[0])) <= TOL * max(1.0, np.max(np.abs(Uo[0])))


def test_deterministic_rerun():
    H = _hp()
    wl = W.small(dim=2, n=4, M_deg=3, M=200, iters=2, precision="fp32")
    _say("determinism")
    outs = []
    for _ in range(2):
        with H.Plan(wl) as plan:
            plan.hpsmc_solve()
            outs.append(plan.hpsmc_get_nodes(0))
    assert np.array_equal(outs[0], outs[1])


def test_fp32_sampling_against_fp64_and_exact():
    """Reading R24: same Philox words in both precisions; the FP32 result is
    within the Monte Carlo noise of the FP64 one and no worse against the
    exact solution than e64 + 3 sigma."""
    H = _hp()
    wl = W.small(dim=2, n=5, M_deg=4, M=512, iters=4, T=0.5, f="sin", src="longtime")
    _say("fp32 vs fp64")
    res = {}
    for prec in ("fp64", "fp32"):
        with H.Plan(wl.with_(precision=prec)) as plan:
            plan.hpsmc_solve()
            res[prec] = plan.hpsmc_get_nodes(0)[0]
            _, ssq = plan.hpsmc_get_increment(0)
            eps, _ = plan.hpsmc_get_increment(0)
            if prec == "fp64":
                sig = np.sqrt(np.maximum(ssq[0] / wl.M - eps[0] ** 2, 0) / wl.M).max()
    pb = O.Problem(wl)
    x, t = pb.grid(0)
    ex = np.zeros_like(res["fp64"])
    for jf in range(wl.nsp):
        X = [x[i] for i in np.unravel_index(jf, (wl.n,) * 2)]
        for l in range(len(t)):
            ex[jf, l] = pb.exact(X, t[l])
    e64 = np.max(np.abs(res["fp64"] - ex))
    e32 = np.max(np.abs(res["fp32"] - ex))
    d = np.max(np.abs(res["fp32"] - res["fp64"]))
    print(f"e64={e64:.3e} e32={e32:.3e} |u32-u64|={d:.3e} sigma={sig:.3e}")
    assert e32 <= e64 + 3 * sig
    assert d <= 3 * sig + 1e-5


def test_graph_replays_match_eager_solve():
    """hipGraph of a whole solve: every replay (with eager work and
    synchronizations in between) equals the eager solve bit for bit."""
    import torch
    H = _hp()
    _say("graph")
    for wl in [W.small(dim=2, n=4, M_deg=3, M=100, iters=2, precision="fp32"),
               W.small(dim=1, n=5, M_deg=[2, 3], M=80, iters=2, T=0.8, n_intervals=2)]:
        with H.Plan(wl) as plan:
            plan.hpsmc_solve()
            ref = [plan.hpsmc_get_nodes(iv) for iv in range(wl.n_intervals)]
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("graph", 1)
            for rep in range(3):
                plan.hpsmc_solve()
                torch.cuda.synchronize()
                got = [plan.hpsmc_get_nodes(iv) for iv in range(wl.n_intervals)]
                for a, b in zip(got, ref):
                    assert np.array_equal(a, b), rep
                x = torch.randn(1 << 20, device="cuda")          # eager work between replays
                (x * 2).sum().item()
                plan.hpsmc_set_nodes(0, np.zeros_like(ref[0]))   # clobber: the replay re-initializes
