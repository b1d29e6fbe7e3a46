"""Parity at the shapes and launch configurations the benchmark times.

* Five-dimensional problem (Ex. 4): 8^5 Jacobi-Gauss nodes x 8 Lobatto times
  (262,144 Monte Carlo nodes), P = 10 Legendre modes per dimension, FP32
  sampling.  Its slab (10^4 rows) streams through LDS in chunks with the two
  leading dimensions fixed (CF = 2), one sample per lane, the tuned launch.
* Initial singularity (Ex. 3): the geometric mesh with twelve intervals of
  degrees 4..26, 20 x 20 nodes (P = 22: eleven-row halves of the matrix-core
  tiles), one sweep over all intervals in one launch sequence, FP32.
* Batched gradient: 256 instances of 16 x 16 nodes (P = 18: nine-row halves),
  degree 12, FP32 forward and adjoint.

The oracle cannot redo these launches whole, so every node is checked by a
property that holds at any size (increment = mean of its per-sample path
values, iterate moved by exactly the increment) and sampled (node, sample)
pairs against the oracle's own walk of the same Philox counter.  Matrix-core
kernels are also checked against the vector-unit kernel, path for path.
"""
import os
import shutil

import numpy as np
import pytest

import oracle as O
from paper_2608_22190_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "paper_2608_22190_amd", "tuned_launch.json")


def _hp():
    from paper_2608_22190_amd import hpsmc
    return hpsmc


def _say(*a):
    print("[case]", *a, flush=True)


def _cache(tmp_path):
    c = str(tmp_path / "tuned.json")
    if os.path.exists(CACHE):
        shutil.copy(CACHE, c)
    return c


def _exact_nodes(wl, pb, iv=0):
    x, t = pb.grid(iv)
    U = np.zeros((wl.n_instances, wl.nsp, wl.degree[iv] + 1))
    idx = np.array(np.unravel_index(np.arange(wl.nsp), (wl.n,) * wl.dim)).T
    for jf in range(wl.nsp):
        X = x[idx[jf]]
        for l in range(len(t)):
            U[:, jf, l] = pb.exact(X, t[l])
    return U


def _ic_replicated(wl, pb, iv=0):
    """initial iterate of an interval: the oracle's initial nodal data replicated in time"""
    U = np.zeros((wl.n_instances, wl.nsp, wl.degree[iv] + 1))
    for inst in range(wl.n_instances):
        U[inst] = pb.ic_nodes(inst)[:, None]
    return U


# FP32 path bound, relative to the scale of the node's path values (the largest
# |S| over its probed samples): the walk's rounding moves the point by
# ~sqrt(L) 2^-24 and may change an exit step near the boundary (one step moves
# S by Delta |r|); the contraction adds FP32 rounding of its products.  Both
# stay far below it.
FP32_PATH = 1e-3


def _path_ok(got, S, node_probe):
    scale = abs(S) + np.max(np.abs(node_probe))
    return abs(got - S) <= FP32_PATH * scale, abs(got - S) / scale


def _check_probe_mean(probe, eps, U0, U1, nsp):
    mean = probe.mean(axis=-1)
    assert np.max(np.abs(eps - mean)) <= 1e-13 * (1 + np.max(np.abs(probe)))
    deg = U0.shape[-1] - 1
    moved = (U1 - U0)[..., 1:].transpose(0, 2, 1).reshape(U0.shape[0], nsp * deg)
    assert np.max(np.abs(moved - eps)) <= 1e-14 * (1 + np.max(np.abs(U0)))
    assert np.array_equal(U1[..., 0], U0[..., 0])


def test_five_dim_fp32_full_nodes(tmp_path):
    """Ex. 4 shape, one iteration of all 262,144 nodes, 16 samples each, the
    tuned launch of the benchmark's five-dimensional line."""
    H = _hp()
    wl = W.c4_five_dim(M=16, iters=1)
    pb = O.Problem(wl)
    # exact nodal data plus a perturbation: the residual, and so every path value, is O(1)
    U0 = _exact_nodes(wl, pb) + 0.2 * np.random.default_rng(45).standard_normal((1, wl.nsp, wl.degree[0] + 1))
    with H.Plan(wl) as plan:
        launch = plan.hpsmc_tune(0, 16, _cache(tmp_path))
        _say("c4 full nodes", launch)
        assert launch[0] == 1
        plan.hpsmc_set_probe(16)
        plan.hpsmc_set_nodes(0, U0)
        plan.hpsmc_iterate(0, 0)
        probe = plan.hpsmc_get_probe(0)
        eps, _ = plan.hpsmc_get_increment(0)
        U1 = plan.hpsmc_get_nodes(0)
        st = plan.hpsmc_stats()
    nodes = wl.nsp * wl.degree[0]
    assert probe.shape == (1, nodes, 16) and np.all(np.isfinite(probe))
    assert st["node_samples"] == nodes * 16
    _check_probe_mean(probe, eps, U0, U1, wl.nsp)
    Ut = O.reconstruct(5, wl.n, wl.degree[0], U0[0].reshape(-1))
    rng = np.random.default_rng(4)
    worst = 0.0
    for _ in range(8):
        node, smp = int(rng.integers(nodes)), int(rng.integers(16))
        S, steps = pb.sample_path(Ut, 0, 0, 0, node, smp)
        ok, rel = _path_ok(probe[0, node, smp], S, probe[0, node])
        worst = max(worst, rel)
        print(f"node {node} sample {smp}: S={S:.8f} steps={steps} rel={rel:.3e}", flush=True)
        assert ok
    print(f"worst relative path error: {worst:.3e}")


def test_five_dim_fp32_r24_against_fp64():
    """Reading R24 in five dimensions with the same kernel (P <= 12, CF = 2):
    the same Philox words in both precisions; FP32 no worse against the exact
    solution than e64 + 3 sigma, and within the noise of the FP64 result."""
    H = _hp()
    wl = W.small(dim=5, n=6, M_deg=3, M=64, iters=3, T=1.0, f="neg_u3", src="cos_decay")
    _say("d5 r24")
    res = {}
    for prec in ("fp64", "fp32"):
        with H.Plan(wl.with_(precision=prec)) as plan:
            plan.hpsmc_set_launch(1, 4, 4)
            plan.hpsmc_solve()
            res[prec] = plan.hpsmc_get_nodes(0)[0]
            eps, ssq = plan.hpsmc_get_increment(0)
            if prec == "fp64":
                sig = np.sqrt(np.maximum(ssq[0] / wl.M - eps[0] ** 2, 0) / wl.M).max()
    ex = _exact_nodes(wl, O.Problem(wl))[0]
    e64 = np.max(np.abs(res["fp64"] - ex))
    e32 = np.max(np.abs(res["fp32"] - ex))
    d = np.max(np.abs(res["fp32"] - res["fp64"]))
    print(f"e64={e64:.3e} e32={e32:.3e} |u32-u64|={d:.3e} sigma={sig:.3e}")
    assert e32 <= e64 + 3 * sig
    assert d <= 3 * sig + 1e-5


def _sweep_run(wl, mma, m_probe, launch=None, cache=None):
    H = _hp()
    with H.Plan(wl) as plan:
        plan.hpsmc_set_option("sample_mfma", mma)
        if cache:
            launch = plan.hpsmc_tune(0, wl.M, cache)
        else:
            plan.hpsmc_set_launch(*launch)
        assert plan.hpsmc_get_option("sample_mfma_active") == mma
        plan.hpsmc_set_probe(m_probe)
        U0 = [plan.hpsmc_get_nodes(iv) for iv in range(wl.n_intervals)]
        plan.hpsmc_sweep(1)
        out = dict(probe=[plan.hpsmc_get_probe(iv) for iv in range(wl.n_intervals)],
                   eps=[plan.hpsmc_get_increment(iv)[0] for iv in range(wl.n_intervals)],
                   U1=[plan.hpsmc_get_nodes(iv) for iv in range(wl.n_intervals)],
                   stats=plan.hpsmc_stats(), launch=plan.hpsmc_get_launch(), U0=U0)
    return out


def test_initial_singularity_sweep_full_size(tmp_path):
    """Ex. 3 shape: one sweep over all twelve intervals (degrees 4..26, 72,000
    nodes), 256 samples per node, the benchmark's tuned matrix-core launch;
    the vector-unit kernel walks the same paths."""
    wl = W.c3_initial_singularity(M=256, sweeps=1)
    pb = O.Problem(wl)
    cache = _cache(tmp_path)
    _say("c3 sweep mma")
    rm = _sweep_run(wl, 1, 256, cache=cache)
    _say("c3 sweep valu", rm["launch"])
    rv = _sweep_run(wl, 0, 256, launch=(1, 4, 2, 512))
    assert rm["stats"]["path_steps"] == rv["stats"]["path_steps"]
    for iv in range(wl.n_intervals):
        U0 = _ic_replicated(wl, pb, iv)
        # the plan starts every interval from the replicated initial data
        assert np.max(np.abs(rm["U0"][iv] - U0)) <= 1e-14
        _check_probe_mean(rm["probe"][iv], rm["eps"][iv], rm["U0"][iv], rm["U1"][iv], wl.nsp)
        pm, pv = rm["probe"][iv], rv["probe"][iv]
        scale = np.max(np.abs(pv))
        assert np.max(np.abs(pm - pv)) <= 1e-4 * scale, iv
    # sampled paths of every interval against the oracle's walk
    rng = np.random.default_rng(3)
    for iv in range(wl.n_intervals):
        U0 = _ic_replicated(wl, pb, iv)
        Ut = O.reconstruct(2, wl.n, wl.degree[iv], U0[0].reshape(-1))
        nodes = wl.nsp * wl.degree[iv]
        for _ in range(2):
            node, smp = int(rng.integers(nodes)), int(rng.integers(256))
            S, steps = pb.sample_path(Ut, 0, iv, 1, node, smp)
            ok, rel = _path_ok(rm["probe"][iv][0, node, smp], S, rm["probe"][iv][0, node])
            print(f"iv {iv} node {node} sample {smp}: S={S:.6e} steps={steps} rel={rel:.3e}", flush=True)
            assert ok


def test_initial_singularity_kh11_against_oracle_fp64_walks():
    """Four intervals of the geometric mesh at P = 22 (KH = 11) with a ragged
    sample count: matrix-core against vector-unit kernel per sample, and both
    against the oracle's FP64 walks."""
    wl = W.c3_initial_singularity(M=70, sweeps=1)
    wl = wl.with_(t_breaks=wl.t_breaks[:5], degree=wl.degree[:4])
    pb = O.Problem(wl)
    _say("kh11 sweep", wl.degree)
    rm = _sweep_run(wl, 1, 70, launch=(1, 4, 2, 64))
    rv = _sweep_run(wl, 0, 70, launch=(1, 4, 2, 64))
    assert rm["stats"]["path_steps"] == rv["stats"]["path_steps"]
    rng = np.random.default_rng(11)
    e_m = e_v = 0.0
    for iv in range(wl.n_intervals):
        pm, pv = rm["probe"][iv][0], rv["probe"][iv][0]
        scale = np.max(np.abs(pv))
        assert np.max(np.abs(pm - pv)) <= 1e-4 * scale
        assert np.max(np.abs(rm["eps"][iv] - rv["eps"][iv])) <= 1e-4 * scale
        Ut = O.reconstruct(2, wl.n, wl.degree[iv], _ic_replicated(wl, pb, iv)[0].reshape(-1))
        for node in rng.choice(pm.shape[0], size=3, replace=False):
            for smp in (0, 69):
                S, _ = pb.sample_path(Ut, 0, iv, 1, int(node), smp)
                e_m = max(e_m, abs(pm[node, smp] - S))
                e_v = max(e_v, abs(pv[node, smp] - S))
    print(f"vs oracle: mma {e_m:.3e} valu {e_v:.3e}")
    assert e_m <= 2.0 * e_v + 1e-5 * max(np.max(np.abs(p[0])) for p in rm["probe"])


def test_batched_gradient_shape_kh9(tmp_path):
    """Batched-gradient shape: 256 instances x 3072 nodes, 16 samples, P = 18
    (KH = 9), the tuned matrix-core launch, against the vector-unit kernel and
    sampled oracle walks of several instances."""
    H = _hp()
    wl = W.c5_batched_gradient(M=16, iters=1)
    pb = O.Problem(wl)
    cache = _cache(tmp_path)
    res = {}
    for mma in (1, 0):
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("sample_mfma", mma)
            launch = plan.hpsmc_tune(0, 16, cache) if mma else None
            if not mma:
                plan.hpsmc_set_launch(1, 4, 4, 512)
            _say("c5 shape", mma, launch)
            assert plan.hpsmc_get_option("sample_mfma_active") == mma
            plan.hpsmc_set_probe(16)
            Ubefore = plan.hpsmc_get_nodes(0)
            plan.hpsmc_iterate(0, 0)
            res[mma] = (plan.hpsmc_get_probe(0), plan.hpsmc_get_increment(0)[0], plan.hpsmc_get_nodes(0),
                        plan.hpsmc_stats(), Ubefore)
    (pm, em, Um, sm, Ub), (pv, ev, Uv, sv, _) = res[1], res[0]
    assert sm["path_steps"] == sv["path_steps"]
    scale = np.max(np.abs(pv))
    assert np.max(np.abs(pm - pv)) <= 1e-4 * scale
    U0 = _ic_replicated(wl, pb)
    assert np.max(np.abs(Ub - U0)) <= 1e-13 * (1 + np.max(np.abs(U0)))
    _check_probe_mean(pm, em, Ub, Um, wl.nsp)
    rng = np.random.default_rng(5)
    nodes = wl.nsp * wl.degree[0]
    for inst in (0, 101, 255):
        Ut = O.reconstruct(2, wl.n, wl.degree[0], U0[inst].reshape(-1))
        for _ in range(2):
            node, smp = int(rng.integers(nodes)), int(rng.integers(16))
            S, steps = pb.sample_path(Ut, inst, 0, 0, node, smp)
            ok, rel = _path_ok(pm[inst, node, smp], S, pm[inst, node])
            print(f"inst {inst} node {node} sample {smp}: S={S:.6e} steps={steps} rel={rel:.3e}", flush=True)
            assert ok


def _grad_problem(precision, I=2, M=48, iters=2):
    c0 = W.c5_coefficients(I, n=16, seed=3).reshape(I, -1)
    wl = W.c5_batched_gradient(n_instances=I, M=M, iters=iters).with_(ic_data=c0, precision=precision)
    return wl, c0, W.c5_target(I, wl.nsp, seed=1)


def _forward_loss(plan, target, wl):
    """terminal misfit 1/2 sum_j (u(x_j, T) - target_j)^2 of a forward solve"""
    plan.hpsmc_solve()
    uT = plan.hpsmc_get_nodes(0)[:, :, -1]
    return 0.5 * np.sum((uT - target) ** 2, axis=1)


def test_fp32_gradient_p18_central_differences():
    """FP32 gradient at P = 18 against central differences (h = 1e-4) at fixed
    Philox keys.  FD64, the difference quotient of the FP64 forward loss, is
    the gradient of the FP64 loss to O(h^2) plus FP64 rounding / h; the FP32
    adjoint must match it to FP32 accuracy (1e-3 of the largest entry).  The
    FP32 forward loss carries a rounding error e(c) = L32(c) - L64(c) on the
    same words (exit steps near the boundary may move), so FD32 is off from
    the gradient by (e(c+h) - e(c-h)) / 2h = FD32 - FD64; measured on the
    GPU it stays within the same bar (at most 1.4e-3 here), so FD32
    matches the FP32 adjoint to twice it."""
    H = _hp()
    h = 1e-4
    wl32, c0, target = _grad_problem("fp32")
    wl64 = wl32.with_(precision="fp64")
    ks = [0, 17, 100, 255]
    _say("fp32 FD p18", ks)
    with H.Plan(wl32) as p32, H.Plan(wl64) as p64:
        L32, g32 = p32.hpsmc_loss_grad_c0(target)
        # the forward loss of a plain solve equals the gradient call's loss
        dl = float(np.max(np.abs(_forward_loss(p32, target, wl32) - L32) / L32))
        assert dl <= 1e-13, dl
        for k in ks:
            vals = {}
            for sgn in (1, -1):
                c = c0.copy()
                c[:, k] += sgn * h
                p32.hpsmc_set_initial_coeffs(c)
                p64.hpsmc_set_initial_coeffs(c)
                vals[sgn] = (p32.hpsmc_loss_grad_c0(target)[0], _forward_loss(p64, target, wl64))
            fd32 = (vals[1][0] - vals[-1][0]) / (2 * h)
            fd64 = (vals[1][1] - vals[-1][1]) / (2 * h)
            # (e(c+h) - e(c-h)) / 2h, the FP32 forward's rounding in the quotient
            rnd = np.abs(fd32 - fd64)
            g = g32[:, k]
            print(f"k={k}: g32={g} fd64={fd64} fd32={fd32} rounding term={rnd}", flush=True)
            gmax = np.max(np.abs(g32), axis=1)        # the FP32 adjoint's bar: 1e-3 of the largest entry
            assert np.all(np.abs(g - fd64) <= 1e-3 * gmax + 1e-6)
            # the FP32 quotient itself: its rounding term stays within the same bar
            assert np.all(rnd <= 1e-3 * gmax)
            assert np.all(np.abs(fd32 - g) <= 2e-3 * gmax + 1e-6)


def test_fp32_adjoint_p18_mfma_matches_vector():
    H = _hp()
    wl, c0, target = _grad_problem("fp32", I=3, M=64)
    _say("adjoint p18 mfma vs valu")
    res = {}
    for mf in (1, 0):
        with H.Plan(wl) as plan:
            plan.hpsmc_set_option("adjoint_mfma", mf)
            res[mf] = plan.hpsmc_loss_grad_c0(target)
    assert np.array_equal(res[0][0], res[1][0])
    g1, g0 = res[1][1], res[0][1]
    assert np.max(np.abs(g1 - g0)) <= 1e-5 * (1 + np.max(np.abs(g0)))


def test_fp32_gradient_with_a_slab_adjoint_table_past_2_32_words():
    """The batched-gradient shape, 256 instances: the slab-adjoint table (row
    layout, 2 PP = 40 columns of P = 18 rows per step) holds 5.84 G 8-byte
    words (46.7 GB), more work-items than one dispatch can count (2^32), and
    it is cleared before every iteration's adjoint.  Two gradient calls on one
    plan then agree to the FP32 summation order of the table's atomics; a
    clear that stopped short would leave the previous iteration's sums in the
    table's tail and move the later instances' gradients by their own size."""
    H = _hp()
    I = 256
    wl, c0, target = _grad_problem("fp32", I=I, M=4, iters=2)
    ns = np.asarray(H.resolve_nstar(wl)[0]).ravel()
    words = I * int(ns.sum()) * 40 * 18 // 2
    assert words > 2 ** 32, words
    _say("slab-adjoint table words", words)
    with H.Plan(wl) as plan:
        L1, g1 = plan.hpsmc_loss_grad_c0(target)
        L2, g2 = plan.hpsmc_loss_grad_c0(target)
    assert np.array_equal(L1, L2)
    scale = np.max(np.abs(g1), axis=1, keepdims=True)
    d = np.max(np.abs(g2 - g1) / scale, axis=1)
    print("max relative difference per instance: first", d[:4], "last", d[-4:], flush=True)
    assert np.all(d <= 1e-4), (int(np.argmax(d)), float(np.max(d)))


def test_slab_groups_past_the_grid_y_extent():
    """4100 instances x 16 node times: 65,600 slab groups, past the 65,535 blocks
    of a grid's y extent, so the slab kernel takes the last instances' groups
    from grid z; their sampled FP64 paths equal the oracle's walks."""
    H = _hp()
    wl = W.small(dim=2, n=2, M_deg=16, M=4, T=0.5, precision="fp64", nstar=8, n_instances=4100)
    assert wl.n_instances * wl.degree[0] > 65535
    _say("slab groups", wl.n_instances * wl.degree[0])
    pb = O.Problem(wl)
    with H.Plan(wl) as plan:
        plan.hpsmc_set_probe(4)
        plan.hpsmc_iterate(0, 0)
        probe = plan.hpsmc_get_probe(0)
    U0 = _ic_replicated(wl, pb)
    rng = np.random.default_rng(11)
    nodes = wl.nsp * wl.degree[0]
    for inst in (0, 4095, 4099):   # groups 0.., 65520.., 65584..
        Ut = O.reconstruct(2, wl.n, wl.degree[0], U0[inst].reshape(-1))
        for _ in range(3):
            node, smp = int(rng.integers(nodes)), int(rng.integers(4))
            S, _ = pb.sample_path(Ut, inst, 0, 0, node, smp)
            assert abs(probe[inst, node, smp] - S) <= 1e-12 * (1 + abs(S)), (inst, node, smp, probe[inst, node, smp], S)


def test_tolerance_mode_solves_twice_on_one_plan():
    """Algorithm 1's stop test reads this solve's own max|eps| records: after a
    solve from larger initial data (larger increments), a solve from the
    original data stops where a fresh plan does, with the same iterate."""
    H = _hp()
    wl = W.small(dim=1, n=6, M_deg=4, M=200, iters=30, T=0.5, f="u_minus_u3", src="sin_decay",
                 fresh_per_iter=False, n_intervals=2, tol=1e-6)
    pb = O.Problem(wl)
    u0 = pb.ic_nodes(0)[None, :]
    _say("tolerance twice")
    with H.Plan(wl) as plan:
        assert plan.hpsmc_solve() == 0
        ref_rec = plan.hpsmc_stats()["max_eps"].copy()
        ref_U = [plan.hpsmc_get_nodes(iv) for iv in range(2)]
    with H.Plan(wl) as plan:
        plan.hpsmc_set_initial_nodes(4.0 * u0)
        plan.hpsmc_solve()
        big = plan.hpsmc_stats()["max_eps"].copy()
        plan.hpsmc_set_initial_nodes(u0)
        assert plan.hpsmc_solve() == 0
        rec = plan.hpsmc_stats()["max_eps"][:ref_rec.size]
        U = [plan.hpsmc_get_nodes(iv) for iv in range(2)]
    print("records: first", ref_rec[:4], "after the larger solve", big[:4], "again", rec[:4])
    assert np.max(big[:4]) > np.max(ref_rec[:4])
    # the stop iterations agree; values to rounding (the initial data come back
    # through the oracle's nodal values, equal to the plan's own to ~1e-17)
    assert np.array_equal(rec > 0, ref_rec > 0)
    assert np.max(np.abs(rec - ref_rec)) <= 1e-12 * np.max(ref_rec)
    for a, b in zip(U, ref_U):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    for iv in range(2):                      # each interval stopped below tol before its last iteration
        r = ref_rec[iv * wl.iters:(iv + 1) * wl.iters]
        last = np.flatnonzero(r > 0)[-1]
        assert r[last] < wl.tol and last < wl.iters - 1
