"""Parity at the full size of the 2-D long-time workload, in the launch shape
the benchmark times (the autotuner's cached entry for this plan shape).

One residual iteration of interval 1: 24 x 24 Jacobi-Gauss nodes x 16 Lobatto
times (9216 Monte Carlo nodes), N* up to ~92k walk steps, the sample slice of
1024 samples per node.  The oracle cannot redo the whole iteration, so:

* every node: the increment equals the mean of its 1024 per-sample path values
  (read back through the probe) and the iterate moved by exactly that increment
  (properties that hold at any size);
* sampled (node, sample) pairs, chosen by a fixed seed over all node times:
  the path value against the oracle's own walk of the same Philox counter --
  FP64 to 1e-12 relative; FP32 (matrix-core kernel) to the FP32 bound below.
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
M_SLICE = 1024


def _say(*a):
    print("[case]", *a, flush=True)


def _exact_nodes(wl, pb):
    x, t = pb.grid(0)
    U = np.zeros((1, wl.nsp, wl.degree[0] + 1))
    for jf in range(wl.nsp):
        X = [x[i] for i in np.unravel_index(jf, (wl.n,) * wl.dim)]
        for l in range(len(t)):
            U[0, jf, l] = pb.exact(X, t[l])
    return U


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_long_time_iteration(precision, tmp_path):
    from paper_2608_22190_amd import hpsmc as H
    wl = W.c2_long_time(M=M_SLICE, iters=1, n_intervals=1, precision=precision)
    pb = O.Problem(wl)
    U0 = _exact_nodes(wl, pb)
    cache = str(tmp_path / "tuned.json")
    if os.path.exists(CACHE):
        shutil.copy(CACHE, cache)
    with H.Plan(wl) as plan:
        launch = plan.hpsmc_tune(0, 4, cache)
        _say("full size", precision, launch, "mma", plan.hpsmc_get_option("sample_mfma_active"))
        plan.hpsmc_set_probe(M_SLICE)
        plan.hpsmc_set_nodes(0, U0)
        plan.hpsmc_iterate(0, 0)
        probe = plan.hpsmc_get_probe(0)[0]
        eps, _ = plan.hpsmc_get_increment(0)
        U1 = plan.hpsmc_get_nodes(0)
    nodes = wl.nsp * wl.degree[0]
    assert probe.shape == (nodes, M_SLICE) and np.all(np.isfinite(probe))
    # increment = sample mean, iterate moved by it (columns l >= 1; column 0 is the initial data)
    mean = probe.mean(axis=1)
    assert np.max(np.abs(eps[0] - mean)) <= 1e-13 * (1 + np.max(np.abs(probe)))
    moved = (U1[0] - U0[0])[:, 1:].T.reshape(-1)     # node j + nsp (l - 1), as the Philox word c0
    assert np.max(np.abs(moved - eps[0])) <= 1e-14 * (1 + np.max(np.abs(U0)))
    assert np.array_equal(U1[0][:, 0], U0[0][:, 0])
    # sampled paths against the oracle's walk
    Ut = O.reconstruct(2, wl.n, wl.degree[0], U0[0].reshape(-1))
    rng = np.random.default_rng(2608)
    picks = [(int(rng.integers(nodes)), int(rng.integers(M_SLICE))) for _ in range(10)]
    worst = 0.0
    for node, smp in picks:
        S, steps = pb.sample_path(Ut, 0, 0, 0, node, smp)
        err = abs(probe[node, smp] - S)
        worst = max(worst, err / (1 + abs(S)))
        print(f"node {node} sample {smp}: S={S:.9f} steps={steps} |diff|={err:.3e}", flush=True)
        if precision == "fp64":
            assert err <= 1e-12 * (1 + abs(S))
        else:
            # FP32 walk and contraction: the walk's rounding moves the point by
            # ~sqrt(L) * 2^-24 and may change the exit step near the boundary
            # (one step changes S by Delta |r|); the contraction adds FP32
            # rounding of ~P^2 products per step.  Both stay far below 1e-3.
            assert err <= 1e-3 * (1 + abs(S))
    print(f"worst relative path error ({precision}): {worst:.3e}")
