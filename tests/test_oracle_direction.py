"""Pin of the oracle's jump-direction law in d = 3, 4, 5 (Lemma 2.1: the jump
direction is uniform on the unit sphere S^{d-1}; reading R9 samples it as a
normalized vector of Box-Muller normals).

The checker below tests what the uniform law on S^{d-1} fixes, independently
of how it is sampled:
  - |theta| = 1;
  - mean 0 and second moments E[theta theta^T] = I/d;
  - fourth moments E[theta_i^4] = 3/(d(d+2)), E[theta_i^2 theta_j^2] = 1/(d(d+2));
  - every coordinate, and the projection on a fixed random axis, has the
    marginal density proportional to (1 - t^2)^{(d-3)/2}, i.e.
    (t + 1)/2 ~ Beta((d-1)/2, (d-1)/2) (uniform on [-1, 1] for d = 3);
  - consecutive steps of a walk are uncorrelated.
It is shown to reject plausible sampler mistakes: a normalized uniform-cube
vector, a Box-Muller pair that reuses the cosine, one word for both radius
and angle, a radius without its square root, and the fifth normal taken from
an already used pair.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O

N_WALKS, N_STEPS = 400, 300          # 120,000 directions per dimension


def sphere_law_failures(th, d, n_steps=None):
    """Names of the checks the sample `th` [N][d] fails (empty: consistent
    with the uniform law on S^{d-1})."""
    fails = []
    N = th.shape[0]
    if np.max(np.abs(np.linalg.norm(th, axis=1) - 1.0)) > 1e-13:
        fails.append("norm")
    # first moments: Var(theta_i) = 1/d
    if np.max(np.abs(th.mean(axis=0))) > 4.5 * np.sqrt(1.0 / (d * N)):
        fails.append("mean")
    # second moments E[theta_i theta_j] = delta_ij / d
    m4 = 3.0 / (d * (d + 2.0))
    m22 = 1.0 / (d * (d + 2.0))
    m8 = 105.0 / (d * (d + 2.0) * (d + 4.0) * (d + 6.0))
    m44 = 9.0 / (d * (d + 2.0) * (d + 4.0) * (d + 6.0))
    C2 = th.T @ th / N
    for i in range(d):
        for j in range(i, d):
            if i == j:
                sd = np.sqrt((m4 - 1.0 / d**2) / N)
                dev = C2[i, i] - 1.0 / d
            else:
                sd = np.sqrt(m22 / N)
                dev = C2[i, j]
            if abs(dev) > 5.0 * sd:
                fails.append(f"cov[{i},{j}]")
    # fourth moments
    t2 = th * th
    for i in range(d):
        if abs(np.mean(t2[:, i] ** 2) - m4) > 5.0 * np.sqrt((m8 - m4**2) / N):
            fails.append(f"m4[{i}]")
        for j in range(i + 1, d):
            if abs(np.mean(t2[:, i] * t2[:, j]) - m22) > 5.0 * np.sqrt((m44 - m22**2) / N):
                fails.append(f"m22[{i},{j}]")
    # marginals: (t+1)/2 ~ Beta((d-1)/2, (d-1)/2), per coordinate and on a fixed axis
    a = (d - 1) / 2.0
    axis = np.random.default_rng(12345).standard_normal(d)
    axis /= np.linalg.norm(axis)
    cols = [th[:, i] for i in range(d)] + [th @ axis]
    for k, c in enumerate(cols):
        p = stats.kstest((c + 1.0) / 2.0, stats.beta(a, a).cdf).pvalue
        if p < 1e-5:
            fails.append(f"marginal[{k}]")
    # consecutive steps of one walk are independent
    if n_steps:
        w = th.reshape(-1, n_steps, d)
        lag = np.einsum("wsi,wsi->i", w[:, :-1], w[:, 1:]) / (w.shape[0] * (n_steps - 1))
        if np.max(np.abs(lag)) > 4.5 * np.sqrt(1.0 / (d * d * w.shape[0] * (n_steps - 1))):
            fails.append("lag1")
    return fails


def oracle_directions(d, seed=0):
    out = [O.walk_directions(d, seed, node=7 + 3 * w, sample=w, q0=0, nq=N_STEPS, inst=1, interval=2,
                             iter_tag=3) for w in range(N_WALKS)]
    return np.concatenate(out, axis=0)


@pytest.mark.parametrize("d", [3, 4, 5])
def test_oracle_directions_uniform_on_sphere(d):
    th = oracle_directions(d)
    assert th.shape == (N_WALKS * N_STEPS, d)
    fails = sphere_law_failures(th, d, N_STEPS)
    assert not fails, fails


@pytest.mark.parametrize("d", [3, 4, 5])
def test_oracle_directions_match_path_counters(d):
    # the exported sampler is the walk's: a different stream position, node,
    # sample or tag gives different words; the same position the same vector
    a = O.walk_directions(d, 5, node=11, sample=2, q0=0, nq=40, inst=0, interval=1, iter_tag=4)
    b = O.walk_directions(d, 5, node=11, sample=2, q0=13, nq=10, inst=0, interval=1, iter_tag=4)
    assert np.array_equal(a[13:23], b)
    for kw in (dict(node=12), dict(sample=3), dict(iter_tag=5), dict(interval=2)):
        args = dict(node=11, sample=2, interval=1, iter_tag=4)
        args.update(kw)
        c = O.walk_directions(d, 5, q0=0, nq=40, inst=0, **args)
        assert not np.allclose(a, c)


def _box_muller(u1, u2):
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)


def _mutant(kind, d, N, rng):
    npairs = (d + 1) // 2
    u = rng.random((N, 2 * npairs))
    g = np.zeros((N, 2 * npairs))
    for k in range(npairs):
        u1, u2 = u[:, 2 * k], u[:, 2 * k + 1]
        if kind == "cube":
            g[:, 2 * k] = 2 * u1 - 1
            g[:, 2 * k + 1] = 2 * u2 - 1
        elif kind == "cos_twice":
            c, _ = _box_muller(u1, u2)
            g[:, 2 * k], g[:, 2 * k + 1] = c, c
        elif kind == "one_word":
            g[:, 2 * k], g[:, 2 * k + 1] = _box_muller(u1, u1)
        elif kind == "no_sqrt":
            r = -2.0 * np.log(u1)
            g[:, 2 * k], g[:, 2 * k + 1] = r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)
        elif kind == "reused_pair":
            g[:, 2 * k], g[:, 2 * k + 1] = _box_muller(u1, u2)
        else:
            raise ValueError(kind)
    if kind == "reused_pair":   # the last normal from the first pair again
        g[:, d - 1] = g[:, 0]
    g = g[:, :d]
    return g / np.linalg.norm(g, axis=1, keepdims=True)


@pytest.mark.parametrize("d", [3, 4, 5])
@pytest.mark.parametrize("kind", ["cube", "cos_twice", "one_word", "no_sqrt", "reused_pair"])
def test_checker_rejects_wrong_samplers(d, kind):
    th = _mutant(kind, d, N_WALKS * N_STEPS, np.random.default_rng(d))
    assert sphere_law_failures(th, d), f"{kind} passed as uniform on S^{d - 1}"


@pytest.mark.parametrize("d", [3, 4, 5])
def test_checker_accepts_exact_law(d):
    # the checker's own control: normalized N(0, I) normals from another generator
    g = np.random.default_rng(100 + d).standard_normal((N_WALKS * N_STEPS, d))
    th = g / np.linalg.norm(g, axis=1, keepdims=True)
    assert not sphere_law_failures(th, d, N_STEPS)
