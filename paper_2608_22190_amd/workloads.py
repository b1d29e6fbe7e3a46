"""Seeded synthetic workloads (inputs only).

This module describes problems: sizes, time partitions, degrees, the
nonlinearity / source / initial-data choices by name, sample counts, seeds, and
the per-node path length N*.  It holds none of the method's arithmetic (no
quadrature, no transforms, no sampling); both the GPU binding and the CPU oracle
read these descriptions.  Random inputs the method consumes (the initial
Legendre-type coefficients of the batched-gradient workload, loss targets) are
drawn here with NumPy's seeded generator and passed in as data.

Workload shapes follow the paper's experiments: the single-step accuracy test
(Ex. 1), the long-time run (Ex. 2, here with the Laplacian, alpha = 2, in 2-D),
the initial singularity with a geometric mesh and linearly increasing degrees
(Ex. 3), the five-dimensional problem (Ex. 4), and a batched-gradient set.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np


@dataclass
class Workload:
    name: str
    dim: int
    n: int                      # Jacobi-Gauss (1,1) points per dimension
    t_breaks: List[float]       # time mesh t_0 < ... < t_Nh
    degree: List[int]           # temporal degree M_n per interval
    nstar: Optional[List[int]] = None   # explicit N* per (interval, ell = 1..M_n), concatenated
    f: str = "u_minus_u3"
    f_param: List[float] = field(default_factory=lambda: [0.0, 0.0, 0.0, 0.0])
    src: str = "none"
    src_param: List[float] = field(default_factory=lambda: [0.0] * 8)
    ic: str = "exact"
    ic_param: List[float] = field(default_factory=lambda: [0.0] * 4)
    ic_data: Optional[np.ndarray] = None   # [instance][n^d]
    M: int = 64
    iters: int = 2
    seed: int = 0
    schedule: str = "sequential"
    n_instances: int = 1
    fresh_per_iter: bool = True
    precision: str = "fp64"     # "fp64", "fp32" (path sampling precision), or "fp32_then_fp64" (FP32
                                # until max|eps| < switch_tol, then FP64)
    switch_tol: float = 0.0
    exact_known: bool = True
    tol: float = 0.0            # > 0: stop an interval once max|eps| < tol (Algorithm 1's loop condition)
    estimator: str = "residual" # "residual" (eq. varepsilon_1) or "picard" (eq. uast, classical MC form)
    accel: str = "none"         # "none" or "aitken" (relaxed iteration, remark after Algorithm 1)
    quad: str = "centre"        # path quadrature: "centre" (eq. interIQ) or "ball" (Green's-function ball point)
    alpha: float = 2.0          # order of the operator: 2 the Laplacian, (0, 2) the fractional Laplacian (d = 1)
    omega: List[float] = field(default_factory=lambda: [0.0, 0.0, 0.0])  # Aitken w0, w_min, w_max (0: default)
    # path lengths (eq. time division): "array" takes `nstar`; the rules give
    # N* = max(nstar_min, ceil((t_{n,l} - t_{n-1}) / Delta_max)) with Delta_max =
    # nstar_c / rho(A_h) per interval ("spectral", rho the spectral radius of the
    # interval's discrete operator, computed by the library at set-up) or dt_max ("dt")
    nstar_mode: str = "spectral"
    nstar_c: float = 0.25
    nstar_min: int = 4
    dt_max: float = 0.0
    src_coeffs: Optional[np.ndarray] = None   # "poly" source: per interval [k_0..k_{d-1}][q], concatenated

    @property
    def n_intervals(self):
        return len(self.degree)

    @property
    def nsp(self):
        return self.n ** self.dim

    @property
    def nodes_per_sweep(self):
        return self.nsp * sum(self.degree)

    def with_(self, **kw):
        return replace(self, **kw)


def fixed_nstar(degree, value):
    return [int(value)] * sum(degree)


def _mk(name, dim, n, t_breaks, degree, c=0.25, nmin=4, **kw):
    """A workload whose path lengths follow the spectral rule with Delta_max = c / rho."""
    return Workload(name=name, dim=dim, n=n, t_breaks=list(t_breaks), degree=list(degree),
                    nstar_mode="spectral", nstar_c=c, nstar_min=nmin, **kw)


# --------------------------------------------------------------------------
# The five workload shapes.
# --------------------------------------------------------------------------
def c1_single_step(M=4096, iters=5, **kw):
    """1-D u_t = u_xx + u - u^3 + s, u = e^{-t} sin(pi x), one interval [0,1],
    16 spatial x 16 temporal nodes, FP64."""
    return _mk("c1_1d_single_step", 1, 16, [0.0, 1.0], [16], f="u_minus_u3", src="sin_decay",
               ic="exact", M=M, iters=iters, seed=0, precision="fp64", **kw)


def c2_long_time(M=65536, iters=6, n_intervals=10, precision="fp32", **kw):
    """2-D u_t = Lap u + sin u + s on [-1,1]^2 to T = 10 with ten unit steps,
    24x24 spatial x 16 temporal nodes per step; exact solution
    prod(1-x_i^2) sin(x+y) e^{cos t}/(1+t^2)."""
    tb = [float(k) for k in range(n_intervals + 1)]
    return _mk("c2_2d_long_time", 2, 24, tb, [16] * n_intervals, f="sin", src="longtime",
               ic="exact", M=M, iters=iters, seed=0, precision=precision, **kw)


def c3_initial_singularity(M=32768, sweeps=None, precision="fp32", **kw):
    """2-D u_t = Lap u + u^2/(1+u^2) with u0 = (1-x^2)(1-y^2)|x|^{1/2}, T = 1,
    geometric mesh t_n = 0.2^{12-n}, degrees M_n = 2n+2 (4..26), 20x20 nodes,
    all intervals swept together."""
    N = 12
    tb = [0.0] + [0.2 ** (N - k) for k in range(1, N + 1)]
    deg = [2 * k + 2 for k in range(1, N + 1)]
    sweeps = N + 6 - 1 if sweeps is None else sweeps
    return _mk("c3_2d_initial_singularity", 2, 20, tb, deg, f="u2_over_1pu2", src="none",
               ic="singular", ic_param=[0.5, 0, 0, 0], M=M, iters=sweeps, seed=0,
               schedule="sweeps", precision=precision, exact_known=False, **kw)


def c4_five_dim(M=16384, iters=4, **kw):
    """5-D u_t = Lap u - u^3 + s, u = e^{-t} prod cos(pi x_i/2), 8^5 spatial x
    8 temporal nodes, FP32 sampling with FP64 reconstruction."""
    return _mk("c4_5d", 5, 8, [0.0, 1.0], [8], f="neg_u3", src="cos_decay", ic="exact",
               M=M, iters=iters, seed=0, precision="fp32", **kw)


def c5_coefficients(n_instances, n=16, seed=0):
    """phi x phi coefficients c[k1,k2] ~ N(0, 1/(1+k1+k2)^2), one set per instance."""
    rng = np.random.default_rng(seed)
    k = np.arange(n)
    sd = 1.0 / (1.0 + k[:, None] + k[None, :])
    return rng.standard_normal((n_instances, n, n)) * sd[None]


def c5_batched_gradient(n_instances=256, M=8192, iters=6, n=16, **kw):
    """256 2-D instances of the long-time equation on [0, 0.5], 16x16 spatial
    x 12 temporal nodes, initial data from random phi-coefficients."""
    c0 = c5_coefficients(n_instances, n=n, seed=0).reshape(n_instances, -1)
    return _mk("c5_2d_batched_gradient", 2, n, [0.0, 0.5], [12], f="sin", src="longtime",
               ic="phi", ic_data=c0, M=M, iters=iters, seed=0, n_instances=n_instances,
               precision="fp32", exact_known=False, **kw)


def c5_target(n_instances, nsp, seed=1, scale=0.1):
    """misfit target at the final time, one nodal vector per instance"""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_instances, nsp)) * scale


def frac_long_time(M=8192, iters=6, n_intervals=20, h=0.5, n=11, deg=6, alpha=0.4, precision="fp64", **kw):
    """1-D fractional Allen-Cahn u_t = -(-Delta)^{alpha/2} u + u - u^3 + s on
    (-1,1), u = 0 outside, exact solution (1-x^2)_+^{alpha/2} sin x
    e^{cos t}/(1+t^2) (Ex. 2: alpha = 0.4, M_n = 6, N_x = 10), unit-free
    intervals of length h to T = n_intervals h."""
    tb = [h * k for k in range(n_intervals + 1)]
    return _mk("frac_long_time", 1, n, tb, [deg] * n_intervals, f="u_minus_u3", src="frac_longtime",
               ic="exact", M=M, iters=iters, seed=0, precision=precision, alpha=alpha, **kw)


def frac_singular(M=8192, iters=6, N=8, T=0.5, n=11, alpha=0.4, rho=0.51, precision="fp64", **kw):
    """Ex. 3: exact solution (1-x^2)_+^{alpha/2} cos(x^3+1)/(10x^2+1) t^rho with a
    weak singularity at t = 0, geometric mesh t_n = T 0.2^{N-n}, degrees
    M_1 = 1, M_n = max(1, floor(1.5 n))."""
    tb = [0.0] + [T * 0.2 ** (N - k) for k in range(1, N + 1)]
    deg = [1] + [max(1, int(math.floor(1.5 * k))) for k in range(2, N + 1)]
    return _mk("frac_singular", 1, n, tb, deg, f="u_minus_u3", src="frac_singular",
               src_param=[rho, 0, 0, 0, 0, 0, 0, 0], ic="exact", M=M, iters=iters, seed=0, precision=precision,
               alpha=alpha, **kw)


CONFIGS = {
    "c1": c1_single_step,
    "c2": c2_long_time,
    "c3": c3_initial_singularity,
    "c4": c4_five_dim,
    "c5": c5_batched_gradient,
}


# --------------------------------------------------------------------------
# Small problems for parity tests (several tiles, ragged tails, all dims).
# --------------------------------------------------------------------------
def small(dim=1, n=6, M_deg=4, M=64, iters=2, f="u_minus_u3", src="sin_decay", ic="exact",
          T=0.5, n_intervals=1, c=0.25, nmin=4, nstar=None, **kw):
    tb = [T * k / n_intervals for k in range(n_intervals + 1)]
    deg = [M_deg] * n_intervals if np.isscalar(M_deg) else list(M_deg)
    wl = _mk(f"small_d{dim}_n{n}", dim, n, tb, deg, c=c, nmin=nmin, f=f, src=src, ic=ic,
             M=M, iters=iters, **kw)
    if nstar is not None:
        wl = wl.with_(nstar=fixed_nstar(deg, nstar), nstar_mode="array")
    return wl
