"""ctypes binding of libhpsmc.so (include/hpsmc.h): argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts
workload descriptions and NumPy / torch buffers into the C structures and
pointers the ABI takes.  The binding raises if the library is missing: there
is no CPU fallback.

PyTorch supplies device memory and streams: any ``stream`` argument may be a
``torch.cuda.Stream`` (or its raw ``cuda_stream`` handle), and the
``on_device`` copies accept CUDA tensors.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpsmc.so")

F_KINDS = {"affine": 0, "u_minus_u3": 1, "sin": 2, "u2_over_1pu2": 3, "neg_u3": 4, "u_sin_u": 5}
SRC_KINDS = {"none": 0, "sin_decay": 1, "cos_decay": 2, "longtime": 3, "quad": 4, "frac_longtime": 5,
             "frac_singular": 6, "frac_poly": 7, "poly": 8}
IC_KINDS = {"exact": 0, "singular": 1, "phi": 2, "nodal": 3}
SCHEDULES = {"sequential": 0, "sweeps": 1}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_then_fp64": 2}
ESTIMATORS = {"residual": 0, "picard": 1}
ACCELS = {"none": 0, "aitken": 1}
QUADS = {"centre": 0, "ball": 1}
NSTAR_MODES = {"array": 0, "dt": 1, "spectral": 2}
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOTSUP", -3: "ENOMEM", -4: "EDEVICE", -5: "EDIVERGED", -6: "ENOTCONVERGED"}
ENOTCONVERGED = -6


class HpsmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class hpsmc_problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32), ("n_intervals", C.c_int32), ("n_instances", C.c_int32),
        ("t_breaks", C.POINTER(C.c_double)), ("degree", C.POINTER(C.c_int32)), ("nstar", C.POINTER(C.c_int32)),
        ("f_kind", C.c_int32), ("src_kind", C.c_int32), ("ic_kind", C.c_int32), ("schedule", C.c_int32),
        ("f_param", C.c_double * 4), ("src_param", C.c_double * 8), ("ic_param", C.c_double * 4),
        ("ic_data", C.POINTER(C.c_double)),
        ("M", C.c_int64), ("iters", C.c_int32), ("fresh_per_iter", C.c_int32), ("seed", C.c_uint64),
        ("precision", C.c_int32), ("estimator", C.c_int32), ("tol", C.c_double),
        ("accel", C.c_int32), ("quad", C.c_int32), ("omega", C.c_double * 3), ("alpha", C.c_double),
        ("nstar_mode", C.c_int32), ("nstar_min", C.c_int32), ("nstar_c", C.c_double), ("dt_max", C.c_double),
        ("src_coeffs", C.POINTER(C.c_double)), ("src_len", C.c_int64), ("switch_tol", C.c_double),
    ]


class hpsmc_stats_t(C.Structure):
    _fields_ = [("path_steps", C.c_uint64), ("lane_steps", C.c_uint64), ("node_samples", C.c_uint64),
                ("n_records", C.c_int32), ("status_flags", C.c_int32), ("sample_launches", C.c_int32),
                ("recon_launches", C.c_int32), ("sample_ms", C.c_double), ("sampling_span_ms", C.c_double),
                ("recon_ms", C.c_double),
                ("slab_ms", C.c_double), ("advance_launches", C.c_int64), ("max_eps", C.c_double * 4096),
                ("adjoint_launches", C.c_int64), ("adjoint_ms", C.c_double)]


class hpsmc_launch(C.Structure):
    _fields_ = [("samples_per_lane", C.c_int32), ("waves_per_block", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("round_steps", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

# name: (restype, argtypes)
_SIGS = {
    "hpsmc_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, C.c_void_p]),
    "hpsmc_create": (C.c_int, [C.POINTER(hpsmc_problem), C.POINTER(C.c_void_p)]),
    "hpsmc_destroy": (None, [C.c_void_p]),
    "hpsmc_grid": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "hpsmc_resolve_nstar": (C.c_int, [C.POINTER(hpsmc_problem), C.c_void_p, C.c_void_p]),
    "hpsmc_get_nstar": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "hpsmc_solve": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hpsmc_start_interval": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "hpsmc_iterate": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "hpsmc_sweep": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "hpsmc_get_nodes": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
    "hpsmc_set_nodes": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
    "hpsmc_get_increment": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hpsmc_eval": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "hpsmc_eval_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_void_p]),
    "hpsmc_set_probe": (C.c_int, [C.c_void_p, C.c_int64]),
    "hpsmc_get_probe": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "hpsmc_set_launch": (C.c_int, [C.c_void_p, C.POINTER(hpsmc_launch)]),
    "hpsmc_get_launch": (C.c_int, [C.c_void_p, C.POINTER(hpsmc_launch)]),
    "hpsmc_tune": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_char_p, C.c_void_p]),
    "hpsmc_stats": (C.c_int, [C.c_void_p, C.POINTER(hpsmc_stats_t), C.c_void_p]),
    "hpsmc_reset_stats": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hpsmc_loss_grad_c0": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "hpsmc_set_initial_coeffs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "hpsmc_set_initial_nodes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "hpsmc_get_coeffs": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
    "hpsmc_set_option": (C.c_int, [C.c_void_p, C.c_char_p, C.c_int64]),
    "hpsmc_get_option": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int64)]),
    "hpsmc_last_error": (C.c_char_p, []),
}
EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """Load libhpsmc.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_22190_amd.build`")
        _lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _check(status, what):
    if status != 0:
        msg = lib().hpsmc_last_error().decode()
        raise HpsmcError(status, f"{what}: {msg}")


def _stream(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _is_device(a):
    return a is not None and hasattr(a, "data_ptr")


def _device_f64(t, count, what):
    """Check that a torch tensor handed over as a device buffer is a contiguous
    float64 GPU tensor of `count` elements (the library copies count * 8 bytes)."""
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what}: expected a GPU tensor (a host array is passed as a NumPy array)")
    import torch
    if t.dtype != torch.float64:
        raise ValueError(f"{what}: expected float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor")
    if t.numel() != count:
        raise ValueError(f"{what}: expected {count} elements, got {t.numel()}")
    return t


def make_problem(wl):
    """hpsmc_problem from a workload description; returns (struct, keep-alive list)."""
    tb = np.ascontiguousarray(wl.t_breaks, dtype=np.float64)
    deg = np.ascontiguousarray(wl.degree, dtype=np.int32)
    mode = NSTAR_MODES[getattr(wl, "nstar_mode", "array")]
    ns = np.ascontiguousarray(wl.nstar, dtype=np.int32) if mode == NSTAR_MODES["array"] else None
    sc = getattr(wl, "src_coeffs", None)
    sc = None if sc is None else np.ascontiguousarray(sc, dtype=np.float64).reshape(-1)
    ic = None if wl.ic_data is None else np.ascontiguousarray(wl.ic_data, dtype=np.float64).reshape(-1)
    p = hpsmc_problem()
    p.dim, p.n, p.n_intervals, p.n_instances = wl.dim, wl.n, len(wl.degree), wl.n_instances
    p.t_breaks = tb.ctypes.data_as(C.POINTER(C.c_double))
    p.degree = deg.ctypes.data_as(C.POINTER(C.c_int32))
    p.nstar = ns.ctypes.data_as(C.POINTER(C.c_int32)) if ns is not None else C.POINTER(C.c_int32)()
    p.nstar_mode = mode
    p.nstar_min = int(getattr(wl, "nstar_min", 0))
    p.nstar_c = float(getattr(wl, "nstar_c", 0.0))
    p.dt_max = float(getattr(wl, "dt_max", 0.0))
    p.src_coeffs = sc.ctypes.data_as(C.POINTER(C.c_double)) if sc is not None else C.POINTER(C.c_double)()
    p.src_len = 0 if sc is None else sc.size
    p.switch_tol = float(getattr(wl, "switch_tol", 0.0))
    p.f_kind, p.src_kind, p.ic_kind = F_KINDS[wl.f], SRC_KINDS[wl.src], IC_KINDS[wl.ic]
    p.schedule = SCHEDULES[wl.schedule]
    for i, v in enumerate(wl.f_param):
        p.f_param[i] = v
    for i, v in enumerate(wl.src_param):
        p.src_param[i] = v
    for i, v in enumerate(wl.ic_param):
        p.ic_param[i] = v
    p.ic_data = ic.ctypes.data_as(C.POINTER(C.c_double)) if ic is not None else C.POINTER(C.c_double)()
    p.M, p.iters, p.fresh_per_iter, p.seed = wl.M, wl.iters, int(wl.fresh_per_iter), wl.seed
    p.precision = PRECISIONS[wl.precision]
    p.tol = float(getattr(wl, "tol", 0.0))
    p.estimator = ESTIMATORS[getattr(wl, "estimator", "residual")]
    p.accel = ACCELS[getattr(wl, "accel", "none")]
    p.quad = QUADS[getattr(wl, "quad", "centre")]
    p.alpha = float(getattr(wl, "alpha", 2.0))
    for i, v in enumerate(getattr(wl, "omega", [0.0, 0.0, 0.0])):
        p.omega[i] = v
    return p, [tb, deg, ns, ic, sc]


def resolve_nstar(wl):
    """(N* per node time, Delta_max per interval) of a workload by the library's
    rule, without a plan or a device (hpsmc_resolve_nstar)."""
    p, keep = make_problem(wl)
    out = np.zeros(sum(wl.degree), dtype=np.int32)
    dt = np.zeros(len(wl.degree))
    _check(lib().hpsmc_resolve_nstar(C.byref(p), _ptr(out), _ptr(dt)), "hpsmc_resolve_nstar")
    return out, dt


# ------------------------------------------------------------ C-ABI mirrors
_alloc_hooks = None   # the ctypes callbacks must outlive every plan created with them


def hpsmc_set_allocator(alloc=None, free=None, ctx=None):
    """Install Python callables alloc(bytes, stream) -> int pointer and
    free(pointer, stream) as the device allocator of plans created afterwards;
    no arguments restores hipMalloc / hipFree."""
    global _alloc_hooks
    if alloc is None and free is None:
        _check(lib().hpsmc_set_allocator(ALLOC_FN(), FREE_FN(), None), "hpsmc_set_allocator")
        return
    a = ALLOC_FN(lambda nbytes, stream, c: int(alloc(int(nbytes), stream)) or None)
    f = FREE_FN(lambda ptr, stream, c: free(int(ptr), stream))
    _check(lib().hpsmc_set_allocator(a, f, ctx), "hpsmc_set_allocator")
    _alloc_hooks = (a, f, alloc, free) if _alloc_hooks is None else _alloc_hooks + (a, f, alloc, free)


def torch_caching_allocator():
    """alloc / free callables backed by PyTorch's CUDA caching allocator."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)
    return alloc, free


def hpsmc_create(wl):
    p, keep = make_problem(wl)
    h = C.c_void_p()
    _check(lib().hpsmc_create(C.byref(p), C.byref(h)), "hpsmc_create")
    return h


def hpsmc_destroy(h):
    lib().hpsmc_destroy(h)


class Plan:
    """Owns one hpsmc_plan; methods mirror the C entry points by name."""

    def __init__(self, wl):
        self.wl = wl
        self.h = hpsmc_create(wl)
        self.nsp = wl.n ** wl.dim

    def close(self):
        if self.h:
            hpsmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- grid and driving
    def hpsmc_grid(self, iv=0):
        x = np.zeros(self.wl.n)
        t = np.zeros(self.wl.degree[iv] + 1)
        _check(lib().hpsmc_grid(self.h, iv, _ptr(x), _ptr(t)), "hpsmc_grid")
        return x, t

    def hpsmc_get_nstar(self):
        out = np.zeros(sum(self.wl.degree), dtype=np.int32)
        dt = np.zeros(len(self.wl.degree))
        _check(lib().hpsmc_get_nstar(self.h, _ptr(out), _ptr(dt)), "hpsmc_get_nstar")
        return out, dt

    def hpsmc_solve(self, stream=None):
        """Returns the status: OK, or ENOTCONVERGED (informational) in tolerance mode."""
        st = lib().hpsmc_solve(self.h, _stream(stream))
        if st != ENOTCONVERGED:
            _check(st, "hpsmc_solve")
        return st

    def hpsmc_start_interval(self, iv, stream=None):
        _check(lib().hpsmc_start_interval(self.h, iv, _stream(stream)), "hpsmc_start_interval")

    def hpsmc_iterate(self, iv, tag, stream=None):
        _check(lib().hpsmc_iterate(self.h, iv, tag, _stream(stream)), "hpsmc_iterate")

    def hpsmc_sweep(self, tag, stream=None):
        _check(lib().hpsmc_sweep(self.h, tag, _stream(stream)), "hpsmc_sweep")

    # -- data in / out
    def _nodes_shape(self, iv):
        return (self.wl.n_instances, self.nsp, self.wl.degree[iv] + 1)

    def hpsmc_get_nodes(self, iv, out=None, stream=None):
        on_dev = _is_device(out)
        if on_dev:
            _device_f64(out, int(np.prod(self._nodes_shape(iv))), "hpsmc_get_nodes out")
        if out is None:
            out = np.zeros(self._nodes_shape(iv))
        _check(lib().hpsmc_get_nodes(self.h, iv, _ptr(out), int(on_dev), _stream(stream)), "hpsmc_get_nodes")
        return out

    def hpsmc_set_nodes(self, iv, values, stream=None):
        on_dev = _is_device(values)
        if on_dev:
            _device_f64(values, int(np.prod(self._nodes_shape(iv))), "hpsmc_set_nodes values")
        else:
            values = np.ascontiguousarray(values, dtype=np.float64).reshape(self._nodes_shape(iv))
        _check(lib().hpsmc_set_nodes(self.h, iv, _ptr(values), int(on_dev), _stream(stream)), "hpsmc_set_nodes")

    def hpsmc_set_initial_nodes(self, u0, stream=None):
        on_dev = _is_device(u0)
        if on_dev:
            _device_f64(u0, self.wl.n_instances * self.nsp, "hpsmc_set_initial_nodes u0")
        else:
            u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(self.wl.n_instances, self.nsp)
        _check(lib().hpsmc_set_initial_nodes(self.h, _ptr(u0), int(on_dev), _stream(stream)), "hpsmc_set_initial_nodes")

    def hpsmc_get_coeffs(self, iv, out=None, stream=None):
        on_dev = _is_device(out)
        if on_dev:
            _device_f64(out, int(np.prod(self._nodes_shape(iv))), "hpsmc_get_coeffs out")
        if out is None:
            out = np.zeros(self._nodes_shape(iv))
        _check(lib().hpsmc_get_coeffs(self.h, iv, _ptr(out), int(on_dev), _stream(stream)), "hpsmc_get_coeffs")
        return out

    def hpsmc_get_increment(self, iv, stream=None):
        cnt = (self.wl.n_instances, self.nsp * self.wl.degree[iv])
        eps, ssq = np.zeros(cnt), np.zeros(cnt)
        _check(lib().hpsmc_get_increment(self.h, iv, _ptr(eps), _ptr(ssq), _stream(stream)), "hpsmc_get_increment")
        return eps, ssq

    def hpsmc_eval(self, iv, inst, pts, stream=None):
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, self.wl.dim + 1)
        out = np.zeros((pts.shape[0], 2))
        _check(lib().hpsmc_eval(self.h, iv, inst, _ptr(pts), pts.shape[0], _ptr(out), _stream(stream)), "hpsmc_eval")
        return out

    def hpsmc_eval_noalloc(self, iv, inst, pts, stream=None):
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, self.wl.dim + 1)
        out = np.zeros((pts.shape[0], 2))
        _check(lib().hpsmc_eval_noalloc(self.h, iv, inst, _ptr(pts), pts.shape[0], _ptr(out), _stream(stream)),
               "hpsmc_eval_noalloc")
        return out

    def hpsmc_set_probe(self, m_probe):
        _check(lib().hpsmc_set_probe(self.h, int(m_probe)), "hpsmc_set_probe")
        self.m_probe = int(m_probe)

    def hpsmc_get_probe(self, iv, stream=None):
        out = np.zeros((self.wl.n_instances, self.nsp * self.wl.degree[iv], self.m_probe))
        _check(lib().hpsmc_get_probe(self.h, iv, _ptr(out), _stream(stream)), "hpsmc_get_probe")
        return out

    # -- launch shape and tuning
    def hpsmc_set_launch(self, samples_per_lane, waves_per_block, blocks_per_cu, round_steps=0):
        l = hpsmc_launch(samples_per_lane, waves_per_block, blocks_per_cu, round_steps)
        _check(lib().hpsmc_set_launch(self.h, C.byref(l)), "hpsmc_set_launch")

    def hpsmc_get_launch(self):
        l = hpsmc_launch()
        _check(lib().hpsmc_get_launch(self.h, C.byref(l)), "hpsmc_get_launch")
        return (l.samples_per_lane, l.waves_per_block, l.blocks_per_cu, l.round_steps)

    def hpsmc_tune(self, iv=0, m_tune=0, cache_path=None, stream=None):
        cp = cache_path.encode() if cache_path else None
        _check(lib().hpsmc_tune(self.h, iv, int(m_tune), cp, _stream(stream)), "hpsmc_tune")
        return self.hpsmc_get_launch()

    # -- counters
    def hpsmc_stats(self, stream=None):
        s = hpsmc_stats_t()
        _check(lib().hpsmc_stats(self.h, C.byref(s), _stream(stream)), "hpsmc_stats")
        return {"path_steps": s.path_steps, "lane_steps": s.lane_steps, "node_samples": s.node_samples,
                "max_eps": np.array(s.max_eps[:s.n_records]), "n_records": s.n_records,
                "status_flags": s.status_flags,
                "sample_launches": s.sample_launches, "recon_launches": s.recon_launches,
                "sample_ms": s.sample_ms, "sampling_span_ms": s.sampling_span_ms, "recon_ms": s.recon_ms,
                "slab_ms": s.slab_ms,
                "advance_launches": s.advance_launches,
                "adjoint_launches": s.adjoint_launches, "adjoint_ms": s.adjoint_ms}

    def hpsmc_reset_stats(self, stream=None):
        _check(lib().hpsmc_reset_stats(self.h, _stream(stream)), "hpsmc_reset_stats")

    def hpsmc_set_option(self, name, value):
        _check(lib().hpsmc_set_option(self.h, name.encode(), int(value)), "hpsmc_set_option")

    def hpsmc_get_option(self, name):
        v = C.c_int64(0)
        _check(lib().hpsmc_get_option(self.h, name.encode(), C.byref(v)), "hpsmc_get_option")
        return int(v.value)

    # -- gradient
    def hpsmc_set_initial_coeffs(self, c0, stream=None):
        on_dev = _is_device(c0)
        if on_dev:
            _device_f64(c0, self.wl.n_instances * self.nsp, "hpsmc_set_initial_coeffs c0")
        else:
            c0 = np.ascontiguousarray(c0, dtype=np.float64).reshape(self.wl.n_instances, self.nsp)
        _check(lib().hpsmc_set_initial_coeffs(self.h, _ptr(c0), int(on_dev), _stream(stream)),
               "hpsmc_set_initial_coeffs")

    def hpsmc_loss_grad_c0(self, target, stream=None):
        on_dev = _is_device(target)
        I = self.wl.n_instances
        if on_dev:
            _device_f64(target, I * self.nsp, "hpsmc_loss_grad_c0 target")
            import torch
            loss = torch.zeros(I, dtype=torch.float64, device=target.device)
            grad = torch.zeros((I, self.nsp), dtype=torch.float64, device=target.device)
        else:
            target = np.ascontiguousarray(target, dtype=np.float64).reshape(I, self.nsp)
            loss, grad = np.zeros(I), np.zeros((I, self.nsp))
        _check(lib().hpsmc_loss_grad_c0(self.h, _ptr(target), _ptr(loss), _ptr(grad), int(on_dev),
                                        _stream(stream)), "hpsmc_loss_grad_c0")
        return loss, grad


def smc_loss_function():
    """torch.autograd.Function whose forward is the terminal misfit of a
    single-interval solve from phi-coefficients c0 ([instances, n^d], float64,
    on the GPU) and whose backward is the library's hand-written adjoint under
    common random numbers (the gradient is computed with the forward)."""
    import torch

    class SMCLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, c0, plan, target, stream=None):
            # the library reads float64 device buffers; other dtypes are converted
            c0 = c0.detach().to(torch.float64).contiguous()
            plan.hpsmc_set_initial_coeffs(c0, stream=stream)
            loss, grad = plan.hpsmc_loss_grad_c0(target.detach().to(c0.device, torch.float64).contiguous(),
                                                 stream=stream)
            ctx.save_for_backward(grad)
            return loss

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            return gout[:, None] * grad, None, None, None

    return SMCLoss
