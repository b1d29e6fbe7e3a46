"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/hpsmc.h, and rejects invalid problems before any device
call."""
import os
import re

import pytest

from paper_2608_22190_amd import hpsmc as H
from paper_2608_22190_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hpsmc.h")).read()
    return sorted(set(re.findall(r"(?:hpsmc_status|void|const char \*)\s*(hpsmc_[a-z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert sorted(H.EXPORTED) == _declared()


def test_library_exports_every_declared_symbol():
    lib = H.lib()
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("change,status", [
    (dict(dim=0), -1), (dict(dim=6), -1), (dict(n=0), -1), (dict(n=33), -1), (dict(M=0), -1),
    (dict(iters=0), -1), (dict(iters=256), -1), (dict(t_breaks=[0.0, 0.0]), -1),
    (dict(t_breaks=[0.0, float("nan")]), -1), (dict(degree=[0]), -1), (dict(degree=[32]), -1),
    (dict(f="affine", seed=1, nstar=[0, 3, 3, 3], nstar_mode="array"), -1),
    (dict(nstar=[1 << 24] * 4, nstar_mode="array"), -1), (dict(nstar_c=1e-9), -1), (dict(nstar_mode="dt"), -1),
    (dict(src="none", ic="exact"), -1), (dict(n_instances=0), -1), (dict(n_instances=65536), -1),
    (dict(dim=5, n=11), -2), (dict(dim=4, n=19), -2)])
def test_invalid_problems_are_rejected_before_device_work(change, status):
    wl = W.small(dim=1, n=4, M_deg=4).with_(**change)
    with pytest.raises(H.HpsmcError) as ei:
        H.Plan(wl)
    assert ei.value.status == status


def test_missing_ic_data_is_rejected():
    wl = W.small(dim=2, n=3, ic="phi")
    with pytest.raises(H.HpsmcError) as ei:
        H.Plan(wl)
    assert ei.value.status == -1


@pytest.mark.parametrize("tol", [-1e-3, float("nan"), float("inf")])
def test_invalid_tolerance_is_rejected(tol):
    wl = W.small(dim=1, n=4, M_deg=4).with_(tol=tol)
    with pytest.raises(H.HpsmcError) as ei:
        H.Plan(wl)
    assert ei.value.status == -1


@pytest.mark.parametrize("omega", [[3.0, 0, 0], [0.3, 0, 0], [1.0, -1.0, 2.0], [float("nan"), 0, 0],
                                   [1.0, 1.5, 1.2], [1.0, 0.5, float("inf")]])
def test_invalid_aitken_weights_are_rejected(omega):
    wl = W.small(dim=1, n=4, M_deg=4).with_(accel="aitken", omega=omega)
    with pytest.raises(H.HpsmcError) as ei:
        H.Plan(wl)
    assert ei.value.status == -1


@pytest.mark.parametrize("change,status", [
    (dict(src="frac_longtime", alpha=2.0), -1), (dict(src="sin_decay", alpha=0.5), -1),
    (dict(src="frac_longtime", alpha=0.5, dim=2, n=3), -2), (dict(src="frac_longtime", alpha=0.5, quad="ball"), -2),
    (dict(src="frac_longtime", alpha=-1.0), -1),
    (dict(src="frac_longtime", alpha=2.5), -1), (dict(src="frac_longtime", alpha=float("nan")), -1),
    (dict(src="frac_longtime", alpha=0.5, ic="phi", ic_data=__import__("numpy").zeros((1, 4))), -2)])
def test_invalid_fractional_problems_are_rejected(change, status):
    wl = W.small(dim=1, n=4, M_deg=4, f="u_minus_u3").with_(**change)
    with pytest.raises(H.HpsmcError) as ei:
        H.Plan(wl)
    assert ei.value.status == status


def test_allocator_hooks_must_come_in_pairs():
    lib = H.lib()
    a = H.ALLOC_FN(lambda n, s, c: None)
    assert lib.hpsmc_set_allocator(a, H.FREE_FN(), None) == -1
    assert lib.hpsmc_set_allocator(H.ALLOC_FN(), H.FREE_FN(), None) == 0


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof / offsetof of the ABI structs from a C compiler against the ctypes mirrors."""
    import ctypes as C
    import subprocess
    structs = {"hpsmc_problem": H.hpsmc_problem, "hpsmc_stats_t": H.hpsmc_stats_t, "hpsmc_launch": H.hpsmc_launch}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hpsmc.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)]).decode().split("\n") if l)
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, (name, f[0])


@pytest.mark.parametrize("change,status", [
    (dict(src_coeffs=None), -1), (dict(src_len_delta=1), -1), (dict(estimator="picard"), -2),
    (dict(ic="exact"), -1), (dict(alpha=0.5), -2), (dict(src_nan=True), -1)])
def test_invalid_polynomial_sources_are_rejected(change, status):
    import numpy as np
    n, M = 3, 2
    coeffs = np.zeros((n + 2) ** 2 * (M + 1))
    wl = W.small(dim=2, n=n, M_deg=M, src="poly", ic="nodal", ic_data=np.zeros((1, n * n))).with_(src_coeffs=coeffs)
    if "src_len_delta" in change:
        wl = wl.with_(src_coeffs=np.zeros(coeffs.size + 1))
    elif "src_nan" in change:
        bad = coeffs.copy()
        bad[3] = float("nan")
        wl = wl.with_(src_coeffs=bad)
    elif "alpha" in change:
        wl = W.small(dim=1, n=n, M_deg=M, src="poly", ic="nodal", ic_data=np.zeros((1, n)), alpha=0.5).with_(
            src_coeffs=np.zeros((n + 2) * (M + 1)))
    else:
        wl = wl.with_(**change)
    with pytest.raises(H.HpsmcError) as ei:
        H.resolve_nstar(wl)
    assert ei.value.status == status
