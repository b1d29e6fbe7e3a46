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
    (dict(f="affine", seed=1, nstar=[0, 3, 3, 3]), -1), (dict(nstar=[1 << 24] * 4), -1),
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
