"""CPU-side checks of the boundary: the library loads, exports every symbol the
header declares, and its host-only logic (argument checks, motion steps)
behaves; nothing here launches device work."""
import os
import re

import numpy as np
import pytest

from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mrv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(mrv_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(mrv.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = mrv.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_motion_steps_matches_workload_recipe():
    rng = np.random.default_rng(1)
    for _ in range(200):
        dq = rng.uniform(-2, 2, 7)
        assert mrv.motion_steps(dq, 1 / 32, "linf") == W.steps_for(dq, 1 / 32, "linf")
        assert mrv.motion_steps(dq, 0.005, "l2") == W.steps_for(dq, 0.005, "l2")
    assert mrv.motion_steps([0.0] * 3, 0.1, "l2") == 0
    with pytest.raises(mrv.MrvError):
        mrv.motion_steps([1.0], 0.0, "l2")
    with pytest.raises(mrv.MrvError):
        mrv.motion_steps([float("nan")], 0.1, "l2")


def test_null_context_is_rejected():
    L = mrv.lib()
    out = np.zeros(1, np.uint8)
    assert L.mrv_mv(None, 1, -1, None, 0, out.ctypes.data) == mrv.MRV_E_HANDLE
    assert L.mrv_destroy(None) == mrv.MRV_OK
    assert L.mrv_sync(None) == mrv.MRV_E_HANDLE
    assert "context" in mrv.last_error()


def test_create_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(mrv.MrvError) as e:
        mrv.Context(0)
    assert e.value.status == mrv.MRV_E_DEVICE
