"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, and rejects bad arguments synchronously."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1512_01641_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libnwmine.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nwm_[a-z_]+)\s*\(", txt)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(_abi.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_strerror():
    lib = _abi.load()
    assert lib.nwm_strerror(0) == b"ok"
    assert lib.nwm_strerror(1) == b"invalid argument"
    assert lib.nwm_strerror(99) == b"unknown status"
    # no entry point has failed on a device in this thread
    assert lib.nwm_last_device_error() == b"none"


def test_null_arguments_rejected():
    lib = _abi.load()
    assert lib.nwm_create(None, 0) == _abi.NWM_EINVAL
    h = ctypes.c_void_p()
    assert lib.nwm_plan_create(None, None, 4, 0, ctypes.byref(h)) == _abi.NWM_EINVAL
    assert lib.nwm_plan_sizes(None, None) == _abi.NWM_EINVAL
    assert lib.nwm_score_pairs(None, None, None, _abi.Scorer(0, 0, 0), None, None, None, None) == _abi.NWM_EINVAL
    assert lib.nwm_align_batch(None, None, -0.2, 0.5, None, None, None, None, None, None, None) == _abi.NWM_EINVAL
    assert lib.nwm_plan_set_timing(None, 1) == _abi.NWM_EINVAL
    lib.nwm_destroy(None)
    lib.nwm_plan_destroy(None)


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _abi.load()
    h = ctypes.c_void_p()
    assert lib.nwm_create(ctypes.byref(h), 0) == _abi.NWM_EDEVICE


def test_product_path_refuses_to_run_without_library(tmp_path):
    with pytest.raises(RuntimeError, match="not built"):
        _abi.load(str(tmp_path / "missing.so"))


def test_null_arguments_rejected_new_calls():
    lib = _abi.load()
    failed = ctypes.c_int32(7)
    assert lib.nwm_align_check(None, None, ctypes.byref(failed), None) == _abi.NWM_EINVAL
    assert failed.value == 0
    assert lib.nwm_plan_set_param(None, 5, 1) == _abi.NWM_EINVAL


def test_build_guard_rejects_scratch_in_hand_counted_kernels():
    """The build fails when a kernel whose memory waits are counted by hand
    spills to scratch (parsed from the compiler's resource-usage remarks)."""
    from paper_1512_01641_amd import build as B

    def remarks(scratch):
        lines = []
        for k in ("_ZN3nwm9k_nw_fillILb1EEEv", "_ZN3nwm9k_nw_walkENS_7PlanDevE"):
            lines.append("k_align.hip:1:1: remark: Function Name: %s [-Rpass-analysis=kernel-resource-usage]" % k)
            lines.append("k_align.hip:1:1: remark:     VGPRs: 64 [-Rpass-analysis=kernel-resource-usage]")
            lines.append("k_align.hip:1:1: remark:     ScratchSize [bytes/lane]: %d "
                         "[-Rpass-analysis=kernel-resource-usage]" % (scratch if "fill" in k else 0))
        return "\n".join(lines)
    assert B.resource_usage(remarks(0))["_ZN3nwm9k_nw_fillILb1EEEv"]["VGPRs"] == 64
    B.check_scratch("k_align.hip", remarks(0))
    with pytest.raises(RuntimeError, match="scratch"):
        B.check_scratch("k_align.hip", remarks(16))
    with pytest.raises(RuntimeError, match="no resource-usage"):
        B.check_scratch("k_align.hip", "")
    B.check_scratch("k_score.hip", "")   # not guarded
