"""The C-ABI library loads and exports every entry point include/tm.h declares (CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2203_01120_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = declared_functions()
    assert "tm_liouvillian_apply" in names and "tm_system_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(binding.EXPORTED) == names


def test_error_path_without_device():
    """With no GPU visible, creation fails with TM_EDEVICE and a message (no CPU fallback)."""
    import numpy as np
    import paper_2203_01120_amd as tm
    import torch
    if torch.cuda.is_available():
        return
    d = tm.SystemDesc(cell=np.eye(3) * 5, fft=(4, 4, 4), nbnd=1,
                      points=[tm.Point(xk=np.zeros(3), mill=np.zeros((1, 3), np.int32),
                                       evc=np.ones((1, 2, 1), complex), et=np.zeros(1))],
                      vrs=np.zeros((4, 4, 4, 4)), rho=np.zeros((4, 4, 4, 4)), dvan=None,
                      xq=np.zeros((1, 3)), roles=np.zeros((1, 1, 4), np.int32))
    try:
        tm.tm_system_create(d)
    except tm.TmError as e:
        assert e.code == -3
    else:
        raise AssertionError("expected TM_EDEVICE")
