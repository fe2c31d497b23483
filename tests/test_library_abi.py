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


def test_nan_in_inputs_is_rejected_before_the_device():
    """A NaN or Inf anywhere in the description's floating-point inputs -> TM_EINVAL,
    found on the host (no GPU needed)."""
    import numpy as np
    import paper_2203_01120_amd as tm

    def desc(**bad):
        pt = dict(xk=np.zeros(3), mill=np.zeros((1, 3), np.int32), evc=np.ones((1, 2, 1), complex),
                  et=np.zeros(1))
        fields = dict(vrs=np.zeros((4, 4, 4, 4)), rho=np.ones((4, 4, 4, 4)))
        for k, v in bad.items():
            (pt if k in pt else fields)[k] = v
        return tm.SystemDesc(cell=np.eye(3) * 5, fft=(4, 4, 4), nbnd=1, points=[tm.Point(**pt)],
                             dvan=None, xq=np.zeros((1, 3)), roles=np.zeros((1, 1, 4), np.int32), **fields)

    evc = np.ones((1, 2, 1), complex)
    evc[0, 1, 0] = complex(0, np.nan)
    vrs = np.zeros((4, 4, 4, 4))
    vrs[2, 1, 2, 3] = np.inf
    et = np.array([np.nan])
    for bad in (dict(evc=evc), dict(vrs=vrs), dict(et=et)):
        try:
            tm.tm_system_create(desc(**bad))
        except tm.TmError as e:
            assert e.code == -1, (list(bad), e.code)
            assert "non-finite" in str(e)
        else:
            raise AssertionError("expected TM_EINVAL")
