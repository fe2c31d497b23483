"""Thin ctypes binding of libtm (include/tm.h): argument marshalling only.

Every step of the Liouvillian, the Lanczos recursions and chi runs inside the
HIP library; this module only packs host arrays into the C structs, passes
device pointers of torch tensors and the current HIP stream, and turns error
codes into exceptions.  There is no CPU fallback: if the library is missing or
no GPU is visible the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtm.so")

TM_OK, TM_EINVAL, TM_ENOMEM, TM_EDEVICE, TM_EBREAKDOWN, TM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
TM_FP64, TM_FP32 = 0, 1
DIRS = {"x": 0, "y": 1, "z": 2, "+": 3, "-": 4, "n": 5}
FLAVOURS = {"nH": 0, "non_hermitian": 0, "pH": 1, "pseudo_hermitian": 1}

EXPORTED = ["tm_system_create", "tm_system_destroy", "tm_qset_info_get", "tm_system_set_resident_limit",
            "tm_system_set_chain_slots",
            "tm_system_resident_bytes", "tm_system_memory", "tm_system_footprint", "tm_liouvillian_apply", "tm_liouvillian_apply_noalloc",
            "tm_autotune_enable", "tm_autotune_force", "tm_autotune_report", "tm_chain_begin", "tm_chains_step", "tm_chains_use_graphs",
            "tm_chain_coeffs", "tm_chain_end", "tm_chi_extrapolated", "tm_structure_factor",
            "tm_chain_state_size", "tm_chain_save", "tm_chain_restore", "tm_chi_tensor",
            "tm_chain_begin_multi", "tm_chain_begin_lanes", "tm_chain_lanes", "tm_tensor_run", "tm_liouvillian_apply_multi",
            "tm_start_vectors", "tm_lanczos_run", "tm_chi", "tm_profile_enable", "tm_profile_reset",
            "tm_profile_count", "tm_profile_get", "tm_last_error"]


class TmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libtm error {code}: {msg}")
        self.code = code


class _Desc(C.Structure):
    _fields_ = [
        ("cell", C.c_double * 9), ("fft", C.c_int * 3), ("nbnd", C.c_int),
        ("npts", C.c_int), ("xk", C.POINTER(C.c_double)), ("npw", C.POINTER(C.c_int)),
        ("mill", C.POINTER(C.POINTER(C.c_int))), ("evc", C.POINTER(C.POINTER(C.c_double))),
        ("et", C.POINTER(C.POINTER(C.c_double))),
        ("vrs", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)),
        ("nproj", C.c_int), ("vkb", C.POINTER(C.POINTER(C.c_double))), ("dvan", C.POINTER(C.c_double)),
        ("nq", C.c_int), ("xq", C.POINTER(C.c_double)), ("nk", C.c_int),
        ("roles", C.POINTER(C.c_int)), ("shifts", C.POINTER(C.c_int)),
    ]


class _QInfo(C.Structure):
    _fields_ = [("nk", C.c_int), ("nbnd", C.c_int), ("npw_pad", C.c_int), ("nelem", C.c_longlong),
                ("lam", C.c_double)]


class _MemInfo(C.Structure):
    _fields_ = [("tables", C.c_longlong), ("resident", C.c_longlong), ("resident_full", C.c_longlong),
                ("columns", C.c_longlong), ("columns_full", C.c_longlong), ("workspace", C.c_longlong),
                ("workspace_per_rhs", C.c_longlong), ("chain_slots", C.c_int)]


class _Coeffs(C.Structure):
    _fields_ = [("capacity", C.c_int), ("steps_done", C.c_int), ("n1", C.c_double),
                ("alpha", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double)),
                ("gamma", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double)),
                ("zn", C.POINTER(C.c_double))]


_lib = None


def load(path: str = LIB_PATH):
    """Load libtm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_2203_01120_amd.build_lib.build()")
    lib = C.CDLL(path)
    lib.tm_system_create.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_void_p)]
    lib.tm_system_destroy.argtypes = [C.c_void_p]
    lib.tm_qset_info_get.argtypes = [C.c_void_p, C.c_int, C.POINTER(_QInfo)]
    lib.tm_system_set_resident_limit.argtypes = [C.c_void_p, C.c_longlong]
    lib.tm_system_set_chain_slots.argtypes = [C.c_void_p, C.c_int]
    lib.tm_chain_begin.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                   C.POINTER(C.c_void_p)]
    lib.tm_chains_step.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_void_p]
    lib.tm_chain_coeffs.argtypes = [C.c_void_p, C.POINTER(_Coeffs)]
    lib.tm_chain_end.argtypes = [C.c_void_p]
    lib.tm_chains_use_graphs.argtypes = [C.c_int]
    lib.tm_chain_state_size.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
    lib.tm_chain_save.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.tm_chain_restore.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p,
                                     C.POINTER(C.c_void_p)]
    lib.tm_chi_extrapolated.argtypes = [C.POINTER(_Coeffs), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                        C.c_int, C.c_double, C.POINTER(C.c_double)]
    lib.tm_chi_tensor.argtypes = [C.POINTER(_Coeffs), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                  C.c_int, C.c_double, C.POINTER(C.c_double)]
    lib.tm_structure_factor.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int,
                                        C.POINTER(C.c_double)]
    lib.tm_system_resident_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_longlong)]
    lib.tm_system_memory.argtypes = [C.c_void_p, C.POINTER(_MemInfo)]
    lib.tm_system_footprint.argtypes = [C.POINTER(_Desc), C.POINTER(_MemInfo)]
    lib.tm_liouvillian_apply.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    lib.tm_liouvillian_apply_noalloc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    lib.tm_autotune_enable.argtypes = [C.c_int]
    lib.tm_autotune_force.argtypes = [C.c_int, C.c_int]
    lib.tm_autotune_report.argtypes = [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.tm_liouvillian_apply_multi.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                               C.c_void_p]
    lib.tm_start_vectors.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.tm_lanczos_run.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(_Coeffs)]
    lib.tm_tensor_run.argtypes = [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int, C.c_int, C.c_int,
                                  C.POINTER(_Coeffs)]
    lib.tm_chain_begin_multi.argtypes = [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int, C.c_int,
                                         C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.tm_chain_begin_lanes.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int,
                                         C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.tm_chain_lanes.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    lib.tm_chi.argtypes = [C.POINTER(_Coeffs), C.c_int, C.POINTER(C.c_double), C.c_int, C.c_double,
                           C.POINTER(C.c_double)]
    lib.tm_profile_enable.argtypes = [C.c_int]
    lib.tm_profile_reset.argtypes = []
    lib.tm_profile_count.argtypes = []
    lib.tm_profile_get.argtypes = [C.c_int, C.c_char_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
    lib.tm_last_error.restype = C.c_char_p
    for name in EXPORTED:
        getattr(lib, name).restype = C.c_int if name != "tm_last_error" else C.c_char_p
    _lib = lib
    return lib


def _check(rc: int, allow=()):
    if rc != TM_OK and rc not in allow:
        raise TmError(rc, load().tm_last_error().decode())
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


@dataclass
class Point:
    """Ground-state data of one k-related point."""
    xk: np.ndarray          # (3,) Cartesian
    mill: np.ndarray        # (npw, 3) int
    evc: np.ndarray         # (nbnd, 2, npw) complex128
    et: np.ndarray          # (nbnd,)
    vkb: Optional[np.ndarray] = None  # (nproj, npw) complex128


@dataclass
class SystemDesc:
    cell: np.ndarray
    fft: Sequence[int]
    nbnd: int
    points: List[Point]
    vrs: np.ndarray          # (4, n1, n2, n3): v_eff, B_x, B_y, B_z
    rho: np.ndarray          # (4, n1, n2, n3): n, m_x, m_y, m_z
    dvan: Optional[np.ndarray]   # (nproj, nproj, 2, 2) complex128
    xq: np.ndarray           # (nq, 3)
    roles: np.ndarray        # (nq, nk, 4) int
    shifts: Optional[np.ndarray] = None   # (nq, nk, 4, 3) int
    keep: list = field(default_factory=list)


def _check_shapes(d: SystemDesc, nproj: int) -> None:
    """The extents the library reads through the descriptor's plain pointers
    (ValueError otherwise, before any pointer is handed over): per point
    mill (npw, 3), evc (>= nbnd, 2, npw) (the first nbnd bands are read), et
    (>= nbnd,), vkb (nproj, npw); vrs and rho (4, n1, n2, n3); dvan
    (nproj, nproj, 2, 2); roles (nq, nk, 4) indexing the points; shifts
    (nq, nk, 4, 3)."""
    def need(ok, msg):
        if not ok:
            raise ValueError(msg)
    fft = tuple(int(x) for x in d.fft)
    nb = int(d.nbnd)
    need(len(fft) == 3 and len(d.points) > 0, "fft needs 3 lengths and there must be ground-state points")
    for i, p in enumerate(d.points):
        mill, evc, et = np.asarray(p.mill), np.asarray(p.evc), np.asarray(p.et)
        need(mill.ndim == 2 and mill.shape[1] == 3, f"point {i}: mill must be (npw, 3)")
        npw = mill.shape[0]
        need(np.asarray(p.xk).size == 3, f"point {i}: xk must hold 3 components")
        need(evc.ndim == 3 and evc.shape[0] >= nb and evc.shape[1:] == (2, npw),
             f"point {i}: evc must be (>= nbnd, 2, npw) = (>= {nb}, 2, {npw}), got {evc.shape}")
        need(et.ndim == 1 and et.shape[0] >= nb, f"point {i}: et must hold at least nbnd = {nb} values")
        if nproj:
            need(p.vkb is not None and np.asarray(p.vkb).shape == (nproj, npw),
                 f"point {i}: vkb must be (nproj, npw) = ({nproj}, {npw})")
    for name in ("vrs", "rho"):
        need(np.asarray(getattr(d, name)).shape == (4,) + fft, f"{name} must be (4, n1, n2, n3) = {(4,) + fft}")
    if nproj:
        need(np.asarray(d.dvan).shape == (nproj, nproj, 2, 2), "dvan must be (nproj, nproj, 2, 2)")
    nq = np.atleast_2d(d.xq).shape[0]
    need(np.atleast_2d(d.xq).shape[1] == 3, "xq must be (nq, 3)")
    roles = np.asarray(d.roles)
    need(roles.ndim == 3 and roles.shape[0] == nq and roles.shape[2] == 4, "roles must be (nq, nk, 4)")
    need(roles.size > 0 and roles.min() >= 0 and roles.max() < len(d.points), "roles must index the points")
    if d.shifts is not None:
        need(np.asarray(d.shifts).shape == roles.shape + (3,), "shifts must be (nq, nk, 4, 3)")


def _marshal_desc(d: SystemDesc, keep: list):
    """A tm_system_desc over host arrays of d (kept alive in `keep`)."""

    def c(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    npts = len(d.points)
    nproj = 0 if d.dvan is None else int(d.dvan.shape[0])
    _check_shapes(d, nproj)
    desc = _Desc()
    desc.cell[:] = list(np.asarray(d.cell, dtype=float).ravel())
    desc.fft[:] = [int(x) for x in d.fft]
    desc.nbnd = int(d.nbnd)
    desc.npts = npts
    xk = c(np.array([p.xk for p in d.points]), np.float64)
    desc.xk = _dptr(xk)
    npw = c(np.array([p.mill.shape[0] for p in d.points]), np.int32)
    desc.npw = _iptr(npw)
    mills = [c(p.mill, np.int32) for p in d.points]
    evcs = [c(p.evc, np.complex128) for p in d.points]
    ets = [c(p.et[:d.nbnd], np.float64) for p in d.points]
    MP = C.POINTER(C.c_int) * npts
    DP = C.POINTER(C.c_double) * npts
    mill_arr = MP(*[_iptr(m) for m in mills])
    evc_arr = DP(*[e.ctypes.data_as(C.POINTER(C.c_double)) for e in evcs])
    et_arr = DP(*[_dptr(e) for e in ets])
    keep += [mill_arr, evc_arr, et_arr]
    desc.mill = C.cast(mill_arr, C.POINTER(C.POINTER(C.c_int)))
    desc.evc = C.cast(evc_arr, C.POINTER(C.POINTER(C.c_double)))
    desc.et = C.cast(et_arr, C.POINTER(C.POINTER(C.c_double)))
    vrs = c(d.vrs, np.float64)
    rho = c(d.rho, np.float64)
    desc.vrs = _dptr(vrs)
    desc.rho = _dptr(rho)
    desc.nproj = nproj
    if nproj:
        vkbs = [c(p.vkb, np.complex128) for p in d.points]
        vkb_arr = DP(*[v.ctypes.data_as(C.POINTER(C.c_double)) for v in vkbs])
        keep.append(vkb_arr)
        desc.vkb = C.cast(vkb_arr, C.POINTER(C.POINTER(C.c_double)))
        dv = c(d.dvan, np.complex128)
        desc.dvan = dv.ctypes.data_as(C.POINTER(C.c_double))
    xq = c(np.atleast_2d(d.xq), np.float64)
    desc.nq = xq.shape[0]
    desc.xq = _dptr(xq)
    roles = c(d.roles, np.int32)
    desc.nk = roles.shape[1]
    desc.roles = _iptr(roles)
    if d.shifts is not None:
        sh = c(d.shifts, np.int32)
        desc.shifts = _iptr(sh)
    return desc


def tm_system_create(d: SystemDesc):
    """Upload a system; returns an opaque handle (int)."""
    lib = load()
    keep = []
    desc = _marshal_desc(d, keep)
    h = C.c_void_p()
    _check(lib.tm_system_create(C.byref(desc), C.byref(h)))
    return h.value


def tm_system_footprint(d: SystemDesc) -> dict:
    """Device bytes a system will hold, from its descriptor (nothing allocated; see tm.h)."""
    keep = []
    desc = _marshal_desc(d, keep)
    m = _MemInfo()
    _check(load().tm_system_footprint(C.byref(desc), C.byref(m)))
    return {k: getattr(m, k) for k, _ in _MemInfo._fields_}


def tm_system_destroy(h):
    if h:
        _check(load().tm_system_destroy(C.c_void_p(h)))


def tm_qset_info_get(h, iq: int = 0) -> dict:
    info = _QInfo()
    _check(load().tm_qset_info_get(C.c_void_p(h), iq, C.byref(info)))
    return dict(nk=info.nk, nbnd=info.nbnd, npw_pad=info.npw_pad, nelem=info.nelem, lam=info.lam)


def tm_system_set_resident_limit(h, nbytes: int) -> None:
    """Limit (bytes) on the resident real-space ground state; -1 = default, 0 = off."""
    _check(load().tm_system_set_resident_limit(C.c_void_p(h), int(nbytes)))


def tm_system_set_chain_slots(h, nslots: int) -> None:
    """At most nslots concurrent workspace slots for the system's chains begun
    afterwards (1: every chain on the caller's stream)."""
    _check(load().tm_system_set_chain_slots(C.c_void_p(h), int(nslots)))


def tm_system_resident_bytes(h) -> int:
    out = C.c_longlong(0)
    _check(load().tm_system_resident_bytes(C.c_void_p(h), C.byref(out)))
    return int(out.value)


def tm_system_memory(h) -> dict:
    """Device bytes of a system (tables, resident copy, columns, workspaces; see tm.h)."""
    m = _MemInfo()
    _check(load().tm_system_memory(C.c_void_p(h), C.byref(m)))
    return {k: getattr(m, k) for k, _ in _MemInfo._fields_}


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_tensor(t, nelem):
    import torch
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous() and t.numel() == nelem):
        raise ValueError(f"expected a contiguous complex128 CUDA tensor with {nelem} elements")


def tm_liouvillian_apply(h, iq: int, xy_in, xy_out, prec: int = TM_FP64, stream=None):
    """xy_out = L xy_in on the device (torch complex128 tensors of BR shape)."""
    nelem = tm_qset_info_get(h, iq)["nelem"]
    _check_tensor(xy_in, nelem)
    _check_tensor(xy_out, nelem)
    _check(load().tm_liouvillian_apply(C.c_void_p(h), iq, C.c_void_p(xy_in.data_ptr()),
                                       C.c_void_p(xy_out.data_ptr()), prec, _stream(stream)))


def tm_liouvillian_apply_noalloc(h, iq: int, xy_in, xy_out, prec: int = TM_FP64, stream=None):
    """xy_out = L xy_in without any device allocation (library scratch; see tm.h)."""
    nelem = tm_qset_info_get(h, iq)["nelem"]
    _check_tensor(xy_in, nelem)
    _check_tensor(xy_out, nelem)
    _check(load().tm_liouvillian_apply_noalloc(C.c_void_p(h), iq, C.c_void_p(xy_in.data_ptr()),
                                               C.c_void_p(xy_out.data_ptr()), prec, _stream(stream)))


TUNE_OPS = {"plane_density": 0, "plane_apply": 1, "zpass_inverse": 2, "zpass_forward": 3, "contraction": 4,
            "update": 5}


def tm_autotune_enable(on: bool) -> None:
    _check(load().tm_autotune_enable(1 if on else 0))


def tm_autotune_force(op: str, variant: int) -> None:
    """Force `variant` of a tunable operation for every shape (-1: the tuned choice)."""
    _check(load().tm_autotune_force(TUNE_OPS[op], int(variant)))


def tm_autotune_report() -> list:
    """The tuned shapes: dicts(op, shape, variants, chosen, us[])."""
    lib = load()
    need = C.c_size_t(0)
    _check(lib.tm_autotune_report(None, 0, C.byref(need)))
    buf = C.create_string_buffer(need.value)
    _check(lib.tm_autotune_report(buf, need.value, C.byref(need)))
    out = []
    for line in buf.value.decode().splitlines():
        op, shape, nv, ch, us = line.split("\t")
        out.append({"op": op, "shape": shape, "variants": int(nv.split()[1]), "chosen": int(ch.split()[1]),
                    "us": [round(float(x), 1) for x in us.split()[1:]]})
    return out


def tm_liouvillian_apply_multi(h, iq: int, nrhs: int, xy_in, xy_out, prec: int = TM_FP64, stream=None):
    """nrhs applications in one pass; xy_in / xy_out hold nrhs BR vectors back to back."""
    nelem = tm_qset_info_get(h, iq)["nelem"]
    _check_tensor(xy_in, nrhs * nelem)
    _check_tensor(xy_out, nrhs * nelem)
    _check(load().tm_liouvillian_apply_multi(C.c_void_p(h), iq, int(nrhs), C.c_void_p(xy_in.data_ptr()),
                                             C.c_void_p(xy_out.data_ptr()), prec, _stream(stream)))


def tm_start_vectors(h, iq: int, direction: str, u=None, v=None, stream=None):
    nelem = tm_qset_info_get(h, iq)["nelem"]
    for t in (u, v):
        if t is not None:
            _check_tensor(t, nelem)
    _check(load().tm_start_vectors(C.c_void_p(h), iq, DIRS[direction],
                                   C.c_void_p(u.data_ptr() if u is not None else 0),
                                   C.c_void_p(v.data_ptr() if v is not None else 0), _stream(stream)))


def _cptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _coeff_arrays(cap: int):
    """Output arrays for `cap` steps: alpha, beta, gamma, z[3] (x, y, z) and zn (charge)."""
    arrs = dict(alpha=np.zeros(cap, dtype=np.complex128), beta=np.zeros(cap),
                gamma=np.zeros(cap, dtype=np.complex128), z=np.zeros((3, cap), dtype=np.complex128),
                zn=np.zeros(cap, dtype=np.complex128))
    co = _Coeffs(cap, 0, 0.0, _cptr(arrs["alpha"]), _cptr(arrs["beta"]), _cptr(arrs["gamma"]), _cptr(arrs["z"]),
                 _cptr(arrs["zn"]))
    return co, arrs


def _coeffs_in(coeffs: dict):
    """A tm_coeffs view of a coefficient dict (arrays kept alive in the returned tuple)."""
    keep = {k: np.ascontiguousarray(coeffs[k], dtype=np.float64 if k == "beta" else np.complex128)
            for k in ("alpha", "beta", "gamma", "z")}
    zn = coeffs.get("zn")
    if zn is not None:
        keep["zn"] = np.ascontiguousarray(zn, dtype=np.complex128)
    # the library reads every array to the capacity (alpha's length): check
    # their extents before handing the pointers over
    cap = keep["alpha"].shape[0] if keep["alpha"].ndim == 1 else -1
    shapes = {k: v.shape for k, v in keep.items()}
    if (cap < 1 or shapes["beta"] != (cap,) or shapes["gamma"] != (cap,) or shapes["z"] != (3, cap)
            or shapes.get("zn", (cap,)) != (cap,) or not 0 <= int(coeffs["steps_done"]) <= cap):
        raise ValueError(f"coefficients must be alpha, beta, gamma (M,), z (3, M), zn (M,) with "
                         f"0 <= steps_done <= M; got {shapes}, steps_done {coeffs['steps_done']}")
    co = _Coeffs(keep["alpha"].shape[0], int(coeffs["steps_done"]), float(coeffs["n1"]), _cptr(keep["alpha"]),
                 _cptr(keep["beta"]), _cptr(keep["gamma"]), _cptr(keep["z"]),
                 _cptr(keep["zn"]) if "zn" in keep else None)
    return co, keep


def tm_lanczos_run(h, iq: int, direction: str, flavour: str, nsteps: int, prec: int = TM_FP64) -> dict:
    """Run one chain; returns dict(alpha, beta, gamma, z[3], zn, n1, steps_done, breakdown)."""
    co, arrs = _coeff_arrays(int(nsteps))
    rc = _check(load().tm_lanczos_run(C.c_void_p(h), iq, DIRS[direction], FLAVOURS[flavour], int(nsteps), prec,
                                      C.byref(co)), allow=(TM_EBREAKDOWN,))
    return dict(arrs, n1=co.n1, steps_done=co.steps_done, breakdown=rc == TM_EBREAKDOWN)


def tm_chain_begin(h, iq: int, direction: str, flavour: str, capacity: int, prec: int = TM_FP64,
                   stream=None) -> int:
    """Start a device-resident chain; returns its handle (asynchronous on `stream`)."""
    out = C.c_void_p()
    _check(load().tm_chain_begin(C.c_void_p(h), iq, DIRS[direction], FLAVOURS[flavour], prec, int(capacity),
                                 _stream(stream), C.byref(out)))
    return out.value


def tm_chains_step(chains, k_steps: int, stream=None) -> None:
    """Advance every chain by up to k_steps steps, one step per chain in turn."""
    arr = (C.c_void_p * max(len(chains), 1))(*chains)
    _check(load().tm_chains_step(arr, len(chains), int(k_steps), _stream(stream)))


def tm_chain_lanes(chain) -> int:
    n = C.c_int(0)
    _check(load().tm_chain_lanes(C.c_void_p(chain), C.byref(n)))
    return n.value


def _lane_coeffs(capacity: int, lanes: int):
    pairs = [_coeff_arrays(int(capacity)) for _ in range(lanes)]
    return (_Coeffs * max(lanes, 1))(*[p[0] for p in pairs]), [p[1] for p in pairs]


def _lane_dicts(carr, arrs, rc):
    return [dict(a, n1=co.n1, steps_done=co.steps_done, breakdown=co.steps_done < co.capacity and rc == TM_EBREAKDOWN)
            for co, a in zip(carr, arrs)]


def tm_chain_coeffs_lanes(chain, capacity: int) -> list:
    """Coefficients of every lane of a chain so far (waits for its stream)."""
    carr, arrs = _lane_coeffs(capacity, tm_chain_lanes(chain))
    rc = _check(load().tm_chain_coeffs(C.c_void_p(chain), carr), allow=(TM_EBREAKDOWN,))
    return _lane_dicts(carr, arrs, rc)


def tm_chain_coeffs(chain, capacity: int) -> dict:
    """Coefficients of a single-direction chain so far (waits for its stream)."""
    co, arrs = _coeff_arrays(int(capacity))
    assert tm_chain_lanes(chain) == 1, "use tm_chain_coeffs_lanes for a chain of several directions"
    rc = _check(load().tm_chain_coeffs(C.c_void_p(chain), C.byref(co)), allow=(TM_EBREAKDOWN,))
    return dict(arrs, n1=co.n1, steps_done=co.steps_done, breakdown=rc == TM_EBREAKDOWN)


def tm_chain_begin_multi(h, iq: int, directions, flavour: str, capacity: int, prec: int = TM_FP64,
                         stream=None) -> int:
    """One chain whose lanes run several field directions together."""
    d = (C.c_int * len(directions))(*[DIRS[x] for x in directions])
    out = C.c_void_p()
    _check(load().tm_chain_begin_multi(C.c_void_p(h), iq, len(directions), d, FLAVOURS[flavour], prec,
                                       int(capacity), _stream(stream), C.byref(out)))
    return out.value


def tm_chain_begin_lanes(h, iqs, directions, flavour: str, capacity: int, prec: int = TM_FP64,
                         stream=None) -> int:
    """One chain whose lane r runs q set iqs[r] and direction directions[r]."""
    if len(iqs) != len(directions):
        raise ValueError("one q set per direction")
    q = (C.c_int * len(iqs))(*[int(i) for i in iqs])
    d = (C.c_int * len(directions))(*[DIRS[x] for x in directions])
    out = C.c_void_p()
    _check(load().tm_chain_begin_lanes(C.c_void_p(h), len(iqs), q, d, FLAVOURS[flavour], prec, int(capacity),
                                       _stream(stream), C.byref(out)))
    return out.value


def tm_tensor_run(h, iq: int, directions, flavour: str, nsteps: int, prec: int = TM_FP64) -> list:
    """tm_lanczos_run for several directions in one pass; one coefficient dict per direction."""
    d = (C.c_int * len(directions))(*[DIRS[x] for x in directions])
    carr, arrs = _lane_coeffs(nsteps, len(directions))
    rc = _check(load().tm_tensor_run(C.c_void_p(h), iq, len(directions), d, FLAVOURS[flavour], int(nsteps), prec,
                                     carr), allow=(TM_EBREAKDOWN,))
    return _lane_dicts(carr, arrs, rc)


def tm_chains_use_graphs(on: bool) -> None:
    """Process-wide: replay chain steps from captured HIP graphs (default) or issue them directly."""
    _check(load().tm_chains_use_graphs(1 if on else 0))


def tm_chain_save(chain) -> np.ndarray:
    """The chain's complete state as a host byte array (waits for its stream)."""
    n = C.c_size_t(0)
    _check(load().tm_chain_state_size(C.c_void_p(chain), C.byref(n)))
    buf = np.empty(n.value, dtype=np.uint8)
    _check(load().tm_chain_save(C.c_void_p(chain), C.c_void_p(buf.ctypes.data), n.value))
    return buf


def tm_chain_restore(h, blob: np.ndarray, capacity: int = 0, stream=None) -> int:
    """A new chain continuing a saved one (capacity may grow)."""
    blob = np.ascontiguousarray(blob, dtype=np.uint8)
    out = C.c_void_p()
    _check(load().tm_chain_restore(C.c_void_p(h), C.c_void_p(blob.ctypes.data), blob.nbytes, int(capacity),
                                   _stream(stream), C.byref(out)))
    return out.value


def tm_chain_end(chain) -> None:
    _check(load().tm_chain_end(C.c_void_p(chain)))


def tm_chi(coeffs: dict, m_use: int, omega, eta: float) -> np.ndarray:
    """chi[l][w] for l = x, y, z from the Lanczos coefficients (runs on the GPU)."""
    co, _keep = _coeffs_in(coeffs)
    om = _omega(omega)
    out = np.zeros((3, om.shape[0]), dtype=np.complex128)
    _check(load().tm_chi(C.byref(co), int(m_use), _dptr(om), om.shape[0], float(eta),
                         out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


EXTRAP = {"no": 0, "constant": 1, "osc": 2}


def _omega(omega) -> np.ndarray:
    om = np.ascontiguousarray(omega, dtype=np.float64)
    if om.ndim != 1:
        raise ValueError(f"omega must be a 1-D frequency grid, got shape {om.shape}")
    return om


def tm_chi_extrapolated(coeffs: dict, m_use: int, m_total: int, mode: str, omega, eta: float) -> np.ndarray:
    """chi[l][w] with the tridiagonal matrix extended to m_total ('no', 'constant', 'osc')."""
    co, _keep = _coeffs_in(coeffs)
    om = _omega(omega)
    out = np.zeros((3, om.shape[0]), dtype=np.complex128)
    _check(load().tm_chi_extrapolated(C.byref(co), int(m_use), int(m_total), EXTRAP[mode], _dptr(om),
                                      om.shape[0], float(eta), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def tm_chi_tensor(coeffs: dict, m_use: int, omega, eta: float, m_total: int = 0, mode: str = "no") -> np.ndarray:
    """One column of the 4 x 4 susceptibility: chi[l][w], rows l = n, x, y, z."""
    co, _keep = _coeffs_in(coeffs)
    om = _omega(omega)
    out = np.zeros((4, om.shape[0]), dtype=np.complex128)
    _check(load().tm_chi_tensor(C.byref(co), int(m_use), int(m_total or m_use), EXTRAP[mode], _dptr(om),
                                om.shape[0], float(eta), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def tm_structure_factor(q, chi) -> np.ndarray:
    """S(q, w) = -Im Tr[P_perp(q) chi(w)] from chi[lambda][mu][w] (complex 3 x 3 x nomega)."""
    qv = np.ascontiguousarray(q, dtype=np.float64)
    ch = np.ascontiguousarray(chi, dtype=np.complex128)
    if qv.size != 3 or ch.ndim != 3 or ch.shape[:2] != (3, 3):
        raise ValueError(f"q must hold 3 components and chi be (3, 3, nomega); got {qv.shape}, {ch.shape}")
    out = np.zeros(ch.shape[2])
    _check(load().tm_structure_factor(_dptr(qv), ch.ctypes.data_as(C.POINTER(C.c_double)), ch.shape[2],
                                      _dptr(out)))
    return out


def tm_profile_enable(on: bool = True):
    _check(load().tm_profile_enable(1 if on else 0))


def tm_profile_reset():
    _check(load().tm_profile_reset())


def tm_profile_read() -> dict:
    """{kernel name: (total ms, launches)} of the launches recorded so far."""
    lib = load()
    n = lib.tm_profile_count()
    if n < 0:
        _check(n)
    out = {}
    buf = C.create_string_buffer(128)
    for i in range(n):
        ms, cnt = C.c_double(), C.c_longlong()
        _check(lib.tm_profile_get(i, buf, 128, C.byref(ms), C.byref(cnt)))
        out[buf.value.decode()] = (ms.value, cnt.value)
    return out
