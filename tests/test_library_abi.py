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


def _footprint_case(fft, kmesh, q_frac, folded=False):
    import sys
    import synth
    from oracle import liouvillian as lv
    from oracle import scf
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import desc_from_problem
    gs = scf.scf(synth.make_tiny(fft=fft, kmesh=kmesh, seed=11), tol=1e-10, beta=0.5)
    if folded:   # q on the mesh: sister points folded onto it with Miller shifts
        return desc_from_problem(lv.Problem(gs, synth.qset_folded(gs.sysd, q_frac)))
    return desc_from_problem(lv.build_problem(gs, synth.cart_from_frac(gs.sysd, q_frac)))


def test_footprint_from_the_descriptor_without_a_device():
    """tm_system_footprint is host work (the serving scheduler admits by it
    before a system exists).  Its resident and column figures follow the
    layouts they describe, recomputed here from the descriptor alone:
    * the resident real-space ground state holds one slot per distinct
      (point, Miller shift, side) among the q sets' roles (X side: k, Y side:
      -k), each nbnd bands x n3 planes x 2 spins x n1 n2 complex doubles; 0 on
      grids without fixed-size plane kernels (10^3 here);
    * the column cache holds, per side and k, nbnd bands x 2 spins x n3
      planes x the largest number of distinct (m1, m2) columns among the k
      and -k spheres, complex doubles."""
    import numpy as np
    import paper_2203_01120_amd as tm
    cases = [((8, 8, 8), ((0.0, 0.0, 0.0),), (0.1, 0.05, 0.0), False),
             ((8, 8, 8), ((0.0, 0.0, 0.0), (0.5, 0.0, 0.0)), (0.5, 0.0, 0.0), True),
             ((8, 8, 8), ((0.0, 0.0, 0.0), (0.5, 0.0, 0.0)), (0.1, 0.0, 0.0), False),
             ((10, 10, 10), ((0.0, 0.0, 0.0),), (0.1, 0.0, 0.0), False)]
    for fft, kmesh, qf, folded in cases:
        d = _footprint_case(fft, kmesh, qf, folded)
        got = tm.tm_system_footprint(d)
        n1, n2, n3 = d.fft
        roles = np.asarray(d.roles)
        shifts = np.zeros(roles.shape + (3,), int) if d.shifts is None else np.asarray(d.shifts)
        nq, nk = roles.shape[:2]
        slots = {(int(roles[iq, ik, s]), tuple(int(v) for v in shifts[iq, ik, s]), s)
                 for iq in range(nq) for ik in range(nk) for s in (0, 1)}
        fixed = (n1, n2) in {(8, 8), (20, 20), (24, 24), (32, 32), (48, 48)}
        want_res = len(slots) * d.nbnd * n3 * 2 * n1 * n2 * 16 if fixed else 0
        ncol = [len({(int(a), int(b)) for a, b, _ in p.mill}) for p in d.points]
        cols_u = max(max(ncol[roles[iq, ik, 0]], ncol[roles[iq, ik, 1]]) for iq in range(nq) for ik in range(nk))
        want_cols = 2 * nk * 2 * d.nbnd * n3 * cols_u * 16
        assert got["resident_full"] == want_res, (fft, kmesh, got, want_res)
        assert got["columns_full"] == want_cols, (fft, kmesh, got, want_cols)
        assert got["tables"] > 0 and got["workspace_per_rhs"] > 0
        assert got["resident"] == got["columns"] == got["workspace"] == got["chain_slots"] == 0
        if folded:
            assert np.any(shifts != 0)   # the shift is part of a slot's identity


def test_unsupported_grids_refused_on_the_host():
    """Grid lengths with a prime factor other than 2, 3, 5, or planes of more
    than 4096 points: tm_system_create refuses them with TM_EUNSUPPORTED before
    it looks for a device, and tm_system_footprint refuses the same grids (the
    scheduler must not charge the budget for a system that cannot exist)."""
    import numpy as np
    import paper_2203_01120_amd as tm

    def desc(fft):
        return tm.SystemDesc(cell=np.eye(3) * 5, fft=fft, nbnd=1,
                             points=[tm.Point(xk=np.zeros(3), mill=np.zeros((1, 3), np.int32),
                                              evc=np.ones((1, 2, 1), complex), et=np.zeros(1))],
                             vrs=np.zeros((4,) + tuple(fft)), rho=np.zeros((4,) + tuple(fft)), dvan=None,
                             xq=np.zeros((1, 3)), roles=np.zeros((1, 1, 4), np.int32))

    for fft in ((7, 8, 8), (8, 8, 14), (48, 96, 8)):
        for call in (tm.tm_system_create, tm.tm_system_footprint):
            try:
                call(desc(fft))
            except tm.TmError as e:
                assert e.code == -5, (fft, call.__name__, e.code)
            else:
                raise AssertionError(f"{call.__name__} accepted the grid {fft}")
    assert tm.tm_system_footprint(desc((8, 8, 30)))["tables"] > 0   # 2 x 3 x 5 is fine


def test_descriptor_extents_checked_before_the_library_reads_them():
    """The library reads the descriptor's arrays through plain pointers, so
    the binding checks their extents first: each too-short or misshapen array
    raises ValueError (never reaches the library), a valid one passes."""
    import numpy as np
    import pytest
    import paper_2203_01120_amd as tm

    fft = (4, 4, 4)

    def desc(**over):
        pt = dict(xk=np.zeros(3), mill=np.zeros((2, 3), np.int32), evc=np.ones((1, 2, 2), complex),
                  et=np.zeros(1), vkb=np.ones((2, 2), complex))
        pt.update(over.pop("pt", {}))
        kw = dict(cell=np.eye(3) * 5, fft=fft, nbnd=1, points=[tm.Point(**pt)], vrs=np.zeros((4,) + fft),
                  rho=np.zeros((4,) + fft), dvan=np.zeros((2, 2, 2, 2), complex), xq=np.zeros((1, 3)),
                  roles=np.zeros((1, 1, 4), np.int32), shifts=np.zeros((1, 1, 4, 3), np.int32))
        kw.update(over)
        return tm.SystemDesc(**kw)

    assert tm.tm_system_footprint(desc())["tables"] > 0
    bad = [dict(pt=dict(evc=np.ones((1, 2, 1), complex))),      # fewer coefficients than the sphere
           dict(pt=dict(evc=np.ones((1, 1, 2), complex))),      # one spin component
           dict(nbnd=2),                                        # evc and et hold one band
           dict(pt=dict(et=np.zeros(0))),
           dict(pt=dict(mill=np.zeros((2, 2), np.int32))),
           dict(pt=dict(vkb=np.ones((1, 2), complex))),         # dvan says 2 projectors
           dict(pt=dict(vkb=None)),
           dict(vrs=np.zeros((4, 4, 4))),
           dict(rho=np.zeros((3,) + fft)),
           dict(dvan=np.zeros((2, 2, 2), complex)),
           dict(roles=np.ones((1, 1, 4), np.int32)),            # points 0 .. 0 only
           dict(roles=np.zeros((2, 1, 4), np.int32)),           # two q sets, one q vector
           dict(shifts=np.zeros((1, 1, 4), np.int32))]
    for over in bad:
        with pytest.raises(ValueError):
            tm.tm_system_footprint(desc(**over))
        with pytest.raises(ValueError):
            tm.tm_system_create(desc(**over))


def test_coefficient_extents_checked_before_the_library_reads_them():
    """tm_chi and its variants read alpha, beta, gamma, z[3] and zn up to the
    capacity (alpha's length): inconsistent arrays raise ValueError in the
    binding, before any pointer reaches the library."""
    import numpy as np
    import pytest
    import paper_2203_01120_amd as tm
    M = 6

    def co(**over):
        d = dict(alpha=np.zeros(M, complex), beta=np.ones(M), gamma=np.ones(M, complex),
                 z=np.zeros((3, M), complex), zn=np.zeros(M, complex), n1=1.0, steps_done=M)
        d.update(over)
        return d

    w = np.zeros(3)
    for bad in (dict(beta=np.ones(M - 1)), dict(gamma=np.ones(M + 1, complex)), dict(z=np.zeros((3, M - 1), complex)),
                dict(z=np.zeros((2, M), complex)), dict(zn=np.zeros(M - 2, complex)), dict(steps_done=M + 1),
                dict(alpha=np.zeros((1, M), complex))):
        with pytest.raises(ValueError):
            tm.tm_chi(co(**bad), 1, w, 0.1)
        with pytest.raises(ValueError):
            tm.tm_chi_extrapolated(co(**bad), 1, 10, "constant", w, 0.1)
        with pytest.raises(ValueError):
            tm.tm_chi_tensor(co(**bad), 1, w, 0.1)


def test_frequency_grid_and_tensor_shapes_checked_in_the_binding():
    """A frequency grid must be 1-D (a scalar is a one-point grid); S(q, w)
    needs three components of q and chi of shape (3, 3, nomega)."""
    import numpy as np
    import pytest
    import paper_2203_01120_amd as tm
    co = dict(alpha=np.zeros(2, complex), beta=np.ones(2), gamma=np.ones(2, complex), z=np.zeros((3, 2), complex),
              n1=1.0, steps_done=2)
    for call in (lambda w: tm.tm_chi(co, 2, w, 0.1), lambda w: tm.tm_chi_extrapolated(co, 2, 4, "constant", w, 0.1),
                 lambda w: tm.tm_chi_tensor(co, 2, w, 0.1)):
        with pytest.raises(ValueError):
            call(np.zeros((2, 3)))
    with pytest.raises(ValueError):
        tm.tm_structure_factor(np.zeros(2), np.zeros((3, 3, 4), complex))
    with pytest.raises(ValueError):
        tm.tm_structure_factor(np.ones(3), np.zeros((3, 4), complex))
