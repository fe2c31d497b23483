"""Helpers shared by the GPU tests: oracle Problem -> library inputs and layouts."""
import sys

import numpy as np

import synth


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def desc_from_problem(prob, rho=None):
    """Library inputs for an oracle Problem; `rho` replaces the ground-state
    density and magnetisation that the kernel fields are built from."""
    from paper_2203_01120_amd import Point, SystemDesc
    sysd = prob.sysd
    nb = prob.nb
    pts = []
    for i, p in enumerate(prob.qset.points):
        mill, evc, et = prob.point_states[i]
        pts.append(Point(xk=np.asarray(p, float), mill=mill, evc=evc[:nb], et=np.asarray(et[:nb]),
                         vkb=synth.projector_table(sysd, p, mill)))
    return SystemDesc(cell=sysd.cell, fft=sysd.fft, nbnd=nb, points=pts, vrs=prob.vrs,
                      rho=prob.gs.rho if rho is None else rho,
                      dvan=synth.dmatrix(sysd), xq=np.asarray(prob.qset.q)[None],
                      roles=np.asarray(prob.qset.roles)[None], shifts=np.asarray(prob.qset.shifts)[None])


def desc_from_problems(probs):
    """One system holding the q sets of several oracle Problems of one ground state."""
    from paper_2203_01120_amd import Point, SystemDesc
    p0 = probs[0]
    sysd, nb = p0.sysd, p0.nb
    pts, roles, shifts = [], [], []
    for prob in probs:
        off = len(pts)
        for i, p in enumerate(prob.qset.points):
            mill, evc, et = prob.point_states[i]
            pts.append(Point(xk=np.asarray(p, float), mill=mill, evc=evc[:nb], et=np.asarray(et[:nb]),
                             vkb=synth.projector_table(sysd, p, mill)))
        roles.append(np.asarray(prob.qset.roles) + off)
        shifts.append(np.asarray(prob.qset.shifts))
    return SystemDesc(cell=sysd.cell, fft=sysd.fft, nbnd=nb, points=pts, vrs=p0.vrs, rho=p0.gs.rho,
                      dvan=synth.dmatrix(sysd), xq=np.array([np.asarray(pr.qset.q) for pr in probs]),
                      roles=np.array(roles), shifts=np.array(shifts))


def to_gpu(x, npw_pad):
    import torch
    out = np.zeros(x.shape[:-1] + (npw_pad,), dtype=np.complex128)
    n = min(npw_pad, x.shape[-1])
    out[..., :n] = x[..., :n]
    return torch.from_numpy(out.ravel()).to("cuda")


def from_gpu(t, shape_gpu, npw_pad_oracle):
    a = t.detach().cpu().numpy().reshape(shape_gpu)
    out = np.zeros(shape_gpu[:-1] + (npw_pad_oracle,), dtype=np.complex128)
    n = min(npw_pad_oracle, shape_gpu[-1])
    out[..., :n] = a[..., :n]
    return out, a


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
