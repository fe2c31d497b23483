#!/usr/bin/env python3
"""Throughput of the Liouville-Lanczos hot path on one MI355X.

Workload (default): the CrI3-monolayer-shaped system -- hexagonal a = 13 bohr,
c = 31 bohr (25 bohr vacuum), 2 'Cr' + 6 'I' Gaussian sites with s/px/py
Kleinman-Bylander projectors (SOC 0.02 Ha on 'I'), ~8000 plane waves per spinor
component, FFT grid 48 x 48 x 180, 104 occupied spinor bands, 6x6x1 k-mesh
(36 k, no symmetry), q = b1/6.  Inputs are seeded and synthetic: the occupied
manifold is a smooth random orthonormal set (no SCF at this size).

A step is one pseudo-Hermitian Lanczos step for the m_+ chain: one
Liouvillian application (FFTs, response density, Hartree + ALSDA potential,
local/nonlocal/SOC terms, empty-manifold projection) plus the FP64 recurrence
and the re-projection.  The chain is begun (start vectors, the first apply
L v) and stepped through W warm-up steps (graph capture) outside the timed
region; the timed region is exactly K further steps of the same chain, issued
as the library issues them (graph replay of step periods), bracketed by
device synchronisations.  `value` is Liouvillian applies per second (one per
pH step).  A second chain stepped with the kernel profiler on (HIP events
around every launch on its stream, kernels issued directly) gives the
per-kernel breakdown and the roofline of the kernel with the largest share.
`spectra_per_s_derived` is value / (M + 1) for M = 3000-step spectra (one
apply per step plus the set-up); --spectrum-steps M measures a whole chain
and its chi instead.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector and FP64 matrix (dense)
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector
HA_PER_MEV = 1.0 / 27211.386245988


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_inputs(workload: str, seed: int):
    import synth
    if workload == "hexslab":
        sysd = synth.make_hexslab()
        q = synth.cart_from_frac(sysd, [1.0 / 6.0, 0.0, 0.0])
    elif workload == "cubic20":
        sysd = synth.make_cubic20()
        q = np.array([0.1, 0.0, 0.0]) * 2 * np.pi / 10.0
    else:
        raise SystemExit(f"unknown workload {workload}")
    return synth.synthetic_inputs(sysd, q, seed=seed)


def make_desc(inp):
    import paper_2203_01120_amd as tm
    qs = inp["qset"]
    pts = [tm.Point(xk=p, mill=m, evc=e, et=et, vkb=v) for (p, m, e, et, v) in inp["points"]]
    sysd = inp["sysd"]
    return tm.SystemDesc(cell=sysd.cell, fft=sysd.fft, nbnd=sysd.nbnd, points=pts, vrs=inp["vrs"],
                         rho=inp["rho"], dvan=inp["dvan"], xq=qs.q[None], roles=qs.roles[None],
                         shifts=qs.shifts[None])


def kernel_models(inp, info, resident: bool, lanes: int = 1):
    """The method's work per launch of the main kernels: flops and HBM bytes.

    Flops (the plane kernels): per band, side, spin and plane i3, an in-plane
    transform of n1 x n2 points counts 5 NP log2 NP (unpruned; the inverse row
    stage actually runs only over the rows the sphere occupies, so the
    executed count is lower -- `flops_pruned`).  With the resident real-space
    ground state the apply transforms x (inverse) and its product (forward),
    the density transforms x (inverse); on the column path both kernels also
    finish the inverse transforms of u.  Point-wise work: 60 flop per point
    per band-side in the apply, 40 in the density.

    Bytes: only what the method must move (one apply reads the response
    vectors and the four ground-state sets U_k, TU_-k, U_k+q, TU_-k-q once,
    the projectors and the fields, and writes the result).  Each kernel is
    charged its part: the plane kernels the ground-state sets they use (u,
    u' on the sphere: 2 of the 4 sets, split between density and apply) and
    the fields; the z passes the response vectors in and out; the
    contractions the occupied sets and the projectors.  Re-reads of a cache
    the implementation keeps (the resident real-space ground state, the
    z-transformed columns) are not the method's bytes: they show up in the
    measured `traffic` instead.
    """
    sysd = inp["sysd"]
    n1, n2, n3 = sysd.fft
    NP = n1 * n2
    nk = info["nk"]
    nb = sysd.nbnd
    P = info["npw_pad"]
    nproj = sysd.nproj
    fft2d = 5.0 * NP * math.log2(NP)
    bands = 2 * nk * nb
    mills = [m for (_, m, _, _, _) in inp["points"]]
    npw_avg = np.mean([m.shape[0] for m in mills])
    # occupied rows of each plane (rows of the n1 x n2 plane the sphere touches)
    rows_avg = np.mean([len({int(a) for a, _, _ in m}) for m in mills])
    row_frac = rows_avg / n1
    fft2d_pruned_inv = 5.0 * NP * (math.log2(n2) + row_frac * math.log2(n1))
    set_bytes = bands * 2 * npw_avg * 16          # one ground-state set over all sides and k
    vec_bytes = set_bytes                          # one BR vector
    fields = 4 * sysd.ngrid * 8 + 10 * sysd.ngrid * 8 + 4 * sysd.ngrid * 16
    n_inv = 2 if resident else 4
    L = lanes
    apply_flops = L * bands * n3 * ((n_inv + 2) * fft2d + 60.0 * NP)
    apply_pruned = L * bands * n3 * (2 * fft2d_pruned_inv + (n_inv - 2) * fft2d_pruned_inv + 2 * fft2d + 60.0 * NP)
    dens_flops = L * bands * n3 * (n_inv * fft2d + 40.0 * NP)
    dens_pruned = L * bands * n3 * (n_inv * fft2d_pruned_inv + 40.0 * NP)
    gemm_flops = L * 8.0 * 2 * nk * (nb * nb * 2 * P + nproj * 2 * nb * P)
    proj_bytes = 2 * nk * nproj * P * 16
    plane_bytes = set_bytes / 2 + fields / 2     # u, u' and the fields, shared by density and apply
    return {
        "k_apply_w": dict(flops=apply_flops, flops_pruned=apply_pruned, bytes=plane_bytes),
        "k_apply_t": dict(flops=apply_flops, flops_pruned=apply_pruned, bytes=plane_bytes),
        "k_apply_planes": dict(flops=apply_flops, flops_pruned=apply_pruned, bytes=plane_bytes),
        "k_density_w": dict(flops=dens_flops, flops_pruned=dens_pruned, bytes=plane_bytes),
        "k_density_t": dict(flops=dens_flops, flops_pruned=dens_pruned, bytes=plane_bytes),
        "k_density": dict(flops=dens_flops, flops_pruned=dens_pruned, bytes=plane_bytes),
        "k_apply_w32": dict(flops=apply_flops, flops_pruned=apply_pruned, bytes=plane_bytes, fp32=True),
        "k_density_w32": dict(flops=dens_flops, flops_pruned=dens_pruned, bytes=plane_bytes, fp32=True),
        # one contraction S = O^H phi of the projector and of P_c (8 real flops per complex MAC)
        "k_gemm_cn_lds": dict(flops=gemm_flops, mfma=True),
        "k_gemm_cn": dict(flops=gemm_flops, mfma=True),
        "k_gemm_update": dict(flops=gemm_flops, mfma=True),
        "k_zinv_t": dict(bytes=L * vec_bytes),
        "k_zfwd_t": dict(bytes=2 * L * vec_bytes),
        # the whole apply: 12 transforms of the full grid per band and k (8 to real space,
        # 4 back) + 2 Hartree, both contractions of the projector and of P_c, point-wise
        # work (60 flop per point and band-side in the apply, 40 in the density); bytes:
        # vectors in and out, the four ground-state sets, the projectors twice, the fields
        "apply": dict(
            flops=L * (bands / 2 * 12 + 2) * 5.0 * sysd.ngrid * math.log2(sysd.ngrid)
            + 2 * gemm_flops + L * bands * sysd.ngrid * 100.0,
            bytes=L * 2 * vec_bytes + 2 * set_bytes + 2 * proj_bytes + fields),
    }


def measured_traffic(kernel: str):
    """HBM bytes per dispatch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    runs (calibrated against a plain copy), or None when the kernel source has
    changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hexslab_48x48x180_hbm_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    k = rec["kernels"].get(kernel)
    return None if k is None else round(k["bytes"], -6)


def host_info():
    """Host cores the process may use, the affinity mask and the CPU model."""
    aff = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass

    def ranges(v):
        out, i = [], 0
        while i < len(v):
            j = i
            while j + 1 < len(v) and v[j + 1] == v[j] + 1:
                j += 1
            out.append(f"{v[i]}-{v[j]}" if j > i else f"{v[i]}")
            i = j + 1
        return ",".join(out)
    return {"os_cpu_count": os.cpu_count(), "affinity": ranges(aff), "affinity_count": len(aff), "cpu_model": model}


def cpu_baseline(workload: str, seed: int, nk_full: int):
    """The oracle's matrix-free apply on one mesh point of the same system (bounded sample).

    scipy.fft on every host thread the process may use (the oracle's grid
    transforms), NumPy/BLAS for the rest; the median of at least two applies
    (about 10-30 s of host time), scaled to all mesh points (the work is
    linear in k)."""
    import synth
    from oracle import grid as ogrid
    from oracle import liouvillian as lv

    class _GS:  # the oracle Problem only reads these fields here
        pass

    if workload == "hexslab":
        sysd = synth.make_hexslab()     # all bands, one mesh point
        q = synth.cart_from_frac(sysd, [1.0 / 6.0, 0.0, 0.0])
        subset = [7]
    else:
        sysd = synth.make_cubic20()
        q = np.array([0.1, 0.0, 0.0]) * 2 * np.pi / 10.0
        subset = [0]
    inp = synth.synthetic_inputs(sysd, q, seed=seed, kmesh_subset=subset)
    gs = _GS()
    gs.sysd, gs.vrs, gs.rho = inp["sysd"], inp["vrs"], inp["rho"]
    prob = lv.Problem(gs, inp["qset"], point_states=[(m, e, et) for (_, m, e, et, _) in inp["points"]])
    x = prob.random_projected(1)
    times = []
    t_start = time.perf_counter()
    while len(times) < 2 or (time.perf_counter() - t_start < 10.0 and len(times) < 1000):
        t0 = time.perf_counter()
        prob.apply(x)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    try:
        from threadpoolctl import threadpool_info
        blas = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        blas = 1
    scale = nk_full / len(subset)
    per_apply = dt * scale
    host = host_info()
    return {"value": 1.0 / per_apply, "unit": "applies/s", "cores": int(ogrid.WORKERS), "kind": "oracle",
            "sample": f"matrix-free oracle applies on {len(subset)} of {nk_full} mesh points with all "
                      f"{sysd.nbnd} bands (same grid, spheres, projectors): median of {len(times)} "
                      f"({dt:.3g} s each, {sum(times):.1f} s in all), scaled x{scale:g} (work is linear in "
                      f"k-points); scipy.fft on {ogrid.WORKERS} threads, BLAS threads {blas}, "
                      f"element-wise NumPy on one",
            "seconds": float(sum(times)), "per_apply_s_sample": dt, **host}


EV = 27.211386245988  # eV per Hartree


def peak_shift(tm, got, ref, m, eta):
    """Position (meV) of the strongest interior peak of |Im chi| of the FP64
    chain `ref` -- searched over -10..10 eV on a 5 meV grid (a transverse
    chain's poles may sit at negative frequency), its strongest component --
    and how far the FP32 chain `got` moves it, both located on a 0.01 meV grid
    within 10 meV; (None, None) when there is no interior peak."""
    wide = (np.arange(4001) - 2000) * 5e-3 / EV
    a = np.abs(tm.tm_chi(ref, m, wide, eta).imag)
    c = int(np.argmax(a.max(axis=1)))
    peaks = [(a[c, i], i) for i in range(1, a.shape[1] - 1) if a[c, i] > a[c, i - 1] and a[c, i] > a[c, i + 1]]
    if not peaks:
        return None, None
    w0 = wide[max(peaks)[1]]
    wf = w0 + np.arange(-1000, 1001) * 1e-5 / EV
    p32 = wf[int(np.argmax(np.abs(tm.tm_chi(got, m, wf, eta)[c].imag)))]
    p64 = wf[int(np.argmax(np.abs(tm.tm_chi(ref, m, wf, eta)[c].imag)))]
    return float(p64 * EV * 1e3), float(abs(p32 - p64) * EV * 1e3)


def qpath_accuracy(tm, got, ref, omega, eta):
    """FP32 spectra against FP64 ones of the same chains: relative L2 error of
    Im chi on the benchmark's frequencies per chain (its strongest component),
    and the shift of each chain's strongest peak (peak_shift); the largest and
    the median over the chains."""
    l2, shift, where = [], [], []
    for g, r in zip(got, ref):
        m = min(g["steps_done"], r["steps_done"])
        if m == 0:
            continue
        x32, x64 = tm.tm_chi(g, m, omega, eta), tm.tm_chi(r, m, omega, eta)
        c = int(np.argmax(np.abs(x64.imag).max(axis=1)))
        l2.append(float(np.linalg.norm(x32.imag[c] - x64.imag[c]) / np.linalg.norm(x64.imag[c])))
        w0, d = peak_shift(tm, g, r, m, eta)
        if w0 is not None:
            where.append(w0)
            shift.append(d)
    return {"l2_rel_im_chi_max": max(l2), "l2_rel_im_chi_median": float(np.median(l2)),
            "peak_shift_meV_max": max(shift) if shift else None,
            "peak_meV_range": [min(where), max(where)] if where else None, "chains": len(l2),
            "omega": "L2 on 400 points 0-1.995 eV, eta 5 meV, per chain its strongest component; "
                     "peaks searched over -10..10 eV"}


def run_qpath(args, tm, torch):
    """Batched chains: the cubic20 system with 24 q along Gamma-M-K-Gamma, three
    directions each (m_+, m_-, m_z), 72 pseudo-Hermitian chains stepped
    together, then chi on 400 omega per chain.  --qpath-lanes 3: the three
    directions of a q set run as the lanes of one chain (24 chains over the
    workspace slots); 6, 12, 24, 72: the three directions of 2, 4, 8 or all
    24 q sets as the lanes of one chain (tm_chain_begin_lanes), so that each
    kernel of a step runs once for all of them; 1: one chain per direction."""
    import synth
    sysd = synth.make_cubic20()
    qfrac = synth.q_path(24)
    qs = np.array([synth.cart_from_frac(sysd, f) for f in qfrac])
    log("building qpath inputs (24 q, 49 points)")
    inp = synth.synthetic_inputs_multi(sysd, qs, seed=args.seed)
    pts = [tm.Point(xk=p, mill=m, evc=e, et=et, vkb=v) for (p, m, e, et, v) in inp["points"]]
    desc = tm.SystemDesc(cell=sysd.cell, fft=sysd.fft, nbnd=sysd.nbnd, points=pts, vrs=inp["vrs"],
                         rho=inp["rho"], dvan=inp["dvan"], xq=inp["xq"], roles=inp["roles"], shifts=inp["shifts"])
    h = tm.tm_system_create(desc)
    tm.tm_system_set_chain_slots(h, args.chain_slots)
    m = args.chain_steps
    omega = np.arange(400) * 5e-3 / EV
    eta = 5e-3 / EV
    specs = [(iq, mu) for iq in range(len(qs)) for mu in ("+", "-", "z")]
    prec = tm.TM_FP32 if args.precision == "fp32" else tm.TM_FP64
    # warm-up: one short chain per q set builds the per-q caches outside the timed region
    for iq in range(len(qs)):
        tm.tm_lanczos_run(h, iq, "+", "pH", 6, prec)
    torch.cuda.synchronize()
    lanes = args.qpath_lanes
    log(f"timed: {len(specs)} chains x {m} steps + chi ({args.precision}, {lanes} lane(s) per chain object)")
    t0 = time.perf_counter()
    if lanes == 3:
        chains = [tm.tm_chain_begin_multi(h, iq, ["+", "-", "z"], "pH", m, prec) for iq in range(len(qs))]
        tm.tm_chains_step(chains, m)
        coeffs = [co for c in chains for co in tm.tm_chain_coeffs_lanes(c, m)]
    elif lanes > 3:
        per = lanes // 3  # q sets per chain
        chains = [tm.tm_chain_begin_lanes(h, [iq for iq in range(k, k + per) for _ in range(3)],
                                          ["+", "-", "z"] * per, "pH", m, prec) for k in range(0, len(qs), per)]
        tm.tm_chains_step(chains, m)
        coeffs = [co for c in chains for co in tm.tm_chain_coeffs_lanes(c, m)]
    else:
        chains = [tm.tm_chain_begin(h, iq, mu, "pH", m, prec) for iq, mu in specs]
        tm.tm_chains_step(chains, m)
        coeffs = [tm.tm_chain_coeffs(c, m) for c in chains]
    # a chain that broke down before its first step has no spectrum (zeros)
    spectra = [tm.tm_chi(co, co["steps_done"], omega, eta) if co["steps_done"] > 0 else
               np.zeros((3, omega.size), complex) for co in coeffs]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for c in chains:
        tm.tm_chain_end(c)
    accuracy = None
    if prec == tm.TM_FP32:  # every spectrum again in FP64 (untimed): the error of the FP32 bulk path
        per = len(qs) // 8
        ref = []
        for k in range(0, len(qs), per):
            c = tm.tm_chain_begin_lanes(h, [iq for iq in range(k, k + per) for _ in range(3)], ["+", "-", "z"] * per,
                                        "pH", m, tm.TM_FP64)
            tm.tm_chains_step([c], m)
            ref += tm.tm_chain_coeffs_lanes(c, m)
            tm.tm_chain_end(c)
        accuracy = qpath_accuracy(tm, coeffs, ref, omega, eta)
        log(f"fp32 vs fp64: {accuracy}")
    tm.tm_system_destroy(h)
    nbroken = sum(int(co["breakdown"]) for co in coeffs)
    steps = sum(int(co["steps_done"]) for co in coeffs)
    log(f"{len(specs)} spectra in {dt:.3f} s; {steps} steps; {nbroken} breakdowns")
    log("steps done per chain: " + " ".join(f"{iq}{mu}:{co['steps_done']}" for (iq, mu), co in zip(specs, coeffs)))
    assert all(np.all(np.isfinite(sp)) for sp in spectra)
    out = {
        "metric": "chi(q,omega) spectra/s (batched chains)",
        "value": round(len(specs) / dt, 4),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": m,
        "warmup": 6,
        "ms_per_step": round(dt / m * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == tm.TM_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": "cubic a=10 bohr, 2 sites, 20^3 grid, 8 bands, Gamma; 24 q on Gamma-M-K-Gamma "
                               "x (m_+, m_-, m_z) = 72 pseudo-Hermitian chains, chi on 400 omega each",
                   "chains": len(specs), "chain_steps": m, "precision": args.precision,
                   "lanes_per_chain": lanes},
        "applies_per_s": round((steps + len(specs)) / dt, 1),
        "breakdowns": nbroken,
        "fp32_accuracy": accuracy,
        "autotune": tm.tm_autotune_report(),
    }
    print(json.dumps(out))


def serving_pool(tm, seed):
    """The served systems: name -> (SystemDef, q vectors, weight).  Cubic a = 10 bohr
    cell on 20^3 / 8 bands / Gamma, 24^3 / 16 bands / 2x2x1 k, 32^3 / 32 bands /
    3x3x1 k, and a CrI3-shaped slab (hexagonal a = 13, c = 16.5 bohr) on
    48x48x96 / 64 bands / 4x4x1 k; two q sets each; drawn 8:4:2:1."""
    import synth
    slab = synth.make_hexslab(c=16.5, fft=(48, 48, 96), nbnd=64, nk=4)
    qc = np.array([[0.1, 0.0, 0.0], [0.0, 0.15, 0.05]]) * 2 * np.pi / 10.0
    return {"cubic20": (synth.make_cubic20(), qc, 8.0), "cubic24": (synth.make_cubic(24, 16, 2), qc, 4.0),
            "cubic32": (synth.make_cubic(32, 32, 3), qc, 2.0),
            "slab96": (slab, np.array([synth.cart_from_frac(slab, [0.25, 0.0, 0.0]),
                                       synth.cart_from_frac(slab, [0.0, 0.25, 0.0])]), 1.0)}


SERVING_LABELS = {"cubic20": "20^3/8/1k (cubic a=10 bohr)", "cubic24": "24^3/16/4k (cubic)",
                  "cubic32": "32^3/32/9k (cubic)", "slab96": "48x48x96/64/16k (hexagonal slab a=13 c=16.5 bohr)"}


def run_serving(args, tm, torch):
    """Poisson arrivals of chi requests on a pool of systems (serving_pool) that
    the server creates on demand and evicts under a device-memory budget that
    counts every system's footprint (tables, ground state -- resident
    real-space copy capped per system, or columns -- and workspaces) and every
    chain; direction uniform over x, y, z, +, -; flavour uniform over pH, nH;
    500..3000 steps.  The continuous-batching server is compared with the
    plain one-at-a-time path (FIFO, tm_lanczos_run with directly issued
    kernels, systems created and evicted under the same budget) on the same
    requests, and every chi of the two is compared."""
    import synth
    from paper_2203_01120_amd import serving as sv
    pool = serving_pool(tm, args.seed)
    keep = [n for n in args.serving_systems.split(",") if n]
    if not keep or set(keep) - set(pool):
        raise SystemExit(f"--serving-systems: choose from {','.join(pool)}")
    pool = {n: pool[n] for n in keep}
    specs = {}
    for name, (sysd, qs, _) in pool.items():
        def make(sysd=sysd, qs=qs):
            inp = synth.synthetic_inputs_multi(sysd, qs, seed=args.seed)
            pts = [tm.Point(xk=p, mill=m, evc=e, et=et, vkb=v) for (p, m, e, et, v) in inp["points"]]
            return tm.SystemDesc(cell=sysd.cell, fft=sysd.fft, nbnd=sysd.nbnd, points=pts, vrs=inp["vrs"],
                                 rho=inp["rho"], dvan=inp["dvan"], xq=inp["xq"], roles=inp["roles"],
                                 shifts=inp["shifts"])
        specs[name] = sv.SystemSpec(make_desc=make, resident_cap=int(args.serving_resident_cap * 1e9))
    budget = int(args.serving_budget * 1e9)
    names = list(pool)
    weights = np.array([pool[n][2] for n in names])
    weights /= weights.sum()
    omega = np.arange(400) * 5e-3 / EV
    eta = 5e-3 / EV
    # descriptors are host work done once (kept by the pools); footprints from them
    probe = sv.SystemPool({}, budget, specs, lanes=args.serving_lanes, chain_slots=args.serving_chain_slots)
    for n in names:
        log(f"system {n}: fft {pool[n][0].fft}, {pool[n][0].nbnd} bands, {len(pool[n][0].kmesh)} k, "
            f"footprint {probe.footprint(n) / 1e9:.2f} GB")
    descs = {n: probe.desc(n) for n in names}
    specs = {n: sv.SystemSpec(make_desc=(lambda d=descs[n]: d), resident_cap=specs[n].resident_cap) for n in names}
    results = []
    maxdiff = 0.0
    for rate in [float(r) for r in args.rates.split(",")]:
        rng = np.random.default_rng(5000 + int(round(rate * 10)))
        t = np.cumsum(rng.exponential(1.0 / rate, args.requests))

        def make_requests():
            out = []
            for i in range(args.requests):
                r2 = np.random.default_rng(7000 + 1000 * int(round(rate * 10)) + i)
                out.append(sv.Request(rid=i, system=names[r2.choice(len(names), p=weights)], iq=int(r2.integers(2)),
                                      direction=str(r2.choice(["x", "y", "z", "+", "-"])),
                                      flavour=str(r2.choice(["pH", "nH"])), nsteps=int(r2.integers(500, 3001)),
                                      omega=omega, eta=eta, arrival=float(t[i])))
            return out
        log(f"rate {rate}/s: {args.requests} requests, batched server")
        server = sv.Server({}, budget_bytes=budget, lanes=args.serving_lanes, max_chains=args.serving_max_chains,
                           chain_slots=args.serving_chain_slots, specs=specs)
        try:
            batched = server.run(make_requests())
        finally:
            server.close()
        log(f"rate {rate}/s: one at a time")
        plain = sv.run_one_at_a_time({}, make_requests(), specs=specs, budget_bytes=budget)
        by_id = {r.rid: r for r in plain}
        for r in batched:
            ref = by_id[r.rid].chi
            maxdiff = max(maxdiff, float(np.abs(r.chi - ref).max() / max(np.abs(ref).max(), 1e-300)))
        sb, sp = sv.summary(batched), sv.summary(plain)
        sb.update(systems_created=server.pool.created, systems_evicted=server.pool.evicted)
        log(f"rate {rate}: batched {sb}  plain {sp}")
        results.append({"rate_per_s": rate, "batched": sb, "one_at_a_time": sp})
    best = max(results, key=lambda r: r["batched"]["spectra_per_s"])
    out = {
        "metric": "chi(q,omega) spectra/s and p50/p99 latency under Poisson load",
        "value": best["batched"]["spectra_per_s"],
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": None,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "serving: pool " + ", ".join(SERVING_LABELS[n] for n in names) + ", drawn "
                               + ":".join(f"{pool[n][2]:g}" for n in names) + ", 500..3000 steps, pH|nH, "
                               "x|y|z|+|-, chi on 400 omega; systems created on demand",
                   "rates_per_s": [r["rate_per_s"] for r in results], "requests_per_rate": args.requests,
                   "budget_GB": args.serving_budget, "resident_cap_GB": args.serving_resident_cap,
                   "lanes_per_chain_max": args.serving_lanes, "chains_per_system_max": args.serving_max_chains},
        "footprints_GB": {n: round(probe.footprint(n) / 1e9, 3) for n in names},
        "per_rate": results,
        "chi_max_rel_diff_batched_vs_alone": maxdiff,
    }
    print(json.dumps(out))


def measure_spectra(args, tm, torch, h, begin, coeffs, lanes, prec):
    """Whole spectra, measured: for each flavour, one chain of M steps from its
    set-up to chi on 400 frequencies (0-1.995 eV, eta 5 meV), stepped in
    pieces so that progress is printed."""
    M = args.spectrum_steps
    om = np.arange(400) * 5e-3 / EV
    eta = 5e-3 / EV
    out = {}
    for flavour in args.spectrum_flavours.split(","):
        log(f"spectrum: {flavour} chain of {M} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = begin(M, prec, flavour)
        done = 0
        while done < M:
            k = min(300, M - done)
            tm.tm_chains_step([c], k)
            torch.cuda.synchronize()
            done += k
            log(f"  {done}/{M} steps, {time.perf_counter() - t0:.1f} s")
        co = coeffs(c, M)
        tm.tm_chain_end(c)
        chi = tm.tm_chi(co, max(1, co["steps_done"]), om, eta)
        dt = time.perf_counter() - t0
        assert np.all(np.isfinite(chi))
        applies = lanes * (M + 1 if flavour == "pH" else 2 * M)
        out[flavour] = {"steps": M, "steps_done": int(co["steps_done"]), "breakdown": bool(co["breakdown"]),
                        "seconds": round(dt, 3), "spectra_per_s": round(lanes / dt, 6),
                        "applies_per_s": round(applies / dt, 4),
                        "beta_mean_second_half": float(np.mean(co["beta"][M // 2:co["steps_done"]]))}
        log(f"  {out[flavour]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="hexslab", choices=["hexslab", "cubic20", "qpath", "serving"])
    ap.add_argument("--chain-steps", type=int, default=2000, help="qpath: steps per chain")
    ap.add_argument("--qpath-lanes", type=int, default=24, choices=[1, 3, 6, 12, 24, 72],
                    help="qpath: lanes per chain object (3: the directions of one q set; 6 .. 72: those of "
                         "2 .. 24 q sets, one launch per kernel for all of them)")
    ap.add_argument("--rates", default="0.2,0.5,1", help="serving: Poisson arrival rates (requests/s)")
    ap.add_argument("--requests", type=int, default=20, help="serving: requests per rate")
    ap.add_argument("--serving-budget", type=float, default=48.0,
                    help="serving: device-memory budget in GB (system footprints + chains)")
    ap.add_argument("--serving-resident-cap", type=float, default=16.0,
                    help="serving: largest resident real-space ground state per system, GB")
    ap.add_argument("--serving-systems", default="cubic20,cubic24,cubic32,slab96",
                    help="serving: the systems of the pool that requests are drawn from (their weights kept)")
    ap.add_argument("--serving-lanes", type=int, default=4, choices=[1, 2, 3, 4],
                    help="serving: pending requests of one system, q set and flavour share a chain (lanes)")
    ap.add_argument("--chain-slots", type=int, default=3,
                    help="qpath: concurrent workspace slots for the system's chains")
    ap.add_argument("--serving-chain-slots", type=int, default=1,
                    help="serving: concurrent workspace slots per system (1: its chains on its stream)")
    ap.add_argument("--serving-max-chains", type=int, default=4,
                    help="serving: chains per system at a time (0: no limit); later requests wait and form lanes")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tensor", default="",
                    help="hexslab/cubic20: field directions run together as lanes of one chain "
                         "(e.g. xyz: the 3 x 3 spin tensor in one pass); default: the m_+ chain alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-samples", type=int, default=20)
    ap.add_argument("--spectrum-steps", type=int, default=0,
                    help="hexslab/cubic20: also run whole chains of this many steps with chi (measured spectra/s)")
    ap.add_argument("--spectrum-flavours", default="pH", help="flavours of the measured spectra (pH,nH)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="fp32: single-precision bulk applies (FP64 recurrence); reports the error against FP64")
    ap.add_argument("--no-resident", action="store_true",
                    help="keep the ground state as z-transformed columns instead of resident real-space planes")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        raise SystemExit("bench.py supports --gpus 1 only: the hot path is built and measured on one GPU")

    import torch
    import paper_2203_01120_amd as tm
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    tm.load()
    if args.workload == "qpath":
        return run_qpath(args, tm, torch)
    if args.workload == "serving":
        return run_serving(args, tm, torch)

    log(f"building {args.workload} inputs")
    t0 = time.time()
    inp = build_inputs(args.workload, args.seed)
    log(f"inputs ready in {time.time() - t0:.1f} s ({len(inp['points'])} ground-state points)")
    h = tm.tm_system_create(make_desc(inp))
    info = tm.tm_qset_info_get(h, 0)
    log(f"system created: nk={info['nk']} nbnd={info['nbnd']} npw_pad={info['npw_pad']} "
        f"vector {info['nelem'] * 16 / 1e9:.2f} GB")

    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.no_resident:
        tm.tm_system_set_resident_limit(h, 0)
    prec = tm.TM_FP32 if args.precision == "fp32" else tm.TM_FP64
    dirs = list(args.tensor) if args.tensor else ["+"]
    lanes = len(dirs)

    def begin(cap, p=prec, flavour="pH"):
        if lanes > 1:
            return tm.tm_chain_begin_multi(h, 0, dirs, flavour, cap, p)
        return tm.tm_chain_begin(h, 0, dirs[0], flavour, cap, p)

    def coeffs(c, cap):
        return tm.tm_chain_coeffs_lanes(c, cap)[0] if lanes > 1 else tm.tm_chain_coeffs(c, cap)

    # warm-up: whole step periods (6 pH steps), so that the step graphs are
    # captured before the timed steps start
    W = 6 * max(1, -(-args.warmup // 6))
    K = args.steps
    log(f"chain set-up and {W} warm-up steps ({args.precision}, directions {''.join(dirs)})")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain = begin(W + K)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    tm.tm_chains_step([chain], W)
    torch.cuda.synchronize()
    resident = tm.tm_system_resident_bytes(h)
    log(f"set-up {setup_s * 1e3:.1f} ms; resident real-space ground state: {resident / 1e9:.2f} GB")

    log(f"timed {K} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tm.tm_chains_step([chain], K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = coeffs(chain, W + K)
    tm.tm_chain_end(chain)

    log(f"profiled chain: {K} steps with HIP events around every launch")
    chain = begin(W + K)
    tm.tm_chains_step([chain], W)
    torch.cuda.synchronize()
    tm.tm_profile_reset()
    tm.tm_profile_enable(True)
    t1 = time.perf_counter()
    tm.tm_chains_step([chain], K)
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    tm.tm_profile_enable(False)
    tm.tm_chain_end(chain)
    accuracy = None
    if prec == tm.TM_FP32:   # the same chain in FP64 (untimed): spectrum error of the FP32 bulk path
        m = min(res["steps_done"], W + K)
        ref = (tm.tm_tensor_run(h, 0, dirs, "pH", m, tm.TM_FP64)[0] if lanes > 1 else
               tm.tm_lanczos_run(h, 0, dirs[0], "pH", m, tm.TM_FP64))
        m = min(m, ref["steps_done"])
        om = np.arange(400) * 5e-3 / EV
        eta = 5e-3 / EV
        x32, x64 = tm.tm_chi(res, m, om, eta), tm.tm_chi(ref, m, om, eta)
        accuracy = {"l2_rel_im_chi": float(np.linalg.norm(x32.imag - x64.imag) / np.linalg.norm(x64.imag)),
                    "steps": int(m), "omega": "400 points 0-1.995 eV, eta 5 meV"}
        w0, d = peak_shift(tm, res, ref, m, eta)
        if w0 is not None:
            accuracy.update(peak_shift_meV=d, peak_meV=w0,
                            peak="strongest interior peak of |Im chi| over -10..10 eV, located on a 0.01 meV grid")
        log(f"fp32 vs fp64: {accuracy}")
    prof = {}
    for k, (ms, cnt) in tm.tm_profile_read().items():
        name = k.strip("()").split("<")[0]
        old = prof.get(name, (0.0, 0))
        prof[name] = (old[0] + ms, old[1] + cnt)
    applies = lanes * K
    applies_per_s = applies / dt
    log(f"{K} steps in {dt:.3f} s -> {applies_per_s:.3f} applies/s (profiled run {dt_prof:.3f} s); "
        f"breakdown={res['breakdown']}")

    # per-apply latency (single applies, HIP events on the launch stream)
    lat = []
    n = info["nelem"]
    x = torch.empty(lanes * n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    for r, d in enumerate(dirs):
        tm.tm_start_vectors(h, 0, d, None, x[r * n:(r + 1) * n])
    for _ in range(args.latency_samples):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        tm.tm_liouvillian_apply_multi(h, 0, lanes, x, y, prec)
        e1.record()
        torch.cuda.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.array(lat) if lat else np.array([dt / applies * 1e3])
    del x, y

    models = kernel_models(inp, info, resident > 0, lanes)
    total_ms = sum(v[0] for v in prof.values())
    kernels = {k: {"ms_total": round(v[0], 3), "launches": v[1], "ms_avg": round(v[0] / max(v[1], 1), 4),
                   "share": round(v[0] / total_ms, 4)} for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    avg_s = prof[dom][0] / prof[dom][1] / 1e3
    roof = None
    if dom in models:
        m = models[dom]
        traffic = measured_traffic(dom) if args.workload == "hexslab" else None
        mbytes = m.get("bytes")
        if "flops" in m:
            tflops = m["flops"] / avg_s / 1e12
            alu_peak = FP32_PEAK_TFLOPS if m.get("fp32") else FP64_PEAK_TFLOPS
            roof = {"kernel": dom, "bound": "mfma" if m.get("mfma") else "alu", "achieved": round(tflops, 3),
                    "peak": alu_peak, "unit": "TFLOP/s", "frac": round(tflops / alu_peak, 4)}
            if "flops_pruned" in m:
                roof["frac_pruned_count"] = round(m["flops_pruned"] / avg_s / 1e12 / alu_peak, 4)
                roof["algorithmic_flops_pruned_per_launch"] = m["flops_pruned"]
            roof["algorithmic_flops_per_launch"] = m["flops"]
        else:
            gbs = mbytes / avg_s / 1e9
            roof = {"kernel": dom, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4)}
        roof.update({"traffic": traffic, "avg_ms": round(avg_s * 1e3, 4)})
        if mbytes:
            roof.update({"method_bytes_per_launch": round(mbytes),
                         "hbm_frac": round(mbytes / avg_s / 1e9 / HBM_PEAK_GBS, 5),
                         "traffic_over_method_bytes": None if traffic is None else round(traffic / mbytes, 2)})
    step_s = dt / K
    am = models["apply"]
    step_roof = {"flops_per_step": am["flops"], "method_bytes_per_step": round(am["bytes"]),
                 "fp64_frac" if prec == tm.TM_FP64 else "fp32_frac":
                     round(am["flops"] / step_s / 1e12 / (FP64_PEAK_TFLOPS if prec == tm.TM_FP64 else FP32_PEAK_TFLOPS), 4),
                 "hbm_frac": round(am["bytes"] / step_s / 1e9 / HBM_PEAK_GBS, 5),
                 "note": "the method's work per step (each lane's apply: 12 full-grid transforms per band and k "
                         "+ 2 Hartree, both contractions, point-wise) over the measured step time"}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(args.workload, args.seed, info["nk"])
        log(f"oracle: {cpu['seconds']:.1f} s for the sample")

    spectrum = None
    if args.spectrum_steps:
        spectrum = measure_spectra(args, tm, torch, h, begin, coeffs, lanes, prec)

    sysd = inp["sysd"]
    chain_m = 3000
    out = {
        "metric": "Liouvillian applies/s and chi(q,omega) spectra/s at stated error; p50/p99 latency",
        "value": round(applies_per_s, 4),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(dt / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == tm.TM_FP32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": ("CrI3-monolayer-shaped hexagonal slab, a=13 c=31 bohr, 2+6 Gaussian sites, "
                         "48x48x180 grid, 104 bands, 6x6x1 mesh (36 k), q=b1/6, "
                         if args.workload == "hexslab" else
                         "cubic a=10 bohr, 2 sites, 20^3 grid, 8 bands, Gamma, q=0.1 2pi/a, ") +
                        (f"pH chains of directions {args.tensor} in one pass" if args.tensor else "pH chain m_+"),
            "directions": "".join(dirs),
            "fft": list(sysd.fft), "nbnd": sysd.nbnd, "nk": info["nk"], "npw_pad": info["npw_pad"],
            "nproj": sysd.nproj, "precision": args.precision, "flavour": "pseudo_hermitian",
        },
        "chain_setup_ms": round(setup_s * 1e3, 2),
        "spectra_per_s_derived": round(applies_per_s / (chain_m + 1), 6),
        "spectra_per_s_derived_from": f"applies/s / {chain_m + 1} (a {chain_m}-step pH chain: set-up apply + one per step)",
        "spectrum_measured": spectrum,
        "apply_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                             "p99": round(float(np.percentile(lat, 99)), 3),
                             "what": "single Liouvillian applies (HIP events); request latencies: --workload serving"},
        "resident_ground_bytes": resident,
        "fp32_accuracy": accuracy,
        "roofline": roof,
        "step_roofline": step_roof,
        "kernels": kernels,
        "autotune": tm.tm_autotune_report(),
        "cpu_baseline": cpu,
    }
    tm.tm_system_destroy(h)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
