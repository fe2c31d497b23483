"""Writes fp32_bound.json: the single-precision error model run on the oracle.

For the cubic 20^3 system (oracle SCF ground state, q = 0.1 2pi/a) and the two
chains the GPU single-precision test runs (pseudo-Hermitian m_+ and
non-Hermitian m_z, 60 steps), eight seeded perturbed chains are compared
with the unperturbed one (tests/fp32_noise.py states the model).  The bounds
the GPU test asserts are twice the largest value over the seeds, and for the
peak shift at least the 0.01 meV resolution of the peak search.

    python tests/golden/make_fp32_bound.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

SEEDS = list(range(1, 9))
CHAINS = [("pH", "+"), ("nH", "z")]
M = 60


def main():
    import synth
    import fp32_noise as fn
    from oracle import liouvillian as lv
    from oracle import scf
    gs = scf.scf(synth.make_cubic20(), tol=1e-10, beta=0.5)
    prob = lv.build_problem(gs, np.array([0.1, 0.0, 0.0]) * 2 * np.pi / 10.0)
    out = {"system": "cubic a=10 bohr, 20^3 grid, 8 bands, Gamma, q=0.1 2pi/a (oracle SCF)",
           "model": "every apply returns L x + delta, ||delta|| = 2^-24 Lam ||x||, random direction",
           "steps": M, "seeds": SEEDS, "chains": {}}
    for flavour, mu in CHAINS:
        ref = fn.chain(prob, mu, flavour, M)
        rows = []
        for s in SEEDS:
            got = fn.chain(prob, mu, flavour, M, seed=s)
            assert got["steps_done"] == ref["steps_done"] == M
            l2, shift = fn.spectrum_error(ref, got, M)
            rows.append({"seed": s, "l2_rel_im_chi": l2, "peak_shift_meV": shift})
            print(flavour, mu, s, f"{l2:.3e}", shift, flush=True)
        l2max = max(r["l2_rel_im_chi"] for r in rows)
        shifts = [r["peak_shift_meV"] for r in rows if r["peak_shift_meV"] is not None]
        shmax = max(shifts) if shifts else None
        out["chains"][f"{flavour}{mu}"] = {
            "per_seed": rows, "l2_max": l2max, "l2_median": float(np.median([r["l2_rel_im_chi"] for r in rows])),
            "peak_shift_max_meV": shmax,
            "bound_l2": float(f"{2.0 * l2max:.1e}"),
            # no interior peak (the longitudinal chain's spectrum only falls off): no peak bound
            "bound_peak_shift_meV": None if shmax is None else max(0.01, float(f"{2.0 * shmax:.2g}")),
        }
    with open(os.path.join(HERE, "fp32_bound.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
