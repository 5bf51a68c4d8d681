"""Writes glass100k_window.json: the eigenvalues of the mass-weighted Hessian
of the 100 000-atom synthetic glass (seed 1) inside the benchmark window,
computed by the CPU oracle alone (Lanczos bounds, piecewise-quadratic filter of
degree 400, filtered subspace iteration with Householder QR and Rayleigh-Ritz
on H, residual tolerance 1e-12).  Nothing here touches the HIP library.

The window is [0.006611, 0.007430] * theta_max, where theta_max is the largest
Ritz value of a 30-step Lanczos run from gaussian_vector(n, 7); both ends lie
in gaps of the spectrum, so the count is insensitive to rounding of theta_max.

Run:  python tests/golden/make_glass100k_window.py   (about 30 min on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import cbsr, filters as F, hessian, lanczos, subspace  # noqa: E402
from synth import gaussian_block, gaussian_vector, lattice_glass  # noqa: E402

SPEC = dict(n_atoms=100000, seed=1, lanczos_steps=30, v0_seed=7, win=(0.006611, 0.007430),
            degree=400, r=0.1 ** 0.25, block=96, x0_seed=11, tol=1e-12)


def main(out_path):
    s = SPEC
    t0 = time.time()
    g = lattice_glass(s["n_atoms"], seed=s["seed"])
    hb = hessian.weight_blocks(g.row_ptr, g.col_idx, g.blocks, g.masses)
    H = cbsr.BsrOperator(g.row_ptr, g.col_idx, hb)
    lb, ub, th = lanczos.lanczos_bounds(H, gaussian_vector(g.n, s["v0_seed"]), s["lanczos_steps"])
    lo, hi = s["win"][0] * th, s["win"][1] * th
    c, e = F.spectral_map(lb, ub)
    xi, eta = (lo - c) / e, (hi - c) / e
    eps = F.eps_rule(xi, eta, s["degree"], s["r"])
    coef = F.filter_coefficients(xi, eta, eps, s["degree"])
    X0 = gaussian_block(g.n, s["block"], s["x0_seed"])

    def cb(it, theta, res):
        inw = (theta >= lo) & (theta <= hi)
        print(f"it {it}: in-window {int(inw.sum())}, max resid {res[inw].max() if inw.any() else 0:.3e}"
              f"  ({time.time() - t0:.0f} s)", flush=True)

    lam, X, res, it = subspace.subspace_iteration(H, c, e, coef, X0, lo, hi, ub, tol=s["tol"],
                                                  callback=cb)
    doc = {
        "_about": "Eigenvalues of the mass-weighted Hessian in the window, from the CPU oracle "
                  "only; written by make_glass100k_window.py",
        **{k: list(v) if isinstance(v, tuple) else v for k, v in s.items()},
        "theta_max": th, "lam_ub": ub, "lo": lo, "hi": hi, "eps": eps,
        "iterations": it, "max_resid": float(res.max()) if res.size else 0.0,
        "count": int(lam.size), "evals": [float(x) for x in lam],
    }
    with open(out_path, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {out_path}: {lam.size} eigenvalues, {it} iterations, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main(os.path.join(os.path.dirname(os.path.abspath(__file__)), "glass100k_window.json"))
