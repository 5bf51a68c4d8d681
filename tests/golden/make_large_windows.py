"""Writes glass1m_window.json: a window of the mass-weighted Hessian of the
1 000 000-atom synthetic glass (seed 1) that holds about the requested number
of eigenvalues, located and counted by the CPU oracle alone.  Nothing here
touches the HIP library.

At these sizes no dense or exact count is affordable, so the count is the
stochastic estimate of Sec. 2.4 (eq. eigval_count_estimator) from Chebyshev
moments (K moments, Jackson damping) of M Gaussian probes, one probe at a
time so that the spread of the per-probe counts gives the estimate's standard
error.  The window starts at the configuration's lower end (a fraction of
theta_max, the largest Ritz value of a 30-step Lanczos run from
gaussian_vector(n, 7)); its upper end is moved until the estimate reaches the
configuration's nev.

Run:  python tests/golden/make_large_windows.py   (about 20 min on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import cbsr, count, filters as F, hessian, lanczos  # noqa: E402
from synth import gaussian_block, gaussian_vector, lattice_glass  # noqa: E402

SPECS = {
    "1m": dict(n_atoms=1000000, seed=1, lanczos_steps=30, v0_seed=7, lo_frac=0.005, nev=128,
               moments=1500, probes=8, probe_seed=13),
}


def main(tag):
    s = SPECS[tag]
    t0 = time.time()
    g = lattice_glass(s["n_atoms"], seed=s["seed"])
    hb = hessian.weight_blocks(g.row_ptr, g.col_idx, g.blocks, g.masses)
    H = cbsr.BsrOperator(g.row_ptr, g.col_idx, hb)
    lb, ub, th = lanczos.lanczos_bounds(H, gaussian_vector(g.n, s["v0_seed"]), s["lanczos_steps"])
    print(f"[{tag}] bounds {lb} {ub} {th} ({time.time() - t0:.0f} s)", flush=True)
    c, e = F.spectral_map(lb, ub)
    V = gaussian_block(g.n, s["probes"], s["probe_seed"])
    mus = []
    for l in range(s["probes"]):
        mus.append(count.chebyshev_moments(H, c, e, V[:, l:l + 1], s["moments"]))
        print(f"[{tag}] probe {l} done ({time.time() - t0:.0f} s)", flush=True)
    lo = s["lo_frac"] * th

    def est(hi):
        xi, eta = (lo - c) / e, (hi - c) / e
        per = np.array([count.count_from_moments(mu, g.n, xi, eta) for mu in mus])
        return float(per.mean()), float(per.std(ddof=1) / np.sqrt(len(per)))

    a, b = lo, 2.0 * lo
    while est(b)[0] < s["nev"]:
        a, b = b, 2.0 * b
    for _ in range(60):
        m = 0.5 * (a + b)
        if est(m)[0] < s["nev"]:
            a = m
        else:
            b = m
    hi = b
    mean, se = est(hi)
    doc = {
        "_about": "Window holding about nev eigenvalues by the oracle's stochastic count; written "
                  "by make_large_windows.py",
        **s, "theta_max": th, "lam_ub": ub, "lo": lo, "hi": hi, "hi_frac": hi / th,
        "count_estimate": mean, "count_stderr": se,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"glass{tag}_window.json")
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"[{tag}] wrote {path}: hi/theta {hi / th:.6f}, count {mean:.1f} +- {se:.1f} "
          f"({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    for tag in (sys.argv[1:] or ["1m"]):
        main(tag)
