"""Writes glass100k_cfg4_fd.json: central finite differences, step 1e-6, of the
filter loss L(k) = <W, p(H_hat) X> in 50 seeded spring constants of the
100 000-atom synthetic glass (seed 1), computed by the CPU oracle alone.
Nothing here touches the HIP library.

The differentiation configuration: window [0.5 %, 1.5 %] * theta_max (theta_max
the largest Ritz value of a 30-step Lanczos run from gaussian_vector(n, 7)),
the piecewise-quadratic filter of degree 150 with its margin by eq. thresh
(r = 0.1^(1/4), no damping), block 64 (X and W Gaussian, seeds 21 and 22), c
and e held constant.  The springs are a seeded sample (seed 17) without
replacement.  Each quotient [L(k+h) - L(k-h)] / (2h) comes from
oracle.adjoint.spring_loss_central_difference, which forms the difference of
the two recurrences directly so that FP64 cancellation between the two
losses does not swamp the quotient at this size.  The filter coefficients
are stored so the library is compared on exactly this filter.

Run:  python tests/golden/make_cfg4_fd.py   (about 40 min on 8 cores;
partial results are kept in the output and a rerun resumes)
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import adjoint, cbsr, filters as F, hessian, lanczos  # noqa: E402
from synth import gaussian_block, gaussian_vector, lattice_glass  # noqa: E402

SPEC = dict(n_atoms=100000, seed=1, lanczos_steps=30, v0_seed=7, win=(0.005, 0.015), degree=150,
            r=0.1 ** 0.25, block=64, x_seed=21, w_seed=22, sample_seed=17, n_sample=50, h=1e-6)


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
    Hhat = cbsr.BsrOperator(g.row_ptr, g.col_idx,
                            hessian.mapped_blocks(g.row_ptr, g.col_idx, hb, c, e))
    X = gaussian_block(g.n, s["block"], s["x_seed"])
    W = gaussian_block(g.n, s["block"], s["w_seed"])
    springs = np.random.default_rng(s["sample_seed"]).choice(g.k.shape[0], s["n_sample"],
                                                             replace=False)
    doc = {
        "_about": "Central differences of <W, p(H_hat) X> in 50 spring constants, from the CPU "
                  "oracle only; written by make_cfg4_fd.py",
        **{k: list(v) if isinstance(v, tuple) else v for k, v in s.items()},
        "theta_max": th, "lam_lb": lb, "lam_ub": ub, "lo": lo, "hi": hi, "c": c, "e": e,
        "xi": xi, "eta": eta, "eps": eps, "coef": [float(v) for v in coef],
        "springs": [int(p) for p in springs], "fd": [],
    }
    if os.path.exists(out_path):
        old = json.load(open(out_path))
        if old.get("springs") == doc["springs"] and old.get("coef") == doc["coef"]:
            doc["fd"] = old.get("fd", [])
    for p in springs[len(doc["fd"]):]:
        i, j = int(g.pairs[p, 0]), int(g.pairs[p, 1])
        quot = adjoint.spring_loss_central_difference(Hhat.__matmul__, e, coef, X, W, i, j,
                                                      g.unit[p], g.masses[i], g.masses[j], s["h"])
        doc["fd"].append(float(quot))
        with open(out_path + ".tmp", "w") as fh:
            json.dump(doc, fh, indent=1)
        os.replace(out_path + ".tmp", out_path)
        print(f"spring {p} ({i}, {j}): {quot:.15e}  [{len(doc['fd'])}/{len(springs)}, "
              f"{time.time() - t0:.0f} s]", flush=True)
    print(f"wrote {out_path}: {len(doc['fd'])} quotients, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main(os.path.join(os.path.dirname(os.path.abspath(__file__)), "glass100k_cfg4_fd.json"))
