"""GPU parity at the two larger configurations, where no reference spectrum is
affordable on the CPU: properties that hold at any size, each recomputed on
the CPU with the oracle.

* N = 1e6 (n = 3e6): the FP32-filter form (FP32 block values, vectors and
  accumulation; CholQR2 and Rayleigh-Ritz in FP64; one FP64 refinement
  sweep) against the plain FP64 solve at block 160, on a window holding about
  128 eigenvalues by the oracle's stochastic count
  (golden/glass1m_window.json, written by golden/make_large_windows.py).
  That window is 0.028 % of theta_max wide; at the configured degree 250 the
  filter margins reach far beyond the block's 160 columns, so the solve runs
  at degree 1200.  Checked: the same number of eigenpairs, eigenvalues of the
  two forms within 1e-8 relative of each other, exactly one refinement sweep,
  residuals ||H v - lambda v|| / lambda_ub recomputed with the oracle's BSR
  product, orthonormality, and the count against the estimate (a coarse
  check: few probes, and a damped kernel that blurs the window's ends).
* N = 4e6 (n = 1.2e7), the largest single-GPU instance: Lanczos bounds
  against the oracle, one filter application at block 256 (FP64 and FP32)
  against the oracle on sampled columns, the time per filter step and the
  device memory footprint.
"""
import json
import os
import time

import numpy as np
import pytest

import paper_1902_07041_amd as P
from oracle import cbsr, chebyshev, hessian, lanczos
from synth import gaussian_block, gaussian_vector, lattice_glass

from gpu_common import banner, rel_err

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(__file__)


def check_pairs(H, out, ub, tol, label):
    lam = out["evals"]
    V = np.ascontiguousarray(out["evecs"].T)            # [n, k]
    R = H @ V - V * lam[None, :]
    res = np.linalg.norm(R, axis=0) / ub
    banner(f"{label}: {lam.size} pairs, max residual {res.max():.3e}")
    assert res.max() <= tol
    np.testing.assert_allclose(res, out["resid"], rtol=0.05, atol=1e-3 * tol)
    G = V.T @ V
    assert np.abs(G - np.eye(lam.size)).max() <= 1e-9


class Case1m:
    pass


@pytest.fixture(scope="module")
def glass1m():
    gd = json.load(open(os.path.join(HERE, "golden", "glass1m_window.json")))
    banner(f"glass N={gd['n_atoms']} (drawing)")
    s = Case1m()
    s.gd = gd
    s.g = lattice_glass(gd["n_atoms"], seed=gd["seed"])
    hb = hessian.weight_blocks(s.g.row_ptr, s.g.col_idx, s.g.blocks, s.g.masses)
    s.H = cbsr.BsrOperator(s.g.row_ptr, s.g.col_idx, hb)
    s.h = P.pfe_create(0)
    P.pfe_set_hessian(s.h, s.g.row_ptr, s.g.col_idx, s.g.blocks, s.g.masses)
    s.lb, s.ub, s.th = P.pfe_estimate_bounds(s.h, gd["lanczos_steps"],
                                             gaussian_vector(s.g.n, gd["v0_seed"]))
    s.lo, s.hi = gd["lo_frac"] * s.th, gd["hi_frac"] * s.th
    s.block, s.degree = 160, 1200
    s.X0 = gaussian_block(s.g.n, s.block, 11)
    s.out = {}
    yield s
    P.pfe_destroy(s.h)


def test_config_1m_fp64(glass1m, monkeypatch):
    monkeypatch.setenv("PFEIG_TRACE", "1")               # one line per outer iteration
    s = glass1m
    assert abs(s.th - s.gd["theta_max"]) <= 1e-10 * s.th
    banner(f"N=1e6 FP64 solve, block {s.block}, degree {s.degree}")
    t0 = time.perf_counter()
    r64 = P.pfe_solve_interval(s.h, s.lo, s.hi, s.block, s.block, degree=s.degree, tol=1e-10,
                               x0=s.X0)
    r64["time"] = time.perf_counter() - t0
    s.out["fp64"] = r64
    banner(f"FP64 solve {r64['time']:.1f} s, {r64['evals'].size} pairs, "
           f"{r64['stats']['iterations']} iterations")
    assert r64["status"] == "PFE_OK"
    gd = s.gd
    assert abs(r64["evals"].size - gd["count_estimate"]) <= 4 * gd["count_stderr"] + 0.25 * gd["count_estimate"]
    check_pairs(s.H, r64, s.ub, 1e-10, "FP64")


def test_config_1m_mixed_precision_one_sweep(glass1m, monkeypatch):
    monkeypatch.setenv("PFEIG_TRACE", "1")
    s = glass1m
    if "fp64" not in s.out:
        pytest.skip("needs the FP64 solve")
    r64 = s.out["fp64"]
    banner(f"N=1e6 FP32-filter form, block {s.block}, degree {s.degree}")
    t0 = time.perf_counter()
    r32 = P.pfe_solve_interval(s.h, s.lo, s.hi, s.block, s.block, degree=s.degree, tol=1e-8,
                               x0=s.X0, precision=P.PFE_FP32)
    t32 = time.perf_counter() - t0
    st = r32["stats"]
    mem = P.pfe_device_bytes(s.h)
    banner(f"FP32 form {t32:.1f} s ({st['iterations'] - st['fp64_iterations']} FP32 iterations, "
           f"one sweep of {st['refine_applications']} FP64 applications) against FP64 "
           f"{r64['time']:.1f} s: {r64['time'] / t32:.2f}x; library device memory "
           f"{mem / 2**30:.1f} GiB")
    assert r32["status"] == "PFE_OK", st
    assert st["refined"] == 1 and st["fp64_iterations"] == 1
    assert r32["evals"].size == r64["evals"].size
    rel = np.abs(r32["evals"] - r64["evals"]) / r64["evals"]
    banner(f"max relative eigenvalue difference FP32 form vs FP64: {rel.max():.3e}")
    assert rel.max() <= 1e-8
    check_pairs(s.H, r32, s.ub, 1e-8, "FP32 form")


def test_config_4m_largest_instance():
    import torch
    N, block, d, sample = 4000000, 256, 5, 16
    banner(f"glass N={N} (drawing)")
    g = lattice_glass(N, seed=1)
    hb = hessian.weight_blocks(g.row_ptr, g.col_idx, g.blocks, g.masses)
    H = cbsr.BsrOperator(g.row_ptr, g.col_idx, hb)
    h = P.pfe_create(0)
    try:
        t0 = time.perf_counter()
        P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks, g.masses)
        banner(f"import {time.perf_counter() - t0:.1f} s; bounds")
        v0 = gaussian_vector(g.n, 7)
        lb, ub, th = P.pfe_estimate_bounds(h, 30, v0)
        _, rub, rth = lanczos.lanczos_bounds(H, v0, 30)
        assert abs(th - rth) <= 1e-12 * rth and abs(ub - rub) <= 1e-10 * rub
        f = P.pfe_design_filter(0.003 * th, 0.006 * th, lb, ub, degree=d)
        for dt, tol in [(torch.float64, 1e-12), (torch.float32, 5e-5)]:
            gen = torch.Generator(device="cuda").manual_seed(5)
            X = torch.randn(g.n, block, dtype=dt, device="cuda", generator=gen)
            Y = torch.empty_like(X)
            P.pfe_apply_filter(h, f, X, Y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.pfe_apply_filter(h, f, X, Y)
            torch.cuda.synchronize()
            step = (time.perf_counter() - t0) / d
            Xs = X[:, :sample].double().cpu().numpy()
            ref = chebyshev.apply_filter(H, f.c, f.e, f.coef, Xs)
            err = rel_err(Y[:, :sample].double().cpu().numpy(), ref)
            banner(f"{str(dt)[-7:]} q={block}: {step * 1e3:.2f} ms per step, sampled columns "
                   f"rel err {err:.2e}")
            assert err < tol
            del X, Y
        mem = P.pfe_device_bytes(h)
        banner(f"library device memory {mem / 2**30:.1f} GiB (H, tile copy, FP32 copy, workspaces)")
        assert mem < 288 * 2**30
    finally:
        P.pfe_destroy(h)
