#!/usr/bin/env python3
"""Benchmark of the polynomial-filtered interior eigensolver on one MI355X.

One step is one pass of the whole hot path over the resident synthetic input
(a spring-network glass of N = 100,000 atoms, n = 300,000, 3x3 FP64 blocks):

  a1  assemble K from the springs, mass-weight, validate   SpringSystem.assemble
      (pfe_set_springs, device inputs; differentiable in k and m)
  a2  30-step Lanczos bounds                               pfe_estimate_bounds
  a3  filter design (degree 400)                           pfe_design_filter
  a4  one filter application Y = p(H_hat) X at q = 96       pfe_apply_filter
      (its launches are the roofline measurement)
  a3-a7  FP64 solve: Chebyshev filter (Clenshaw) with locking, CholQR2,
      Rayleigh-Ritz, residuals -> all eigenpairs in the window
  a8  the same solve with the FP32 filter + one FP64 refinement sweep
  a9  reverse mode through torch.autograd: L = <dY, p(H_hat) X> (block 64,
      degree 150, sqrt(d) checkpoints) back to X, every spring constant and
      mass; Hellmann-Feynman gradient of the 32 lowest eigenvalues found,
      chain rule to springs and masses

Prints one JSON line (see --help).  `value` is the wall time of one step in
seconds (lower is better); the FP64 and FP32-form solve times, the filter
kernel's achieved HBM bandwidth and its roofline fraction are reported beside
it, with the CPU oracle's cost for the FP64 solve estimated from a bounded
sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
WORKLOAD = {
    "name": "glass-N100000-fp64-q96",
    "n_atoms": 100_000,
    "seed": 1,
    "block": 96,
    "degree": 400,
    # window as fractions of theta_max of the 30-step Lanczos run; both edges
    # sit in spectral gaps (68 eigenvalues inside)
    "win": (0.006611, 0.007430),
    "nev": 96,
    "tol64": 1e-10,
    "tol32": 1e-8,
    "adj_block": 64,
    "adj_degree": 150,
    "hf_count": 32,
}


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_1902_07041_amd", "csrc", "k_sparse.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_from_profile(q: int, degree: int):
    """HBM bytes per filter launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "k1_fp64_q96_glass100k_traffic.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(g, H_bounds, stats64, W):
    """The oracle (its plain C block-CSR product on all host cores, numpy QR and
    eigh) timed on a bounded sample of the FP64 solve: a few Chebyshev steps
    and one orthonormalisation + Rayleigh-Ritz pass at the full size, scaled
    by the step and iteration counts of the GPU solve (the oracle iteration
    converges in the same number of iterations, without locking)."""
    import numpy as np
    from oracle import cbsr, chebyshev, hessian, subspace
    from synth import gaussian_block
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    hb = hessian.weight_blocks(g.row_ptr, g.col_idx, g.blocks, g.masses)
    H = cbsr.BsrOperator(g.row_ptr, g.col_idx, hb)
    lb, ub = H_bounds
    c, e = 0.5 * (ub + lb), 0.5 * (ub - lb)
    q = W["block"]
    X = gaussian_block(g.n, q, 11)
    ksteps = 8
    coef = np.ones(ksteps + 1)
    chebyshev.apply_filter(H, c, e, coef[:2], X)          # first call loads the library
    t0 = time.perf_counter()
    chebyshev.apply_filter(H, c, e, coef, X)
    t_steps = (time.perf_counter() - t0) / ksteps
    t0 = time.perf_counter()
    Q, _ = np.linalg.qr(X)
    subspace.rayleigh_ritz(H, Q)
    t_orth_rr = time.perf_counter() - t0
    est = t_steps * stats64["filter_steps"] + t_orth_rr * stats64["iterations"]
    return {
        "value": est, "unit": "s", "cores": threads, "kind": "oracle",
        "sample": (f"{ksteps} Chebyshev steps (oracle C block-CSR product, {threads} OpenMP "
                   f"threads) and one Householder QR + Rayleigh-Ritz on n={g.n}, q={q}, timed "
                   f"({t_steps:.3f} s/step, {t_orth_rr:.3f} s/iteration) and scaled to the "
                   f"GPU FP64 solve's {stats64['filter_steps']} steps and "
                   f"{stats64['iterations']} iterations"),
    }


def extras(P, sysm, g, last, W, X0):
    """One timed run each of the solver variants beyond the benchmark step."""
    import numpy as np
    import torch
    h = sysm.h
    lo, hi, th = last["lo"], last["hi"], last["theta_max"]
    ev64 = last["o64"]["evals"]
    res = {}
    print("[bench] extras: Lanczos on the Dirac filter", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    o = P.pfe_solve_lanczos(h, lo, hi, W["nev"], block=32, max_basis=224, tol=W["tol64"])
    t = time.perf_counter() - t0
    st = o["stats"]
    res["lanczos_dirac"] = {
        "block": 32, "max_basis": 224, "phi": 0.8, "degree": st["degree"], "seconds": t,
        "restart_cycles": st["iterations"], "filter_steps": st["filter_steps"],
        "filter_columns": st["filter_columns"], "n_found": int(o["evals"].size),
        "max_resid": float(o["resid"].max()),
        "max_rel_eig_diff_vs_si": float(np.max(np.abs(o["evals"] - ev64) / ev64))
        if o["evals"].shape == ev64.shape else None}
    print("[bench] extras: FP64 solve without locking", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    o = P.pfe_solve_interval(h, lo, hi, W["nev"], W["block"], degree=W["degree"], tol=W["tol64"],
                             x0=X0, locking=0, vectors_on_device=True)
    res["fp64_no_locking"] = {"seconds": time.perf_counter() - t0,
                              "iterations": o["stats"]["iterations"],
                              "filter_columns": o["stats"]["filter_columns"]}
    print("[bench] extras: count estimate", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    cnt = P.pfe_estimate_count(h, lo, hi, 1000, P.PFE_SMOOTH_JACKSON, nsamples=32, seed=13)
    res["count_estimate"] = {"window_count": int(ev64.size), "estimate": cnt, "degree": 1000,
                             "probes": 32, "seconds": time.perf_counter() - t0}
    lo2, hi2 = 0.005 * th, 0.015 * th
    print("[bench] extras: sliced solve of [0.5%, 1.5%] theta_max", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    o = P.pfe_solve_sliced(h, lo2, hi2, 1024, W["block"], per_slice=48, tol=W["tol64"],
                           want_vectors=True, vectors_on_device=True)
    t = time.perf_counter() - t0
    V = o["evecs"]
    G = (V @ V.T.contiguous()).cpu().numpy() if V is not None and V.shape[0] else np.zeros((0, 0))
    res["sliced_literal_window"] = {
        "window_frac_theta": [0.005, 0.015], "seconds": t, "n_found": int(o["evals"].size),
        "n_slices": o["n_slices"], "iterations_total": o["stats"]["iterations"],
        "filter_steps": o["stats"]["filter_steps"], "max_resid": float(o["resid"].max()),
        "max_offdiag_overlap": float(np.abs(G - np.eye(G.shape[0])).max()) if G.size else None}
    return res


def copy_calibration() -> int:
    """Device-to-device copy of 2 GiB (reads 2 GiB, writes 2 GiB per copy):
    the scale for FETCH_SIZE / WRITE_SIZE counters and the achievable copy
    bandwidth."""
    import torch
    nbytes = 2 * 2**30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    print(json.dumps({"copy_bytes": nbytes, "seconds_per_copy": t,
                      "copy_GBps_read_plus_write": 2 * nbytes / t / 1e9}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", action="store_true",
                    help="after the timed steps, also time the rows beyond the hot path once: "
                         "thick-restart Lanczos on the Dirac filter, spectrum slicing of the "
                         "literal window [0.5%%, 1.5%%] theta_max, locking off, the count estimate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 2 GiB device buffer 5 times and print the copy bandwidth "
                         "(the reference for the HBM traffic counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this library has no "
              "multi-GPU path (a slab decomposition with halo exchange is designed, not built)",
              file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import paper_1902_07041_amd as P
    from synth import gaussian_block, gaussian_vector, lattice_glass

    W = WORKLOAD
    t_gen = time.perf_counter()
    g = lattice_glass(W["n_atoms"], seed=W["seed"])
    n = g.n
    print(f"[bench] generated {W['name']}: nnzb={g.nnzb} in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    from paper_1902_07041_amd.autograd import SpringSystem

    dev = torch.device("cuda:0")
    k0 = torch.from_numpy(g.k).to(dev)
    m0 = torch.from_numpy(g.masses).to(dev)
    v0 = torch.from_numpy(gaussian_vector(n, 7)).to(dev)
    X0 = torch.from_numpy(gaussian_block(n, W["block"], 11)).to(dev)
    Xa0 = torch.from_numpy(gaussian_block(n, W["adj_block"], 21)).to(dev)
    Ya = torch.from_numpy(gaussian_block(n, W["adj_block"], 22)).to(dev)
    sysm = SpringSystem(g.row_ptr, g.col_idx, g.pairs, g.unit)
    h = sysm.h
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)     # the library's stream (pfe_create takes torch's)

    def step():
        r = {}
        k = k0.clone().requires_grad_()
        m = m0.clone().requires_grad_()
        Xa = Xa0.clone().requires_grad_()
        t0 = time.perf_counter()
        Hb = sysm.assemble(k, m)
        t1 = time.perf_counter()
        lb, ub, th = P.pfe_estimate_bounds(h, 30, v0)
        t2 = time.perf_counter()
        lo, hi = W["win"][0] * th, W["win"][1] * th
        f = P.pfe_design_filter(lo, hi, lb, ub, degree=W["degree"])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.pfe_apply_filter(h, f, X0)
        e1.record(stream)
        t3 = time.perf_counter()
        o64 = P.pfe_solve_interval(h, lo, hi, W["nev"], W["block"], degree=W["degree"],
                                   tol=W["tol64"], x0=X0, vectors_on_device=True)
        t4 = time.perf_counter()
        o32 = P.pfe_solve_interval(h, lo, hi, W["nev"], W["block"], degree=W["degree"],
                                   tol=W["tol32"], x0=X0, precision=P.PFE_FP32,
                                   vectors_on_device=True)
        t5 = time.perf_counter()
        fa = P.pfe_design_filter(lo, hi, lb, ub, degree=W["adj_degree"])
        loss = (Ya * sysm.filter(Xa, Hb, fa)).sum()
        loss.backward()
        V = o64["evecs"][: W["hf_count"]].contiguous()
        G = P.pfe_eigvec_block_gradient(h, V, g.nnzb)
        dk, dm = P.pfe_spring_gradient(h, sysm.pairs, sysm.unit, G, g.n_atoms)
        torch.cuda.synchronize()
        t6 = time.perf_counter()
        r.update(t_hessian=t1 - t0, t_bounds=t2 - t1, t_a4=e0.elapsed_time(e1) / 1e3,
                 t_fp64=t4 - t3, t_fp32=t5 - t4, t_adjoint=t6 - t5, lam_lb=lb, lam_ub=ub,
                 theta_max=th, lo=lo, hi=hi, o64=o64, o32=o32, dk=dk, dm=dm,
                 dk_filter=k.grad, dm_filter=m.grad, lam_hf=o64["evals"][: W["hf_count"]],
                 a4_degree=f.degree)
        return r

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last = res[-1]
    o64, o32 = last["o64"], last["o32"]
    s64, s32 = o64["stats"], o32["stats"]

    def med(key):
        return float(np.median([r[key] for r in res]))

    # dominant kernel: the fused Chebyshev/Clenshaw step, measured on the a4
    # application (d launches at q = 96, HIP events on the library's stream).
    # Algorithmic bytes per launch, averaged over the application: matrix
    # (values + column indices) and row pointers every launch, and 4d - 3
    # multivector streams (2 in the first launch, 3 in the second, 4 after).
    q, d = W["block"], last["a4_degree"]
    mat = g.nnzb * (9 * 8 + 4) + 8 * (g.n_atoms + 1)
    vec = n * q * 8
    bytes_per_launch = mat + vec * (4 * d - 3) / d
    avg_launch = med("t_a4") / d
    achieved = bytes_per_launch / avg_launch / 1e9
    ev64, ev32 = o64["evals"], o32["evals"]
    rel32 = float(np.max(np.abs(ev32 - ev64) / np.abs(ev64))) if ev32.shape == ev64.shape else None
    dk = last["dk"].cpu().numpy()
    dm = last["dm"].cpu().numpy()
    lam_sum = float(np.sum(last["lam_hf"]))
    out = {
        "metric": "time-to-nev eigenpairs in window + filter HBM GB/s, FP64 vs FP32-filter @res<=1e-8",
        "value": elapsed / args.steps,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": W["name"], "n_atoms": W["n_atoms"], "n": n, "nnzb": g.nnzb,
                   "block": q, "degree": d, "window_frac_theta": list(W["win"]),
                   "nev_found": int(ev64.size), "parallelism": "single-gpu"},
        "time_to_solution_fp64_s": med("t_fp64"),
        "time_to_solution_fp32_form_s": med("t_fp32"),
        "fp32_form_speedup": med("t_fp64") / med("t_fp32"),
        "t_set_hessian_s": med("t_hessian"),
        "t_bounds_s": med("t_bounds"),
        "t_adjoint_and_gradients_s": med("t_adjoint"),
        "t_a4_filter_s": med("t_a4"),
        "orthogonalisation_mfma": {
            "kernels": "k_gram_small + k_gram_reduce (Gram), k_gemm_bres (X R^-1, X Q, W Q); FP64 MFMA",
            "flops": s64["gemm_flops"], "seconds": s64["t_gemm"],
            "achieved_TFLOPs": s64["gemm_flops"] / s64["t_gemm"] / 1e12 if s64["t_gemm"] else None,
            "peak_TFLOPs": 78.6,
            "frac": s64["gemm_flops"] / s64["t_gemm"] / 78.6e12 if s64["t_gemm"] else None},
        "fp64": {"n_found": int(ev64.size), "iterations": s64["iterations"],
                 "filter_steps": s64["filter_steps"], "filter_columns": s64["filter_columns"],
                 "max_resid": float(np.max(o64["resid"])),
                 "t_filter": s64["t_filter"], "filter_GBps": s64["filter_bytes"] / s64["t_filter"] / 1e9,
                 "t_orth": s64["t_orth"], "t_rr": s64["t_rr"],
                 "t_resid": s64["t_resid"], "eps": s64["eps"]},
        "fp32_form": {"n_found": int(ev32.size), "iterations": s32["iterations"],
                      "refined": s32["refined"], "filter_steps": s32["filter_steps"],
                      "filter_columns": s32["filter_columns"],
                      "max_resid": float(np.max(o32["resid"])) if ev32.size else None,
                      "max_rel_eig_diff_vs_fp64": rel32, "t_filter": s32["t_filter"],
                      "filter_GBps": s32["filter_bytes"] / s32["t_filter"] / 1e9},
        "gradients": {"sum_k_dlam_dk_over_sum_lam": float(np.dot(g.k, dk)) / lam_sum,
                      "sum_m_dlam_dm_over_sum_lam": float(np.dot(g.masses, dm)) / lam_sum,
                      "filter_loss_grad_norm_k": float(last["dk_filter"].norm()),
                      "filter_loss_grad_norm_m": float(last["dm_filter"].norm())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profile(q, d),
                     "kernel": "k_cheb_tile<double,2,1,2,2> (fused BSR3 Clenshaw step, 2-row tiles), "
                               "the a4 application's launches",
                     "avg_launch_us": 1e6 * avg_launch,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    if args.extras:
        out["extras"] = extras(P, sysm, g, last, W, X0)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, (last["lam_lb"], last["lam_ub"]), s64, W)
    sysm.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
