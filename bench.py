#!/usr/bin/env python3
"""Benchmark of the polynomial-filtered interior eigensolver on one MI355X.

Workload: the largest single-GPU instance, a spring-network glass of
N = 4,000,000 atoms (n = 12,000,000; 70.8 M stored 3x3 FP64 blocks), block
q = 256, filter degree 300, window [0.3 %, 0.314 %] of theta_max (the lower
end of the configured [0.3 %, 0.6 %], its upper end moved so that the window
holds about nev = 200 eigenvalues by the low-frequency density of states of
this glass).  Inputs are resident in HBM before timing.

One step is one pass of the hot path:

  a1  assemble K from the springs, mass-weight, validate   SpringSystem.assemble
      (pfe_set_springs on device arrays)
  a2  30-step Lanczos bounds                               pfe_estimate_bounds
  a3-a7  one outer iteration of the FP64 method: filter design, Y = p(H_hat) X
      (300 fused Clenshaw steps at q = 256), CholQR2, Rayleigh-Ritz on H,
      residuals (pfe_solve_interval with max_iter 1; its filter launches are
      the roofline measurement)
  a8  one outer iteration of the FP32-filter form: FP32 H_hat formed from the
      new H, FP32 filter, FP64 CholQR2, Rayleigh-Ritz and residuals
  a9  the differentiation form on its own instance (N = 100,000 glass, block
      64, degree 150, window [0.5 %, 1.5 %] theta_max): L = <W, p(H_hat) X>
      through torch.autograd back to X, every spring constant and mass, with
      the adjoint recomputing each ceil(sqrt(d))-step segment from
      checkpoints; Hellmann-Feynman gradient of the 32 lowest eigenvalues of
      a solved window and its chain rule to springs and masses

`value` is the FP32-filter form's time per outer iteration on the 4e6-atom
instance (seconds, lower is better; median over the steps); the FP64 form's
time per iteration, their ratio, the filter's HBM bandwidth and roofline
fraction, the orthogonalisation's MFMA rate, and the time-to-solution of both
forms on the 1e5-atom instance (measured once, before the timed steps) are
reported beside it.  `cpu_baseline` is the CPU oracle's time per FP64 outer
iteration on the 4e6-atom instance, extrapolated from a bounded sample timed
on the host cores.
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
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix, published
WORKLOAD = {
    "name": "glass-N4000000-q256-d300",
    "n_atoms": 4_000_000,
    "seed": 1,
    "block": 256,
    "degree": 300,
    "win": (0.003, 0.00314),
    "win_configured": (0.003, 0.006),
    "nev": 256,
    "tol64": 1e-10,
    "tol32": 1e-8,
    "x0_seed": 11,
}
DIFF = {
    "name": "glass-N100000-q64-d150",
    "n_atoms": 100_000,
    "seed": 1,
    "block": 64,
    "degree": 150,
    "win": (0.005, 0.015),
    "x_seed": 21,
    "w_seed": 22,
    # window of the 1e5-atom glass solved once for the Hellmann-Feynman
    # gradient and the time-to-solution keys: 68 eigenvalues, both ends in
    # spectral gaps (degree 400 puts the filter margins inside the gaps)
    "solve_win": (0.006611, 0.007430),
    "solve_block": 96,
    "solve_degree": 400,
    "hf_count": 32,
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the filter kernel's source and of the row orders its tiles are
    built in (both decide its memory traffic)."""
    h = hashlib.sha256()
    for f in ("k_sparse.hip", "reorder.cpp"):
        h.update(open(os.path.join(ROOT, "paper_1902_07041_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


# the FP64 filter's kernel at the benchmark shape: three-row tiles (one record
# per batch) of the wide-block tile set, two 128-column passes per launch
K64_INSTANCE = "k_cheb_tile<double, 2, 1, 1, 3>"


def traffic_from_profile():
    """HBM bytes per FP64 filter launch at the benchmark shape from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source and kernel instance."""
    p = os.path.join(ROOT, "profiles", "k1_fp64_q256_glass4m_traffic.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if d.get("kernel_instance") != K64_INSTANCE:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(g, bounds, degree):
    """The CPU oracle's time per FP64 outer iteration on this instance,
    extrapolated from a timed sample on the host cores: two Chebyshev steps of
    the oracle's C block-CSR product at 64 columns (scaled to 256; the step is
    bound by the 3q-element neighbour rows it gathers), and Householder QR plus
    the Rayleigh-Ritz products on a tenth of the rows (scaled to all rows;
    their cost is linear in n)."""
    import numpy as np
    from oracle import cbsr, chebyshev, hessian
    from synth import gaussian_block
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    hb = hessian.weight_blocks(g.row_ptr, g.col_idx, g.blocks, g.masses)
    H = cbsr.BsrOperator(g.row_ptr, g.col_idx, hb)
    lb, ub = bounds
    c, e = 0.5 * (ub + lb), 0.5 * (ub - lb)
    qs, q = 64, WORKLOAD["block"]
    X = gaussian_block(g.n, qs, 11)
    H @ X[:, :1]                                               # loads the library
    t0 = time.perf_counter()
    chebyshev.apply_filter(H, c, e, np.ones(3), X)             # two steps
    t_step = (time.perf_counter() - t0) / 2 * (q / qs)
    del X
    rows = g.n // 10
    Xs = gaussian_block(rows, q, 12)
    t0 = time.perf_counter()
    Qs, _ = np.linalg.qr(Xs)
    S = Qs.T @ Xs                  # X^T W, with W of the same shape
    _, U = np.linalg.eigh(0.5 * (S + S.T))
    Qs @ U
    Xs @ U
    t_orth_rr = (time.perf_counter() - t0) * (g.n / rows)
    est = degree * t_step + t_step + t_orth_rr             # filter, W = H X, QR + RR
    return {
        "value": est, "unit": "s per FP64 outer iteration", "cores": threads, "kind": "oracle",
        "sample": (f"extrapolated: 2 Chebyshev steps of the oracle's C block-CSR product "
                   f"({threads} OpenMP threads) at 64 of the 256 columns, scaled to 256 "
                   f"({t_step:.2f} s per step), and Householder QR + Rayleigh-Ritz products "
                   f"(numpy) on {rows} of the {g.n} rows, scaled to all rows "
                   f"({t_orth_rr:.1f} s); one iteration = {degree} steps + W = H X + QR + RR"),
    }


def solver_variants(P, h, lo, hi, th, X0, ev64, D, W):
    """One timed run each of the solver variants beyond the benchmark step on
    the 1e5-atom instance: the FP64 solve without locking, the stochastic
    count, thick-restart block Lanczos on the Dirac filter, and spectrum
    slicing of the configured window [0.5 %, 1.5 %] theta_max."""
    import numpy as np
    import torch
    res = {}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = fn()
        torch.cuda.synchronize()
        return o, time.perf_counter() - t0

    log("variants: FP64 solve without locking")
    o, t = timed(lambda: P.pfe_solve_interval(h, lo, hi, D["solve_block"], D["solve_block"],
                                              degree=D["solve_degree"], tol=W["tol64"], x0=X0,
                                              locking=0, vectors_on_device=True))
    res["fp64_no_locking"] = {"seconds": t, "iterations": o["stats"]["iterations"],
                              "filter_columns": o["stats"]["filter_columns"],
                              "n_found": int(o["evals"].size)}
    log("variants: count estimate")
    cnt, t = timed(lambda: P.pfe_estimate_count(h, lo, hi, 1000, P.PFE_SMOOTH_JACKSON,
                                                nsamples=32, seed=13))
    res["count_estimate"] = {"window_count": int(ev64.size), "estimate": cnt, "degree": 1000,
                             "probes": 32, "seconds": t}
    log("variants: Lanczos on the Dirac filter")
    o, t = timed(lambda: P.pfe_solve_lanczos(h, lo, hi, D["solve_block"], block=32,
                                             max_basis=224, tol=W["tol64"]))
    st = o["stats"]
    res["lanczos_dirac"] = {
        "block": 32, "max_basis": 224, "phi": 0.8, "degree": st["degree"], "seconds": t,
        "restart_cycles": st["iterations"], "filter_columns": st["filter_columns"],
        "n_found": int(o["evals"].size), "max_resid": float(o["resid"].max()),
        "max_rel_eig_diff_vs_subspace_iteration":
            float(np.max(np.abs(o["evals"] - ev64) / ev64)) if o["evals"].shape == ev64.shape else None}
    log("variants: sliced solve of [0.5%, 1.5%] theta_max")
    o, t = timed(lambda: P.pfe_solve_sliced(h, 0.005 * th, 0.015 * th, 1024, D["solve_block"],
                                            per_slice=48, tol=W["tol64"], want_vectors=True,
                                            vectors_on_device=True))
    V = o["evecs"]
    G = (V @ V.T.contiguous()).cpu().numpy() if V is not None and V.shape[0] else np.zeros((0, 0))
    res["sliced_configured_window"] = {
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
    ap.add_argument("--variants", action="store_true",
                    help="also time the solver variants (no locking, count, Lanczos, slicing) "
                         "on the 1e5-atom instance and add them to the line")
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
    from paper_1902_07041_amd.autograd import SpringSystem
    from synth import gaussian_block, gaussian_vector, lattice_glass

    W, D = WORKLOAD, DIFF
    dev = torch.device("cuda:0")
    # the library runs on this stream (pfe_create takes torch's current
    # stream), so events recorded on it bracket the library's launches
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)

    t_gen = time.perf_counter()
    g = lattice_glass(W["n_atoms"], seed=W["seed"])
    n = g.n
    log(f"generated {W['name']}: nnzb={g.nnzb} in {time.perf_counter() - t_gen:.1f}s")
    g4 = lattice_glass(D["n_atoms"], seed=D["seed"])
    log(f"generated {D['name']}: nnzb={g4.nnzb}")

    sysm = SpringSystem(g.row_ptr, g.col_idx, g.pairs, g.unit)
    h = sysm.h
    k0 = torch.from_numpy(g.k).to(dev)
    m0 = torch.from_numpy(g.masses).to(dev)
    v0 = torch.from_numpy(gaussian_vector(n, 7)).to(dev)
    gen = torch.Generator(device=dev).manual_seed(W["x0_seed"])
    X0 = torch.randn((n, W["block"]), dtype=torch.float64, device=dev, generator=gen)

    sys4 = SpringSystem(g4.row_ptr, g4.col_idx, g4.pairs, g4.unit)
    h4 = sys4.h
    k4 = torch.from_numpy(g4.k).to(dev)
    m4 = torch.from_numpy(g4.masses).to(dev)
    Xa = torch.from_numpy(gaussian_block(g4.n, D["block"], D["x_seed"])).to(dev)
    Wa = torch.from_numpy(gaussian_block(g4.n, D["block"], D["w_seed"])).to(dev)

    # once, before the timed steps: the 1e5-atom instance's bounds, the
    # time-to-solution of both forms on its solved window, and the
    # eigenvectors whose eigenvalues the Hellmann-Feynman gradient follows
    H4 = sys4.assemble(k4, m4)
    lb4, ub4, th4 = P.pfe_estimate_bounds(h4, 30, torch.from_numpy(gaussian_vector(g4.n, 7)).to(dev))
    slo, shi = D["solve_win"][0] * th4, D["solve_win"][1] * th4
    S0 = torch.from_numpy(gaussian_block(g4.n, D["solve_block"], 11)).to(dev)
    tts = {}
    for form, prec, tol in (("fp64", P.PFE_FP64, W["tol64"]), ("fp32_form", P.PFE_FP32, W["tol32"])):
        for rep in range(2):                 # the first run also builds the FP32 tiles and copy
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = P.pfe_solve_interval(h4, slo, shi, D["solve_block"], D["solve_block"],
                                     degree=D["solve_degree"], tol=tol, x0=S0, precision=prec,
                                     vectors_on_device=True)
            t = time.perf_counter() - t0
        tts[form] = (t, o)
    ev64, ev32 = tts["fp64"][1]["evals"], tts["fp32_form"][1]["evals"]
    variants = solver_variants(P, h4, slo, shi, th4, S0, ev64, D, W) if args.variants else None
    V_hf = tts["fp64"][1]["evecs"][: D["hf_count"]].contiguous()
    lam_hf = ev64[: D["hf_count"]]
    c4, e4 = 0.5 * (ub4 + lb4), 0.5 * (ub4 - lb4)
    fa = P.pfe_design_filter(D["win"][0] * th4, D["win"][1] * th4, lb4, ub4, degree=D["degree"])
    log(f"N=1e5 window of {ev64.size}: FP64 {tts['fp64'][0]:.3f} s, FP32 form "
        f"{tts['fp32_form'][0]:.3f} s")

    # once, before the timed steps: the 4e6-atom pattern's row tiles of both
    # filters at this block width (built at a filter's first call on a
    # pattern and kept while it stays), so that every timed step, also with
    # --warmup 0, is a steady outer iteration
    with torch.no_grad():
        sysm.assemble(k0, m0)
    lbp, ubp, thp = P.pfe_estimate_bounds(h, 30, v0)
    fp = P.pfe_design_filter(W["win"][0] * thp, W["win"][1] * thp, lbp, ubp, degree=1)
    for dt in (torch.float64, torch.float32):
        Xp = X0.to(dt)
        P.pfe_apply_filter(h, fp, Xp, torch.empty_like(Xp))
        del Xp
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("tile sets of both filters built")

    def step():
        r = {}
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        with torch.no_grad():
            sysm.assemble(k0, m0)                                           # a1
        lb, ub, th = P.pfe_estimate_bounds(h, 30, v0)                       # a2
        lo, hi = W["win"][0] * th, W["win"][1] * th
        ev[1].record(stream)
        o64 = P.pfe_solve_interval(h, lo, hi, W["nev"], W["block"], degree=W["degree"],  # a3-a7
                                   tol=W["tol64"], x0=X0, max_iter=1, want_vectors=False,
                                   allow_noconv=True)
        ev[2].record(stream)
        o32 = P.pfe_solve_interval(h, lo, hi, W["nev"], W["block"], degree=W["degree"],  # a8
                                   tol=W["tol32"], x0=X0, max_iter=1, precision=P.PFE_FP32,
                                   want_vectors=False, allow_noconv=True)
        ev[3].record(stream)
        k = k4.clone().requires_grad_()                                     # a9
        m = m4.clone().requires_grad_()
        Xg = Xa.clone().requires_grad_()
        Hb = sys4.assemble(k, m)
        loss = (Wa * sys4.filter(Xg, Hb, fa)).sum()
        loss.backward()
        G = P.pfe_eigvec_block_gradient(h4, V_hf, g4.nnzb)
        dk, dm = P.pfe_spring_gradient(h4, sys4.pairs, sys4.unit, G, g4.n_atoms)
        ev[4].record(stream)
        stream.synchronize()
        t1 = time.perf_counter()
        r.update(wall=t1 - t0, t_a12=ev[0].elapsed_time(ev[1]) / 1e3,
                 t_it64=ev[1].elapsed_time(ev[2]) / 1e3, t_it32=ev[2].elapsed_time(ev[3]) / 1e3,
                 t_a9=ev[3].elapsed_time(ev[4]) / 1e3, lam_lb=lb, lam_ub=ub, theta_max=th,
                 o64=o64, o32=o32, dk=dk, dm=dm, dk_filter=k.grad, dm_filter=m.grad)
        return r

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for i in range(args.steps):
        res.append(step())
        log(f"step {i + 1}/{args.steps}: {res[-1]['wall']:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last = res[-1]
    s64, s32 = last["o64"]["stats"], last["o32"]["stats"]

    def med(key):
        return float(np.median([r[key] for r in res]))

    def med_stat(form, key):
        return float(np.median([r[form]["stats"][key] for r in res]))

    # dominant kernel: the fused FP64 Clenshaw step (K64_INSTANCE, two
    # 128-column passes per launch at q = 256), in the FP64 iteration's
    # filter: its launches are timed by the library with HIP events on this
    # stream.  Algorithmic bytes per launch as in the method's fused step
    # (Algorithm 2 with a running sum): matrix values, column indices and
    # row pointers once, five multivector streams of n q elements.
    q, d = W["block"], W["degree"]
    bstep = g.nnzb * (9 * 8 + 4) + 4 * (g.n_atoms + 1) + 5 * n * q * 8
    clen = g.nnzb * (9 * 8 + 4) + 8 * (g.n_atoms + 1) + (4 - 3 / d) * n * q * 8
    launch64 = med_stat("o64", "t_filter") / s64["filter_steps"]
    launch32 = med_stat("o32", "t_filter") / s32["filter_steps"]
    bstep32 = g.nnzb * (9 * 4 + 4) + 4 * (g.n_atoms + 1) + 5 * n * q * 4
    achieved = bstep / launch64 / 1e9
    dk = last["dk"].cpu().numpy()
    dm = last["dm"].cpu().numpy()
    lam_sum = float(np.sum(lam_hf))
    t64, t32 = med("t_it64"), med("t_it32")
    s64_2, s32_2 = tts["fp64"][1]["stats"], tts["fp32_form"][1]["stats"]
    out = {
        "metric": "time-to-nev eigenpairs in window + filter HBM GB/s, FP64 vs FP32-filter @res<=1e-8",
        "value": t32,
        "value_is": "FP32-filter form, seconds per outer iteration (FP32 filter of degree 300 at "
                    "q = 256, FP64 CholQR2, Rayleigh-Ritz and residuals) on the 4e6-atom glass",
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 filter, f64 orthogonalisation",
        "data": "synthetic",
        "config": {"workload": W["name"], "n_atoms": W["n_atoms"], "n": n, "nnzb": g.nnzb,
                   "block": q, "degree": d, "window_frac_theta": list(W["win"]),
                   "window_configured_frac_theta": list(W["win_configured"]),
                   "differentiation_workload": D["name"], "parallelism": "single-gpu"},
        "fp64_s_per_iteration": t64,
        "fp32_form_s_per_iteration": t32,
        "fp32_form_speedup_per_iteration": t64 / t32,
        "filter_fp64": {"ms_per_step": 1e3 * launch64, "GBps_algorithmic": bstep / launch64 / 1e9,
                        "frac_of_peak": bstep / launch64 / 1e9 / HBM_PEAK_GBS},
        "filter_fp32": {"ms_per_step": 1e3 * launch32,
                        "GBps_algorithmic": bstep32 / launch32 / 1e9,
                        "frac_of_peak": bstep32 / launch32 / 1e9 / HBM_PEAK_GBS,
                        "note": "filter phase incl. the FP64<->FP32 casts of the block"},
        "t_assembly_and_bounds_s": med("t_a12"),
        "t_adjoint_and_gradients_s": med("t_a9"),
        "device_bytes_library": P.pfe_device_bytes(h),
        "device_bytes_torch_peak": int(torch.cuda.max_memory_allocated(dev)),
        "orthogonalisation_mfma": {
            "kernels": "k_gram_rt + k_gram_reduce (Gram; 2 n q^2 flops each, the symmetric ones form 3 of 4 tiles), k_gemm_rt (X R^-1, X Q, W Q); FP64 MFMA",
            "flops": s64["gemm_flops"], "seconds": med_stat("o64", "t_gemm"),
            "achieved_TFLOPs": s64["gemm_flops"] / med_stat("o64", "t_gemm") / 1e12,
            "peak_TFLOPs": FP64_MFMA_PEAK_TFLOPS,
            "frac": s64["gemm_flops"] / med_stat("o64", "t_gemm") / 1e12 / FP64_MFMA_PEAK_TFLOPS},
        "time_to_solution_N1e5": {
            "window_frac_theta": list(D["solve_win"]), "block": D["solve_block"],
            "degree": D["solve_degree"], "n_found": int(ev64.size),
            "fp64_s": tts["fp64"][0], "fp32_form_s": tts["fp32_form"][0],
            "fp32_form_speedup": tts["fp64"][0] / tts["fp32_form"][0],
            "fp64_iterations": s64_2["iterations"],
            "fp32_form_iterations": s32_2["iterations"],
            "fp32_form_refinement_sweeps": s32_2["refined"],
            "fp32_form_refinement_applications": s32_2["refine_applications"],
            "max_rel_eig_diff_fp32_form_vs_fp64":
                float(np.max(np.abs(ev32 - ev64) / ev64)) if ev32.shape == ev64.shape else None,
            "max_resid_fp64": float(np.max(tts["fp64"][1]["resid"])),
            "max_resid_fp32_form": float(np.max(tts["fp32_form"][1]["resid"]))},
        "gradients_N1e5": {"sum_k_dlam_dk_over_sum_lam": float(np.dot(g4.k, dk)) / lam_sum,
                           "sum_m_dlam_dm_over_sum_lam": float(np.dot(g4.masses, dm)) / lam_sum,
                           "filter_loss_grad_norm_k": float(last["dk_filter"].norm()),
                           "filter_loss_grad_norm_m": float(last["dm_filter"].norm()),
                           "adjoint": "ceil(sqrt(150)) = 13-step checkpoint segments, recomputed"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profile(),
                     "kernel": K64_INSTANCE + " (fused BSR3 Clenshaw step, three-row tiles, "
                               "two 128-column passes), the FP64 iteration's 300 launches",
                     "avg_launch_us": 1e6 * launch64,
                     "algorithmic_bytes_per_launch": bstep,
                     "clenshaw_stream_bytes_per_launch": clen,
                     "frac_on_clenshaw_bytes": clen / launch64 / 1e9 / HBM_PEAK_GBS},
    }
    if variants is not None:
        out["solver_variants_N1e5"] = variants
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample on the host cores)")
        out["cpu_baseline"] = cpu_baseline(g, (last["lam_lb"], last["lam_ub"]), d)
    sys4.close()
    sysm.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
