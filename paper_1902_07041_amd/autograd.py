"""torch.autograd Functions over the library's hand-written reverse modes.

    AssembleSprings    (k, masses) -> H blocks [nnzb,3,3]
                       backward: chain rule through H_ij = K_ij / sqrt(m_i m_j)
                       with K_ij = -k u u^T (pfe_spring_gradient)
    ChebFilter         (X, H blocks) -> p_d(H_hat) X  (Algorithm 2's operator)
                       backward: adjoint recurrence over checkpoint segments of
                       ceil(sqrt(d)) steps, recomputing each segment's forward
                       vectors (pfe_apply_filter_adjoint; `resident` keeps them
                       on the device instead), giving dX and dL/dH per block
    WindowEigenvalues  H blocks -> eigenvalues of H in [lo, hi] (and their
                       eigenvectors, not differentiable)
                       backward: Hellmann-Feynman, dL/dH = sum_s (dL/dlam_s) v_s v_s^T
                       (pfe_eigvec_block_gradient)

Each forward and each backward is one library call on the GPU; torch holds
the device memory and orders the calls on its current stream.  The filter's
c, e and coefficients, the window and the solver options are constants.

A SpringSystem binds one library handle to one spring network's pattern.  The
handle holds one Hessian at a time: a Function whose H blocks are not the ones
the handle holds reloads them first (pfe_set_hessian with the blocks as H), so
forward and backward always run on the H they were given.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _capi as C


class SpringSystem:
    """A spring network on one GPU: BSR pattern (row_ptr, col_idx), springs
    (pairs [P,2] int64 with i < j in increasing order, unit vectors [P,3]);
    spring constants and masses are the differentiable parameters."""

    def __init__(self, row_ptr, col_idx, pairs, unit, device: int = 0):
        dev = torch.device("cuda", device)
        t = lambda a, dt: torch.as_tensor(np.asarray(a), dtype=dt).to(dev).contiguous()  # noqa: E731
        self.device = dev
        self.row_ptr = t(row_ptr, torch.int64)
        self.col_idx = t(col_idx, torch.int32)
        self.pairs = t(pairs, torch.int64)
        self.unit = t(unit, torch.float64)
        self.n_atoms = int(self.row_ptr.shape[0]) - 1
        self.nnzb = int(self.col_idx.shape[0])
        self.n = 3 * self.n_atoms
        self.h = C.pfe_create(device)
        self._held = None          # (H blocks tensor, its version, masses) the handle holds

    def close(self) -> None:
        if self.h is not None:
            C.pfe_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- which H the handle holds
    def _holds(self, hblocks) -> bool:
        # the held tensor is kept referenced, so its storage cannot be reused
        if self._held is None:
            return False
        held, version, _ = self._held
        return (held.data_ptr() == hblocks.data_ptr() and held.shape == hblocks.shape
                and version == hblocks._version)

    def _load(self, hblocks, masses) -> None:
        if not self._holds(hblocks):
            C.pfe_set_hessian(self.h, self.row_ptr, self.col_idx, hblocks.detach().contiguous(),
                              None if masses is None else masses.detach().contiguous(),
                              blocks_are_h=True)
            self._held = (hblocks, hblocks._version, masses)

    # -- differentiable calls
    def assemble(self, k, masses):
        """H blocks of the network with spring constants k [P] and masses [N]."""
        return AssembleSprings.apply(k, masses, self)

    def filter(self, X, hblocks, f: C.Filter, ckpt_stride: int = 0, resident: bool = False):
        """p_d(H_hat) X for the filter f, X [n, q] on this GPU.  The backward
        pass recomputes the forward vectors from checkpoints every ckpt_stride
        steps (0: ceil(sqrt(d))); resident=True keeps them instead when they
        fit in device memory (same results)."""
        return ChebFilter.apply(X, hblocks, self, f, ckpt_stride, resident)

    def window_eigenvalues(self, hblocks, lam_lo, lam_hi, nev, block, bounds, **solve_kw):
        """(eigenvalues [m], eigenvectors [m, n]) of H in [lam_lo, lam_hi]; bounds
        = (lam_lb, lam_ub) of the spectrum for the spectral map."""
        return WindowEigenvalues.apply(hblocks, self, lam_lo, lam_hi, nev, block, bounds, solve_kw)

    def estimate_bounds(self, hblocks, steps: int = 30, v0=None, seed: int = 7):
        self._load(hblocks, self._held[2] if self._held else None)
        return C.pfe_estimate_bounds(self.h, steps, v0, seed)


class AssembleSprings(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k, masses, sysm: SpringSystem):
        k = k.detach().contiguous()
        masses = masses.detach().contiguous()
        H = C.pfe_set_springs(sysm.h, sysm.row_ptr, sysm.col_idx, sysm.pairs, sysm.unit, k, masses,
                              want_blocks=True)
        sysm._held = (H, H._version, masses)
        ctx.sysm = sysm
        ctx.save_for_backward(H, masses)
        return H

    @staticmethod
    def backward(ctx, dH):
        sysm = ctx.sysm
        H, masses = ctx.saved_tensors
        sysm._load(H, masses)
        dk, dm = C.pfe_spring_gradient(sysm.h, sysm.pairs, sysm.unit, dH.contiguous(), sysm.n_atoms)
        return dk, dm, None


class ChebFilter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, hblocks, sysm: SpringSystem, f: C.Filter, ckpt_stride: int,
                resident: bool = False):
        sysm._load(hblocks, sysm._held[2] if sysm._held else None)
        X = X.detach().contiguous()
        Y = C.pfe_apply_filter(sysm.h, f, X)
        ctx.sysm, ctx.f, ctx.stride, ctx.resident = sysm, f, ckpt_stride, resident
        ctx.save_for_backward(X, hblocks)
        return Y

    @staticmethod
    def backward(ctx, dY):
        sysm = ctx.sysm
        X, hblocks = ctx.saved_tensors
        sysm._load(hblocks, sysm._held[2] if sysm._held else None)
        dX, dH = C.pfe_apply_filter_adjoint(sysm.h, ctx.f, X, dY.contiguous(), sysm.nnzb, ctx.stride,
                                            resident=ctx.resident)
        return (dX if ctx.needs_input_grad[0] else None,
                dH if ctx.needs_input_grad[1] else None, None, None, None, None)


class WindowEigenvalues(torch.autograd.Function):
    @staticmethod
    def forward(ctx, hblocks, sysm: SpringSystem, lam_lo, lam_hi, nev, block, bounds, solve_kw):
        sysm._load(hblocks, sysm._held[2] if sysm._held else None)
        C.pfe_set_bounds(sysm.h, float(bounds[0]), float(bounds[1]))
        x0 = solve_kw.get("x0")
        if x0 is not None and not isinstance(x0, torch.Tensor):
            solve_kw = dict(solve_kw, x0=torch.as_tensor(np.ascontiguousarray(x0)).to(sysm.device))
        out = C.pfe_solve_interval(sysm.h, lam_lo, lam_hi, nev, block, vectors_on_device=True,
                                   **solve_kw)
        lam = torch.as_tensor(out["evals"], dtype=torch.float64).to(sysm.device)
        V = out["evecs"]
        ctx.sysm = sysm
        ctx.V = V
        ctx.mark_non_differentiable(V)
        ctx.set_materialize_grads(False)
        return lam, V

    @staticmethod
    def backward(ctx, dlam, dV):
        if dV is not None and bool(torch.any(dV != 0)):
            raise RuntimeError("eigenvector gradients are not provided; differentiate eigenvalues only")
        if dlam is None:
            return (None,) * 8
        sysm = ctx.sysm
        if ctx.V.shape[0] == 0:
            return (torch.zeros(sysm.nnzb, 3, 3, dtype=torch.float64, device=sysm.device),) + (None,) * 7
        dH = C.pfe_eigvec_block_gradient(sysm.h, ctx.V, sysm.nnzb, dlam.contiguous())
        return (dH, None, None, None, None, None, None, None)
