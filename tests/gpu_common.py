"""Shared helpers for the GPU parity tests (inputs from synth, references from oracle)."""
import sys

import numpy as np

import paper_1902_07041_amd as P
from oracle import hessian
from synth import lattice_glass


def banner(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


class GlassCase:
    def __init__(self, n_atoms: int, seed: int = 1, dense: bool = True):
        self.g = lattice_glass(n_atoms, seed=seed)
        self.H, self.hb = hessian.glass_H(self.g)
        self.n = self.g.n
        if dense:
            self.lam, self.U = np.linalg.eigh(self.H.toarray())

    def handle(self):
        h = P.pfe_create(0)
        P.pfe_set_hessian(h, self.g.row_ptr, self.g.col_idx, self.g.blocks, self.g.masses)
        return h


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
