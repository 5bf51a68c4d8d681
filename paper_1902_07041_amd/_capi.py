"""ctypes declarations of include/pfeig.h and argument marshalling."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

PFE_DEVICE_PTRS = 1
PFE_BLOCKS_ARE_H = 2
PFE_ADJOINT_RESIDENT = 4
PFE_SMOOTH_NONE, PFE_SMOOTH_JACKSON, PFE_SMOOTH_LANCZOS = 0, 1, 2
PFE_FP64, PFE_FP32 = 0, 1
STATUS = {0: "PFE_OK", -1: "PFE_EINVAL", -2: "PFE_ENOTSYM", -3: "PFE_ENOMEM", -4: "PFE_EHIP",
          -5: "PFE_ENOCONV", -6: "PFE_ECAPACITY", -7: "PFE_EBOUNDS", -8: "PFE_ESTATE",
          -9: "PFE_EBREAKDOWN"}


class PfeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class CFilterOpts(C.Structure):
    _fields_ = [("degree", C.c_int32), ("eps", C.c_double), ("r", C.c_double),
                ("smoothing", C.c_int32)]


class CFilter(C.Structure):
    _fields_ = [("degree", C.c_int32), ("smoothing", C.c_int32), ("c", C.c_double),
                ("e", C.c_double), ("xi", C.c_double), ("eta", C.c_double), ("eps", C.c_double),
                ("coef", C.POINTER(C.c_double))]


class CSolveOpts(C.Structure):
    _fields_ = [("block", C.c_int32), ("degree", C.c_int32), ("eps", C.c_double),
                ("r", C.c_double), ("smoothing", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("precision", C.c_int32), ("seed", C.c_uint64),
                ("x0", C.c_void_p), ("flags", C.c_uint32), ("locking", C.c_int32),
                ("refine_sweeps", C.c_int32)]


class CDiracFilter(C.Structure):
    _fields_ = [("degree", C.c_int32), ("smoothing", C.c_int32), ("c", C.c_double), ("e", C.c_double),
                ("xi", C.c_double), ("eta", C.c_double), ("gamma", C.c_double), ("tau", C.c_double),
                ("peak", C.c_double), ("coef", C.c_void_p)]


class CLanczosOpts(C.Structure):
    _fields_ = [("block", C.c_int32), ("max_basis", C.c_int32), ("degree", C.c_int32),
                ("phi", C.c_double), ("smoothing", C.c_int32), ("tol", C.c_double),
                ("max_restarts", C.c_int32), ("seed", C.c_uint64), ("flags", C.c_uint32)]


class CSliceOpts(C.Structure):
    _fields_ = [("n_slices", C.c_int32), ("per_slice", C.c_int32), ("margin", C.c_double),
                ("count_degree", C.c_int32), ("count_samples", C.c_int32), ("count_seed", C.c_uint64),
                ("cuts", C.c_void_p)]


class CSolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("fp64_iterations", C.c_int32), ("refined", C.c_int32),
                ("degree", C.c_int32), ("eps", C.c_double), ("c", C.c_double), ("e", C.c_double),
                ("xi", C.c_double), ("eta", C.c_double), ("filter_steps", C.c_int64),
                ("filter_bytes", C.c_double), ("t_total", C.c_double), ("t_filter", C.c_double),
                ("t_orth", C.c_double), ("t_rr", C.c_double), ("t_resid", C.c_double),
                ("gemm_flops", C.c_double), ("max_resid", C.c_double), ("n_window", C.c_int32),
                ("filter_columns", C.c_int64), ("t_gemm", C.c_double),
                ("shifted_passes", C.c_int32), ("refine_applications", C.c_int32)]


_lib = None
_N = {}   # matrix order per handle, for output allocation


def lib_path() -> str:
    return os.path.join(_HERE, "libpfeig.so")


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    p = lib_path()
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built (python -m paper_1902_07041_amd.build); "
                           "there is no fallback path")
    # PyTorch-ROCm ships its own HIP runtime.  Loading torch first makes the
    # library bind to that same runtime (one HIP runtime per process); loaded
    # the other way round the process holds two runtimes and the second one
    # finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(p)
    vp, i32, i64, u32, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    pd = C.POINTER(C.c_double)
    L.pfe_version.restype = C.c_char_p
    L.pfe_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    L.pfe_destroy.argtypes = [vp]
    L.pfe_destroy.restype = None
    L.pfe_last_error.argtypes = [vp]
    L.pfe_last_error.restype = C.c_char_p
    L.pfe_device_bytes.argtypes = [vp]
    L.pfe_device_bytes.restype = i64
    L.pfe_set_hessian.argtypes = [vp, i64, i64, vp, vp, vp, vp, u32]
    L.pfe_set_springs.argtypes = [vp, i64, i64, vp, vp, i64, vp, vp, vp, vp, vp, u32]
    L.pfe_estimate_bounds.argtypes = [vp, i32, vp, u64, u32, pd, pd, pd]
    L.pfe_set_bounds.argtypes = [vp, dbl, dbl]
    L.pfe_design_filter.argtypes = [dbl, dbl, dbl, dbl, C.POINTER(CFilterOpts), pd, i32,
                                    C.POINTER(CFilter)]
    L.pfe_apply_filter.argtypes = [vp, C.POINTER(CFilter), i32, vp, vp, i64, i32, u32]
    L.pfe_apply_filter_noalloc.argtypes = [vp, C.POINTER(CFilter), i32, vp, vp, i64]
    L.pfe_apply_filter_adjoint.argtypes = [vp, C.POINTER(CFilter), i32, vp, vp, vp, vp, i64, i32,
                                           u32]
    L.pfe_eigvec_block_gradient.argtypes = [vp, i32, vp, vp, vp, u32]
    L.pfe_spring_gradient.argtypes = [vp, i64, vp, vp, vp, vp, vp, u32]
    L.pfe_solve_opts_default.argtypes = [C.POINTER(CSolveOpts)]
    L.pfe_solve_opts_default.restype = None
    L.pfe_solve_interval.argtypes = [vp, dbl, dbl, i32, C.POINTER(CSolveOpts), C.POINTER(i32), vp,
                                     vp, vp, C.POINTER(CSolveStats)]
    L.pfe_estimate_count.argtypes = [vp, dbl, dbl, i32, i32, i32, vp, u64, u32, pd]
    L.pfe_solve_sliced.argtypes = [vp, dbl, dbl, i32, C.POINTER(CSolveOpts), C.POINTER(CSliceOpts),
                                   C.POINTER(i32), vp, vp, vp, C.POINTER(i32), vp, i32,
                                   C.POINTER(CSolveStats)]
    L.pfe_count_moments.argtypes = [vp, i32, i32, vp, u64, u32, vp]
    L.pfe_design_dirac.argtypes = [dbl, dbl, dbl, dbl, i32, dbl, i32, vp, i32, C.POINTER(CDiracFilter)]
    L.pfe_locality_order.argtypes = [i64, i64, vp, vp, i32, i32, i64, vp, C.POINTER(dbl), C.POINTER(dbl)]
    L.pfe_lanczos_opts_default.argtypes = [C.POINTER(CLanczosOpts)]
    L.pfe_lanczos_opts_default.restype = None
    L.pfe_solve_lanczos.argtypes = [vp, dbl, dbl, i32, C.POINTER(CLanczosOpts), C.POINTER(i32), vp,
                                    vp, vp, C.POINTER(CSolveStats)]
    for name in ("pfe_create", "pfe_set_hessian", "pfe_set_springs", "pfe_estimate_bounds", "pfe_set_bounds",
                 "pfe_design_filter", "pfe_apply_filter", "pfe_apply_filter_noalloc",
                 "pfe_apply_filter_adjoint",
                 "pfe_eigvec_block_gradient", "pfe_spring_gradient", "pfe_solve_interval",
                 "pfe_estimate_count", "pfe_solve_sliced", "pfe_count_moments", "pfe_design_dirac",
                 "pfe_solve_lanczos"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


# ------------------------------------------------------------- marshalling
def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _arr(a, dtype, name):
    """(pointer, on_device) of a numpy array or a torch tensor; checks dtype and layout."""
    if a is None:
        return None, None
    if _is_torch(a):
        import torch
        tdt = {np.float64: torch.float64, np.float32: torch.float32, np.int64: torch.int64,
               np.int32: torch.int32}[dtype]
        if a.dtype != tdt or not a.is_contiguous():
            raise TypeError(f"{name}: need a contiguous {tdt} tensor")
        return a.data_ptr(), a.is_cuda
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
        raise TypeError(f"{name}: need a C-contiguous numpy array of {np.dtype(dtype)}")
    return a.ctypes.data, False


def _same_side(*flags):
    fl = [f for f in flags if f is not None]
    if fl and any(f != fl[0] for f in fl):
        raise TypeError("array arguments of one call must all be host or all device")
    return bool(fl and fl[0])


def _check(h, st):
    if st != 0:
        L = load_library()
        msg = L.pfe_last_error(h).decode() if h else ""
        raise PfeError(st, msg)


def _empty_like_side(ref, shape, dtype):
    if _is_torch(ref):
        import torch
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        return torch.empty(shape, dtype=tdt, device=ref.device)
    return np.empty(shape, dtype=dtype)


# ------------------------------------------------------------------ calls
def pfe_version() -> str:
    return load_library().pfe_version().decode()


def pfe_create(device: int = 0, stream=None):
    """Handle on `device`.  stream: a hipStream_t as int, or None for torch's
    current stream on that device.  Torch's default stream (handle 0) is not
    passed: the library then runs on its own blocking stream, which is ordered
    against the legacy default stream, so tensors torch is still writing there
    are complete before the library reads them."""
    L = load_library()
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                stream = torch.cuda.current_stream(device).cuda_stream
        except Exception:
            stream = None
    h = C.c_void_p()
    st = L.pfe_create(device, C.c_void_p(stream) if stream else None, C.byref(h))
    if st != 0:
        raise PfeError(st, "pfe_create: " + L.pfe_last_error(None).decode())
    return h


def pfe_destroy(h) -> None:
    load_library().pfe_destroy(h)


def pfe_last_error(h) -> str:
    return load_library().pfe_last_error(h).decode()


def pfe_device_bytes(h) -> int:
    return int(load_library().pfe_device_bytes(h))


def pfe_set_hessian(h, row_ptr, col_idx, blocks, masses=None, blocks_are_h=False) -> None:
    L = load_library()
    n_atoms = int(row_ptr.shape[0]) - 1
    nnzb = int(col_idx.shape[0])
    p_rp, d1 = _arr(row_ptr, np.int64, "row_ptr")
    p_ci, d2 = _arr(col_idx, np.int32, "col_idx")
    p_bl, d3 = _arr(blocks, np.float64, "blocks")
    p_m, d4 = _arr(masses, np.float64, "masses")
    dev = _same_side(d1, d2, d3, d4)
    flags = (PFE_DEVICE_PTRS if dev else 0) | (PFE_BLOCKS_ARE_H if blocks_are_h else 0)
    _check(h, L.pfe_set_hessian(h, n_atoms, nnzb, p_rp, p_ci, p_bl, p_m, flags))
    _N[h.value] = 3 * n_atoms


def pfe_set_springs(h, row_ptr, col_idx, pairs, unit, k, masses, want_blocks=False):
    """Spring-network Hessian assembled on the device; returns H's blocks
    ([nnzb,3,3], on the inputs' side) when want_blocks."""
    L = load_library()
    n_atoms = int(row_ptr.shape[0]) - 1
    nnzb = int(col_idx.shape[0])
    P = int(pairs.shape[0])
    out = _empty_like_side(k, (nnzb, 3, 3), np.float64) if want_blocks else None
    p_rp, d1 = _arr(row_ptr, np.int64, "row_ptr")
    p_ci, d2 = _arr(col_idx, np.int32, "col_idx")
    p_pr, d3 = _arr(pairs, np.int64, "pairs")
    p_un, d4 = _arr(unit, np.float64, "unit")
    p_k, d5 = _arr(k, np.float64, "k")
    p_m, d6 = _arr(masses, np.float64, "masses")
    p_o, d7 = _arr(out, np.float64, "hblocks")
    dev = _same_side(d1, d2, d3, d4, d5, d6, d7)
    _check(h, L.pfe_set_springs(h, n_atoms, nnzb, p_rp, p_ci, P, p_pr, p_un, p_k, p_m, p_o,
                                PFE_DEVICE_PTRS if dev else 0))
    _N[h.value] = 3 * n_atoms
    return out


def pfe_estimate_bounds(h, steps: int = 30, v0=None, seed: int = 7):
    """(lam_lb, lam_ub, theta_max)."""
    L = load_library()
    p_v, dv = _arr(v0, np.float64, "v0")
    lb, ub, th = C.c_double(), C.c_double(), C.c_double()
    _check(h, L.pfe_estimate_bounds(h, steps, p_v, seed, PFE_DEVICE_PTRS if dv else 0,
                                    C.byref(lb), C.byref(ub), C.byref(th)))
    return lb.value, ub.value, th.value


def pfe_set_bounds(h, lam_lb: float, lam_ub: float) -> None:
    _check(h, load_library().pfe_set_bounds(h, lam_lb, lam_ub))


@dataclass
class Filter:
    """A designed filter: the C struct plus the coefficient array it points to."""
    degree: int
    smoothing: int
    c: float
    e: float
    xi: float
    eta: float
    eps: float
    coef: np.ndarray

    def cstruct(self) -> CFilter:
        self.coef = np.ascontiguousarray(self.coef, dtype=np.float64)
        return CFilter(self.degree, self.smoothing, self.c, self.e, self.xi, self.eta, self.eps,
                       self.coef.ctypes.data_as(C.POINTER(C.c_double)))


def pfe_design_filter(lam_lo, lam_hi, lam_lb, lam_ub, degree=0, eps=0.0, r=0.0,
                      smoothing=PFE_SMOOTH_NONE) -> Filter:
    L = load_library()
    opts = CFilterOpts(degree, eps, r, smoothing)
    out = CFilter()
    cap = max(degree + 1, 1)
    while True:
        buf = np.zeros(cap, dtype=np.float64)
        st = L.pfe_design_filter(lam_lo, lam_hi, lam_lb, lam_ub, C.byref(opts),
                                 buf.ctypes.data_as(C.POINTER(C.c_double)), cap, C.byref(out))
        if st == -6 and out.degree + 1 > cap:
            cap = out.degree + 1
            continue
        if st != 0:
            raise PfeError(st, "pfe_design_filter failed")
        return Filter(out.degree, out.smoothing, out.c, out.e, out.xi, out.eta, out.eps,
                      buf[: out.degree + 1].copy())


def pfe_apply_filter(h, f: Filter, X, Y=None, precision=None):
    """Y = p(H_hat) X for X [n][ld] (FP64 or FP32 by dtype unless precision given)."""
    L = load_library()
    dt = np.float32 if (getattr(X, "dtype", None) in (np.float32,) or str(getattr(X, "dtype", "")) == "torch.float32") else np.float64
    if precision is None:
        precision = PFE_FP32 if dt == np.float32 else PFE_FP64
    if Y is None:
        Y = _empty_like_side(X, tuple(X.shape), dt)
    p_x, dx = _arr(X, dt, "X")
    p_y, dy = _arr(Y, dt, "Y")
    dev = _same_side(dx, dy)
    ld = int(X.shape[1])
    cf = f.cstruct()
    _check(h, L.pfe_apply_filter(h, C.byref(cf), ld, p_x, p_y, ld, precision,
                                 PFE_DEVICE_PTRS if dev else 0))
    return Y


def pfe_apply_filter_noalloc(h, f: Filter, X, Y, nvec=None):
    """Y = p(H_hat) X (FP64) for device tensors X, Y [n][ld] with no device
    allocation by the library.  Only enqueues the work on the handle's stream
    (no synchronisation); nvec: leading columns to filter (default all)."""
    L = load_library()
    p_x, dx = _arr(X, np.float64, "X")
    p_y, dy = _arr(Y, np.float64, "Y")
    if not (dx and dy):
        raise TypeError("pfe_apply_filter_noalloc takes device tensors only")
    ld = int(X.shape[1])
    if tuple(Y.shape) != tuple(X.shape):
        raise TypeError("X and Y must have the same shape")
    cf = f.cstruct()
    _check(h, L.pfe_apply_filter_noalloc(h, C.byref(cf), ld if nvec is None else int(nvec), p_x, p_y,
                                         ld))
    return Y


def pfe_apply_filter_adjoint(h, f: Filter, X, dY, nnzb: int, ckpt_stride: int = 0, nvec=None,
                             resident: bool = False):
    """(dX, dblocks[nnzb,3,3]) of the FP64 filter.  ckpt_stride: steps per
    checkpoint segment (0: ceil(sqrt(d))).  resident (with ckpt_stride 0):
    PFE_ADJOINT_RESIDENT, keep the forward (and adjoint) vectors on the
    device when they fit instead of recomputing them (identical results).
    nvec: the leading columns of X and dY that are vectors (default all; the
    rest is row padding, and dX's padding columns are left undefined)."""
    L = load_library()
    dX = _empty_like_side(X, tuple(X.shape), np.float64)
    dB = _empty_like_side(X, (nnzb, 3, 3), np.float64)
    p_x, d1 = _arr(X, np.float64, "X")
    p_dy, d2 = _arr(dY, np.float64, "dY")
    p_dx, d3 = _arr(dX, np.float64, "dX")
    p_db, d4 = _arr(dB, np.float64, "dblocks")
    dev = _same_side(d1, d2, d3, d4)
    ld = int(X.shape[1])
    nv = ld if nvec is None else int(nvec)
    cf = f.cstruct()
    _check(h, L.pfe_apply_filter_adjoint(h, C.byref(cf), nv, p_x, p_dy, p_dx, p_db, ld,
                                         ckpt_stride, (PFE_DEVICE_PTRS if dev else 0) |
                                         (PFE_ADJOINT_RESIDENT if resident else 0)))
    return dX, dB


def pfe_eigvec_block_gradient(h, V, nnzb: int, w=None):
    """dblocks[b] = sum_s w_s v_s[i] v_s[j]^T for V [nvec][n] (vector s contiguous)."""
    L = load_library()
    dB = _empty_like_side(V, (nnzb, 3, 3), np.float64)
    p_v, d1 = _arr(V, np.float64, "V")
    p_w, d2 = _arr(w, np.float64, "w")
    p_b, d3 = _arr(dB, np.float64, "dblocks")
    dev = _same_side(d1, d2, d3)
    _check(h, L.pfe_eigvec_block_gradient(h, int(V.shape[0]), p_v, p_w, p_b,
                                          PFE_DEVICE_PTRS if dev else 0))
    return dB


def pfe_spring_gradient(h, pairs, unit, dblocks, n_atoms: int):
    """(dk[P], dm[N]) through H = M^{-1/2} K M^{-1/2} of a spring network."""
    L = load_library()
    P = int(pairs.shape[0])
    dk = _empty_like_side(dblocks, (P,), np.float64)
    dm = _empty_like_side(dblocks, (n_atoms,), np.float64)
    p_p, d1 = _arr(pairs, np.int64, "pairs")
    p_u, d2 = _arr(unit, np.float64, "unit")
    p_g, d3 = _arr(dblocks, np.float64, "dblocks")
    p_k, d4 = _arr(dk, np.float64, "dk")
    p_m, d5 = _arr(dm, np.float64, "dm")
    dev = _same_side(d1, d2, d3, d4, d5)
    _check(h, L.pfe_spring_gradient(h, P, p_p, p_u, p_g, p_k, p_m, PFE_DEVICE_PTRS if dev else 0))
    return dk, dm


def pfe_solve_interval(h, lam_lo, lam_hi, nev, block, degree=0, eps=0.0, r=0.0,
                       smoothing=PFE_SMOOTH_NONE, tol=0.0, max_iter=100, precision=PFE_FP64,
                       seed=11, x0=None, want_vectors=True, vectors_on_device=False,
                       allow_noconv=False, locking=1, refine_sweeps=0):
    """Eigenpairs in [lam_lo, lam_hi].  Returns a dict with evals, evecs
    ([n_found][n], numpy or a GPU tensor), resid, stats, status."""
    L = load_library()
    o = CSolveOpts()
    L.pfe_solve_opts_default(C.byref(o))
    o.block, o.degree, o.eps, o.r, o.smoothing = block, degree, eps, r, smoothing
    o.tol, o.max_iter, o.precision, o.seed = tol, max_iter, precision, seed
    o.locking = locking
    o.refine_sweeps = refine_sweeps
    p_x0, dx = _arr(x0, np.float64, "x0")
    o.x0 = p_x0
    o.flags = PFE_DEVICE_PTRS if (dx or vectors_on_device) else 0
    if dx is not None and bool(dx) != bool(vectors_on_device) and want_vectors:
        vectors_on_device = bool(dx)
        o.flags = PFE_DEVICE_PTRS if dx else 0
    n_found = C.c_int32()
    ev = np.zeros(max(nev, 1))
    rs = np.zeros(max(nev, 1))
    stats = CSolveStats()
    vecs = None
    p_vec = None
    if want_vectors and nev > 0 and h.value in _N:
        n = _n_of(h)
        if vectors_on_device:
            import torch
            vecs = torch.zeros((nev, n), dtype=torch.float64, device="cuda")
            p_vec = vecs.data_ptr()
        else:
            vecs = np.zeros((nev, n))
            p_vec = vecs.ctypes.data
    st = L.pfe_solve_interval(h, lam_lo, lam_hi, nev, C.byref(o), C.byref(n_found), ev.ctypes.data,
                              p_vec, rs.ctypes.data, C.byref(stats))
    if st != 0 and not (allow_noconv and st == -5):
        _check(h, st)
    k = n_found.value
    sd = {f: getattr(stats, f) for f, _ in CSolveStats._fields_}
    return {"evals": ev[:k].copy(), "evecs": None if vecs is None else vecs[:k],
            "resid": rs[:k].copy(), "stats": sd, "status": STATUS.get(st, st)}


def pfe_solve_sliced(h, lam_lo, lam_hi, nev, block, n_slices=0, per_slice=0, margin=0.0,
                     count_degree=0, count_samples=0, count_seed=13, cuts=None, r=0.0,
                     smoothing=PFE_SMOOTH_NONE, tol=0.0, max_iter=100, precision=PFE_FP64, seed=11,
                     locking=1, want_vectors=True, vectors_on_device=False, refine_sweeps=0):
    """Eigenpairs in [lam_lo, lam_hi] by spectrum slicing.  Returns a dict with
    evals, evecs ([n_found][n]), resid, stats, status, n_slices and the
    sub-window boundaries."""
    L = load_library()
    o = CSolveOpts()
    L.pfe_solve_opts_default(C.byref(o))
    o.block, o.r, o.smoothing, o.tol, o.max_iter = block, r, smoothing, tol, max_iter
    o.precision, o.seed, o.locking = precision, seed, locking
    o.refine_sweeps = refine_sweeps
    o.flags = PFE_DEVICE_PTRS if vectors_on_device else 0
    so = CSliceOpts()
    so.n_slices, so.per_slice, so.margin = n_slices, per_slice, margin
    so.count_degree, so.count_samples, so.count_seed = count_degree, count_samples, count_seed
    cuts_arr = None
    if cuts is not None:
        cuts_arr = np.ascontiguousarray(cuts, dtype=np.float64)
        so.n_slices = cuts_arr.size + 1
        so.cuts = cuts_arr.ctypes.data
    n_found = C.c_int32()
    ns = C.c_int32()
    ev = np.zeros(max(nev, 1))
    rs = np.zeros(max(nev, 1))
    cut_out = np.zeros(4098)
    stats = CSolveStats()
    vecs = None
    p_vec = None
    if want_vectors and nev > 0 and h.value in _N:
        n = _n_of(h)
        if vectors_on_device:
            import torch
            vecs = torch.zeros((nev, n), dtype=torch.float64, device="cuda")
            p_vec = vecs.data_ptr()
        else:
            vecs = np.zeros((nev, n))
            p_vec = vecs.ctypes.data
    st = L.pfe_solve_sliced(h, lam_lo, lam_hi, nev, C.byref(o), C.byref(so), C.byref(n_found),
                            ev.ctypes.data, p_vec, rs.ctypes.data, C.byref(ns), cut_out.ctypes.data,
                            cut_out.size, C.byref(stats))
    _check(h, st)
    k = n_found.value
    sd = {f: getattr(stats, f) for f, _ in CSolveStats._fields_}
    return {"evals": ev[:k].copy(), "evecs": None if vecs is None else vecs[:k],
            "resid": rs[:k].copy(), "stats": sd, "status": STATUS.get(st, st),
            "n_slices": ns.value, "cuts": cut_out[: ns.value + 1].copy()}


@dataclass
class DiracFilter:
    degree: int
    smoothing: int
    c: float
    e: float
    xi: float
    eta: float
    gamma: float
    tau: float
    peak: float
    coef: np.ndarray


def pfe_design_dirac(lam_lo, lam_hi, lam_lb, lam_ub, degree=0, phi=0.8,
                     smoothing=PFE_SMOOTH_NONE) -> DiracFilter:
    """Dirac-delta filter (host only)."""
    L = load_library()
    out = CDiracFilter()
    cap = max(degree + 1, 1)
    while True:
        buf = np.zeros(cap)
        st = L.pfe_design_dirac(lam_lo, lam_hi, lam_lb, lam_ub, degree, phi, smoothing,
                                buf.ctypes.data, cap, C.byref(out))
        if st == -6 and out.degree + 1 > cap:
            cap = out.degree + 1
            degree = out.degree      # keep the degree found, skip the search
            continue
        if st != 0:
            raise PfeError(st, "pfe_design_dirac failed")
        return DiracFilter(out.degree, out.smoothing, out.c, out.e, out.xi, out.eta, out.gamma,
                           out.tau, out.peak, buf[: out.degree + 1].copy())


def pfe_locality_order(row_ptr, col_idx, leaf=256, group=2, window=32768):
    """(order, far_in, far_out): compact-range order of the atoms of a block-CSR
    pattern (host only); far_* are the fractions of off-diagonal blocks whose
    atoms lie more than `window` positions apart before / after."""
    L = load_library()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.shape[0] - 1
    order = np.zeros(max(n, 1), dtype=np.int32)
    fi, fo = C.c_double(), C.c_double()
    st = L.pfe_locality_order(n, ci.shape[0], rp.ctypes.data, ci.ctypes.data, leaf, group, window,
                              order.ctypes.data, C.byref(fi), C.byref(fo))
    if st != 0:
        raise PfeError(st, "pfe_locality_order failed")
    return order[:n], fi.value, fo.value


def pfe_solve_lanczos(h, lam_lo, lam_hi, nev, block=16, max_basis=0, degree=0, phi=0.8,
                      smoothing=PFE_SMOOTH_NONE, tol=0.0, max_restarts=0, seed=11,
                      want_vectors=True, vectors_on_device=False):
    """Eigenpairs in [lam_lo, lam_hi] by thick-restart block Lanczos on the
    Dirac filter.  Returns a dict like pfe_solve_interval."""
    L = load_library()
    o = CLanczosOpts()
    L.pfe_lanczos_opts_default(C.byref(o))
    o.block, o.max_basis, o.degree, o.phi, o.smoothing = block, max_basis, degree, phi, smoothing
    o.tol, o.max_restarts, o.seed = tol, max_restarts, seed
    o.flags = PFE_DEVICE_PTRS if vectors_on_device else 0
    n_found = C.c_int32()
    ev = np.zeros(max(nev, 1))
    rs = np.zeros(max(nev, 1))
    stats = CSolveStats()
    vecs = None
    p_vec = None
    if want_vectors and nev > 0 and h.value in _N:
        n = _n_of(h)
        if vectors_on_device:
            import torch
            vecs = torch.zeros((nev, n), dtype=torch.float64, device="cuda")
            p_vec = vecs.data_ptr()
        else:
            vecs = np.zeros((nev, n))
            p_vec = vecs.ctypes.data
    st = L.pfe_solve_lanczos(h, lam_lo, lam_hi, nev, C.byref(o), C.byref(n_found), ev.ctypes.data,
                             p_vec, rs.ctypes.data, C.byref(stats))
    _check(h, st)
    k = n_found.value
    sd = {f: getattr(stats, f) for f, _ in CSolveStats._fields_}
    return {"evals": ev[:k].copy(), "evecs": None if vecs is None else vecs[:k],
            "resid": rs[:k].copy(), "stats": sd, "status": STATUS.get(st, st)}


def pfe_count_moments(h, K: int, nsamples: int = 32, V=None, seed: int = 13):
    """mu_k = (1/M) sum_l v_l^T T_k(H_hat) v_l, k = 0..K (numpy)."""
    L = load_library()
    p_v, dv = _arr(V, np.float64, "V")
    mu = np.zeros(K + 1)
    _check(h, L.pfe_count_moments(h, K, nsamples, p_v, seed, PFE_DEVICE_PTRS if dv else 0,
                                  mu.ctypes.data))
    return mu


def _n_of(h) -> int:
    v = _N.get(h.value)
    if v is None:
        raise RuntimeError("matrix order unknown: call pfe_set_hessian through this module first")
    return v


def pfe_estimate_count(h, lam_lo, lam_hi, degree, smoothing=PFE_SMOOTH_JACKSON, nsamples=30,
                       V=None, seed=13) -> float:
    L = load_library()
    p_v, dv = _arr(V, np.float64, "V")
    if V is not None:
        nsamples = int(V.shape[1])
    out = C.c_double()
    _check(h, L.pfe_estimate_count(h, lam_lo, lam_hi, degree, smoothing, nsamples, p_v, seed,
                                   PFE_DEVICE_PTRS if dv else 0, C.byref(out)))
    return out.value
