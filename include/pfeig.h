/*
 * pfeig — polynomial-filtered interior eigensolver for the mass-weighted
 * Hessian of a 3N-dimensional vibrational problem, on one AMD MI355X (gfx950).
 *
 * Method: Accaputo, Derlet, Arbenz, "Solving large-scale interior eigenvalue
 * problems to investigate the vibrational properties of the boson peak regime
 * in amorphous materials" (2019).  The calls follow the paper's BosonPeak
 * pipeline (Algorithm 3): import H (step 2), Lanczos bounds (step 3), spectral
 * map (step 4, eq. transf.1), filter design (step 6, Sec. 2.6), eigenpairs in
 * [lam_lo, lam_hi] with small residuals (step 7, Algorithm 4 with
 * Rayleigh-Ritz, Algorithm 1), plus the filter application itself
 * (Algorithm 2), its reverse-mode adjoint, and the eigenvalue count (Sec. 2.4).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Matrices are 3x3 block-CSR over atoms: row_ptr[n_atoms+1] (int64),
 *   col_idx[nnzb] (int32, strictly increasing within a row, the diagonal block
 *   present in every row), values [nnzb][3][3] row-major FP64.  n = 3 n_atoms.
 * - Multivectors are row-major [n][ld]: the q columns of one matrix row are
 *   contiguous, row r starts at r*ld.  Vector i of an eigenvector output is
 *   contiguous instead ([nev][n]).
 * - Pointers are host memory unless the call's flags contain PFE_DEVICE_PTRS,
 *   in which case they are device memory of the handle's device.  The caller
 *   owns every pointer it passes; the library copies what it keeps.  Device
 *   inputs are read stream-ordered on the handle's stream and must stay valid
 *   until the call returns (every call synchronises its stream before
 *   returning, except where stated).
 * - Errors are returned as pfe_status, never thrown; pfe_last_error gives a
 *   message.  A handle is not thread-safe; use one handle per host thread.
 */
#ifndef PFEIG_H
#define PFEIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfe_ctx* pfe_handle;

typedef enum {
  PFE_OK = 0,
  PFE_EINVAL = -1,      /* bad argument, NaN/Inf, unsorted columns, mass <= 0 */
  PFE_ENOTSYM = -2,     /* a stored block K_ij differs from K_ji^T, or K_ji missing */
  PFE_ENOMEM = -3,      /* device allocation failed */
  PFE_EHIP = -4,        /* HIP runtime error */
  PFE_ENOCONV = -5,     /* max_iter reached; partial results are returned */
  PFE_ECAPACITY = -6,   /* more eigenvalues in the window than nev */
  PFE_EBOUNDS = -7,     /* filter iterates grew: the spectrum exceeds [lam_lb, lam_ub] */
  PFE_ESTATE = -8,      /* call out of order (no Hessian, no bounds) */
  PFE_EBREAKDOWN = -9   /* orthonormalisation broke down even with a shift */
} pfe_status;

/* flags */
#define PFE_DEVICE_PTRS 1u   /* array arguments are device pointers */
#define PFE_BLOCKS_ARE_H 2u  /* set_hessian: blocks are already mass-weighted H */

/* smoothing of the Chebyshev coefficients (Sec. 2.3) */
#define PFE_SMOOTH_NONE 0
#define PFE_SMOOTH_JACKSON 1   /* eq. jackson_smoothing */
#define PFE_SMOOTH_LANCZOS 2   /* eq. lanczos_smoothing (sigma damping) */

/* arithmetic of the filter */
#define PFE_FP64 0
#define PFE_FP32 1   /* FP32 block values and vectors, FP32 accumulation */

/* Create a handle on HIP device `device`.  `hip_stream` is a hipStream_t to
 * run on (NULL: the library creates its own blocking stream, ordered against
 * the legacy default stream, so device arrays written there before the call
 * are complete when the library reads them).  The stream must have the
 * default priority. */
pfe_status pfe_create(int device, void* hip_stream, pfe_handle* out);
void pfe_destroy(pfe_handle h);
/* Message describing the last non-OK status of this handle ("" if none);
 * with h == NULL, the reason the calling thread's last pfe_create failed. */
const char* pfe_last_error(pfe_handle h);
/* Library version string. */
const char* pfe_version(void);

/* ---------------------------------------------------------------- Hessian
 * Import the Hessian (Algorithm 3, step 2) and form H_ij = K_ij/sqrt(m_i m_j)
 * on the device (Sec. 1, eq. intro.2) unless PFE_BLOCKS_ARE_H.  Validates:
 * sorted columns with the diagonal present (EINVAL), finite values and masses
 * > 0 (EINVAL), every block's transpose partner present and equal to its
 * transpose (ENOTSYM).  Replaces any previous Hessian and clears the bounds.
 * `masses` may be NULL only with PFE_BLOCKS_ARE_H (the spring gradient call
 * then needs them and fails with ESTATE). */
pfe_status pfe_set_hessian(pfe_handle h, int64_t n_atoms, int64_t nnzb,
                           const int64_t* row_ptr, const int32_t* col_idx,
                           const double* blocks, const double* masses, uint32_t flags);

/* Import a harmonic spring network (the pair-potential Hessian of Sec. 1,
 * eq. intro.1, with one spring constant per pair): spring p joins atoms
 * pairs[p] = (i, j) with 0 <= i < j < n_atoms, listed in strictly increasing
 * (i, j) order, along the unit vector unit[p][3] and with constant k[p].  On
 * the device K_ij = K_ji = -k_p u_p u_p^T, K_ii = -sum_{j != i} K_ij on the
 * given BSR pattern, which must hold exactly the diagonal blocks and both
 * orientations of every spring (nnzb = n_atoms + 2 n_springs; EINVAL
 * otherwise, or if an off-diagonal block has no spring); then everything
 * pfe_set_hessian does with these K and masses (mass weighting, validation).
 * hblocks_out (nullable, [nnzb][3][3], same side as the inputs) receives
 * H = M^{-1/2} K M^{-1/2} in the pattern's order.  pairs, unit and k are only
 * read during the call; the spring gradient call takes them again. */
pfe_status pfe_set_springs(pfe_handle h, int64_t n_atoms, int64_t nnzb, const int64_t* row_ptr,
                           const int32_t* col_idx, int64_t n_springs, const int64_t* pairs,
                           const double* unit, const double* k, const double* masses,
                           double* hblocks_out, uint32_t flags);

/* Host-only, pure: an order of the atoms of a block-CSR pattern (symmetric
 * structure, host arrays as for pfe_set_hessian) in which contiguous ranges
 * are compact regions of the pattern's graph.  The atoms are bisected
 * recursively at breadth-first levels from a pseudo-peripheral atom down to
 * ranges of `leaf` atoms (>= 2 group); inside a range they are taken
 * `group` at a time (1..4), each group grown by the free neighbour sharing
 * the most block columns.  order[k] (n_atoms entries, caller-owned) is the
 * atom taken k-th.  The filter applies the same order to its own work when
 * the given numbering scatters neighbours (the results do not change); a
 * caller may also renumber its atoms with it.  far_in / far_out (either may
 * be NULL) receive the fraction of off-diagonal blocks whose atoms lie more
 * than `window` positions apart in the given numbering / in the order.
 * EINVAL for inconsistent arrays or parameters. */
pfe_status pfe_locality_order(int64_t n_atoms, int64_t nnzb, const int64_t* row_ptr,
                              const int32_t* col_idx, int32_t leaf, int32_t group, int64_t window,
                              int32_t* order, double* far_in, double* far_out);

/* ----------------------------------------------------------------- bounds
 * `steps` Lanczos steps with full re-orthogonalisation on H (Algorithm 3,
 * step 3) from start vector v0 (length n; NULL: a seeded Gaussian vector from
 * the library's own counter-based generator).  Returns theta_max (largest Ritz
 * value), lam_ub = theta_max + |beta_m s_m| (Ritz residual bound) and
 * lam_lb = 0 (H is positive semi-definite by construction), and stores
 * (lam_lb, lam_ub) in the handle for the spectral map. */
pfe_status pfe_estimate_bounds(pfe_handle h, int32_t steps, const double* v0, uint64_t seed,
                               uint32_t flags, double* lam_lb, double* lam_ub, double* theta_max);
/* Store explicit bounds [lam_lb, lam_ub] of the spectrum (lam_lb < lam_ub). */
pfe_status pfe_set_bounds(pfe_handle h, double lam_lb, double lam_ub);

/* ---------------------------------------------------------------- filters */
typedef struct {
  int32_t degree;     /* d >= 1; 0: smallest d satisfying eq. thresh at eps */
  double eps;         /* margin in mapped units; 0: smallest eps (geometric grid,
                         factor 1.01 from (eta-xi)/1000) satisfying eq. thresh at d */
  double r;           /* rate of eq. thresh; 0 -> 0.1^(1/4) */
  int32_t smoothing;  /* PFE_SMOOTH_* */
} pfe_filter_opts;

typedef struct {
  int32_t degree;      /* d */
  int32_t smoothing;
  double c, e;         /* H_hat = (H - c I)/e  (eq. transf.1; e is the paper's half-width d) */
  double xi, eta, eps; /* mapped window [xi, eta] and margin */
  const double* coef;  /* d+1 host coefficients g_j gamma_j (eq. rho_k_smoothened); caller-owned */
} pfe_filter;

/* Host-only, pure: design the piecewise-quadratic filter pi_d of Sec. 2.6
 * for [lam_lo, lam_hi] within bounds [lam_lb, lam_ub]: c, e of eq. transf.1,
 * coefficients by the exact integrals of Appendix A with each piece clipped to
 * [-1, 1], damping factors, degree or margin by eq. thresh (a margin end
 * outside [-1, 1] constrains nothing and is dropped from the test).  Writes
 * d+1 coefficients to coef_out (capacity coef_cap; ECAPACITY if too small)
 * and sets out->coef = coef_out. */
pfe_status pfe_design_filter(double lam_lo, double lam_hi, double lam_lb, double lam_ub,
                             const pfe_filter_opts* opts, double* coef_out, int32_t coef_cap,
                             pfe_filter* out);

/* Y = pi(H_hat) X for nvec columns (Algorithm 2), X and Y row-major [n][ld].
 * precision PFE_FP64: double arrays, H in FP64 with c and e applied as FP64
 * scalars.  PFE_FP32: float arrays; H_hat is formed in FP64 and rounded to
 * FP32 (cached per (c, e)), the recurrence runs in FP32.  X and Y must not
 * overlap. */
pfe_status pfe_apply_filter(pfe_handle h, const pfe_filter* f, int32_t nvec, const void* X,
                            void* Y, int64_t ld, int32_t precision, uint32_t flags);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * filter of pfe_apply_filter, Y = pi(H_hat) X for nvec columns of device
 * arrays X and Y ([n][ld], row-major, must not overlap), with the same
 * kernels and the same results.  The recurrence's scratch multivector lives in
 * a static device array of 256 MiB that each device holds from pfe_create
 * until the process ends, so the call allocates nothing: n * ld * 8 must not
 * exceed 268435456 bytes (EINVAL otherwise).  The call only enqueues work on
 * the handle's stream and returns without synchronising; Y is complete when
 * that work is.  Every call on one device shares the one scratch array: calls
 * whose work overlaps in time on one device (other streams, other handles,
 * other host threads) race and give wrong results.  EINVAL also for a bad
 * filter, nvec or ld; ESTATE without a Hessian. */
pfe_status pfe_apply_filter_noalloc(pfe_handle h, const pfe_filter* f, int32_t nvec,
                                    const double* X, double* Y, int64_t ld);

/* Reverse mode of pfe_apply_filter (FP64): given X and dY = dL/dY ([n][ld]),
 * returns dX = dL/dX ([n][ld]) and dblocks = dL/dH on every stored block
 * ([nnzb][3][3], each stored block an independent parameter, c and e held
 * constant), by the adjoint recurrence a_k = g_k dY + 2 H_hat a_{k+1} - a_{k+2}
 * (the reverse of Algorithm 2's recurrence), over segments of s = ckpt_stride
 * steps (0: ceil(sqrt(d))), each segment's block gradient formed in one
 * batched pass.  The forward recurrence vectors of a segment are recomputed
 * from a checkpoint pair kept per segment (2 ceil(d/s) + 2 s + 2 vectors of
 * workspace, about one more forward filter of work).  flags may add
 * PFE_ADJOINT_RESIDENT (with ckpt_stride = 0): when the forward and the
 * adjoint vectors fit in half the free device memory (2 (d + 2) vectors;
 * nvec == ld), one fused step advances both recurrences side by side; else,
 * when the d forward vectors fit, they are kept; else checkpoints as above
 * (also when that workspace cannot be allocated).  No vector is recomputed in
 * the resident cases, and the library holds their workspace until
 * pfe_destroy.  All modes give identical results. */
#define PFE_ADJOINT_RESIDENT 4u
pfe_status pfe_apply_filter_adjoint(pfe_handle h, const pfe_filter* f, int32_t nvec,
                                    const double* X, const double* dY, double* dX,
                                    double* dblocks, int64_t ld, int32_t ckpt_stride,
                                    uint32_t flags);

/* dblocks[b] = sum_s w_s v_s[i] v_s[j]^T on every stored block b = (i, j):
 * the Hellmann-Feynman gradient dL/dH of L = sum_s w_s lambda_s for unit
 * eigenvectors V ([nvec][n], vector s contiguous).  w == NULL: all ones. */
pfe_status pfe_eigvec_block_gradient(pfe_handle h, int32_t nvec, const double* V, const double* w,
                                     double* dblocks, uint32_t flags);

/* Chain rule through H_ij = K_ij / sqrt(m_i m_j) for a spring network with
 * K_ij = K_ji = -k u u^T, K_ii = -sum_j K_ij: from dblocks = dL/dH ([nnzb][3][3])
 * to dk[P] (springs given as pairs[P][2] int64 (i != j) and unit vectors
 * unit[P][3]) and dm[n_atoms]:
 *   dk = <u u^T, G_ii/m_i + G_jj/m_j - (G_ij + G_ji)/sqrt(m_i m_j)>,
 *   dm_i = -(1/(2 m_i)) [sum_j <G_ij, H_ij> + sum_j <G_ji, H_ji>].
 * Needs the masses given to set_hessian. */
pfe_status pfe_spring_gradient(pfe_handle h, int64_t n_springs, const int64_t* pairs,
                               const double* unit, const double* dblocks, double* dk, double* dm,
                               uint32_t flags);

/* ------------------------------------------------------------------ solve */
typedef struct {
  int32_t block;       /* q: subspace width (1..256); should exceed the number of
                          eigenvalues in [xi - eps, eta + eps] (Sec. 2.6) */
  int32_t degree;      /* filter degree (0: by eq. thresh from eps) */
  double eps;          /* filter margin in mapped units (0: by eq. thresh at degree) */
  double r;            /* eq. thresh rate; 0 -> 0.1^(1/4) */
  int32_t smoothing;   /* PFE_SMOOTH_* */
  double tol;          /* residual ||H v - lambda v|| / lam_ub; 0 -> 1e-10 (FP64),
                          1e-8 (FP32 filter form) */
  int32_t max_iter;    /* outer iterations (filter applications); 0 -> 100 */
  int32_t precision;   /* PFE_FP64, or PFE_FP32: FP32 filter with FP64
                          orthonormalisation, Rayleigh-Ritz and residuals until
                          the residuals plateau at the FP32 rounding floor (or
                          come within 30 tol), then one FP64 refinement sweep:
                          m FP64 filter applications, each followed by CholQR2,
                          then Rayleigh-Ritz and the residual check.  m (at most
                          16) is the number of applications that takes the
                          residual below tol at the contraction rate kappa,
                          the larger of min_j |pi(theta_j)| / min_i
                          |pi(theta_i)| (j over the Ritz values, i over those
                          near the window) and the FP32 iterations' last
                          contraction before the plateau, from min(plateau,
                          kappa x the previous iteration's largest
                          near-window residual).  If
                          the residuals still exceed tol: ENOCONV with the
                          converged pairs (see refine_sweeps) */
  uint64_t seed;       /* start block seed when x0 == NULL */
  const double* x0;    /* optional start block [n][block] (host, or device with
                          PFE_DEVICE_PTRS in flags) */
  uint32_t flags;      /* PFE_DEVICE_PTRS applies to x0 and evecs */
  int32_t locking;     /* 1 (default): locking of converged Ritz vectors (Sec. 3,
                          after Algorithm 4): in-window Ritz pairs whose residual
                          is <= tol/10 are not filtered in the next iteration (the
                          filter runs on the others, rounded up to a multiple of
                          8 columns); they stay in the orthonormalisation and in
                          the Rayleigh-Ritz step, so they keep improving and
                          rejoin the filtered set if their residual grows.
                          0: every column is filtered in every iteration. */
  int32_t refine_sweeps; /* FP32 form: refinement sweeps allowed (0 -> 1, the
                          method's one sweep); more than one is opt-in, each
                          further sweep sized from the residual the last left */
} pfe_solve_opts;

typedef struct {
  int32_t iterations;        /* outer iterations in total */
  int32_t fp64_iterations;   /* of which with the FP64 filter */
  int32_t refined;           /* FP64 refinement sweeps run (FP32 form) */
  int32_t degree;
  double eps, c, e, xi, eta;
  int64_t filter_steps;      /* fused Chebyshev step launches */
  double filter_bytes;       /* algorithmic HBM bytes of those steps */
  double t_total;            /* seconds, solve call */
  double t_filter;           /* seconds in filter steps (events on the stream) */
  double t_orth;             /* CholQR2 */
  double t_rr;               /* Rayleigh-Ritz incl. H X and the small eigensolve */
  double t_resid;            /* residuals and selection */
  double gemm_flops;         /* flops of the MFMA kernels (Gram and tall GEMM, 2 n q^2
                                each) in CholQR2 and Rayleigh-Ritz */
  double max_resid;          /* largest returned residual */
  int32_t n_window;          /* in-window Ritz values at the end */
  int64_t filter_columns;    /* sum over iterations of the filtered columns */
  double t_gemm;             /* seconds in those MFMA kernels (events on the stream) */
  int32_t shifted_passes;    /* CholQR breakdowns answered by a shifted pass (or, for a
                                rank-deficient start block, by a refilled column) */
  int32_t refine_applications; /* FP64 filter applications in the refinement sweeps */
} pfe_solve_stats;

/* Fill opts with defaults (block 0 must then be set by the caller). */
void pfe_solve_opts_default(pfe_solve_opts* opts);

/* Eigenpairs of H with eigenvalue in the closed window [lam_lo, lam_hi]
 * (eq. intro.33) by filtered subspace iteration (Algorithm 4 with the filter
 * pi(H_hat) of Sec. 2.6, CholQR2 orthonormalisation and Rayleigh-Ritz on H,
 * Algorithm 1).  Needs bounds (pfe_estimate_bounds or pfe_set_bounds).
 * Outputs: *n_found pairs, evals[nev] ascending (host), evecs [nev][n]
 * (unit 2-norm, largest-magnitude entry positive; host, or device with
 * PFE_DEVICE_PTRS in opts->flags; may be NULL), resid[nev] =
 * ||H v - lambda v|| / lam_ub (host, may be NULL), stats (may be NULL).
 * Stops when every Ritz value within 1e-6 lam_ub of the window has a
 * residual <= tol in the current iteration, the in-window count equals the
 * previous iteration's, and at least three iterations have run.  ECAPACITY: *n_found = number of in-window Ritz values, which
 * exceeds nev, or equals the block (every Ritz value in the window, so the
 * block cannot show the count is complete); nothing else written.  ENOCONV: the converged in-window pairs are
 * returned. */
pfe_status pfe_solve_interval(pfe_handle h, double lam_lo, double lam_hi, int32_t nev,
                              const pfe_solve_opts* opts, int32_t* n_found, double* evals,
                              double* evecs, double* resid, pfe_solve_stats* stats);

/* ------------------------------------------------ Dirac filter + Lanczos */
typedef struct {
  int32_t degree;      /* k */
  int32_t smoothing;
  double c, e;         /* H_hat = (H - c I)/e */
  double xi, eta;      /* mapped window */
  double gamma;        /* centre, balanced so that rho(xi) = rho(eta) */
  double tau;          /* rho(xi) = rho(eta): eigenvalues of rho(H_hat) above it are wanted */
  double peak;         /* rho(gamma) */
  const double* coef;  /* k+1 coefficients g_j T_j(gamma) / <T_j, T_j>; caller-owned */
} pfe_dirac_filter;

/* Host-only, pure: the Dirac-delta filter of Sec. 2.5 (eq. cheby-delta.1,
 * damping of Sec. 2.3) for [lam_lo, lam_hi] within [lam_lb, lam_ub].
 * degree 0: the smallest k with rho_k(xi) / rho_k(gamma) <= phi (the reading
 * that reproduces the Dirac degrees of Tables 1-3); gamma by bisection so that
 * rho_k(xi) = rho_k(eta).  Writes k+1 coefficients to coef_out (ECAPACITY, with
 * out->degree set, if coef_cap is smaller). */
pfe_status pfe_design_dirac(double lam_lo, double lam_hi, double lam_lb, double lam_ub,
                            int32_t degree, double phi, int32_t smoothing, double* coef_out,
                            int32_t coef_cap, pfe_dirac_filter* out);

typedef struct {
  int32_t block;         /* Lanczos block size b (1..64; default 16) */
  int32_t max_basis;     /* basis size m before a restart (multiple of b, 3b <= m,
                            m + b <= 511; 0: max(4b, 3 nev), the paper's 3 nev) */
  int32_t degree;        /* Dirac filter degree (0: by phi) */
  double phi;            /* rho(xi) / rho(gamma) target (0 -> 0.8, as chosen in Sec. 4.1) */
  int32_t smoothing;     /* PFE_SMOOTH_* */
  double tol;            /* residual ||H v - lambda v|| / lam_ub (0 -> 1e-10) */
  int32_t max_restarts;  /* restart cycles (0 -> 200) */
  uint64_t seed;         /* start block seed */
  uint32_t flags;        /* PFE_DEVICE_PTRS applies to evecs */
} pfe_lanczos_opts;

void pfe_lanczos_opts_default(pfe_lanczos_opts* opts);

/* Eigenpairs of H in [lam_lo, lam_hi] by block Lanczos with thick restart on
 * rho_k(H_hat) (Sec. 2.5 and Sec. 3, the Krylov alternative to subspace
 * iteration): every new block is projected against the basis twice
 * (classical Gram-Schmidt) and orthonormalised by CholQR2 (a block without
 * new directions is refilled with random ones), T = V^T rho(H_hat) V is
 * formed from Gram products, and a thick restart keeps the largest
 * Ritz vectors.  When every Ritz value >= tau has a rho-residual below
 * 0.1 tol rho(gamma) in two consecutive cycles with the same count, one
 * Rayleigh-Ritz step on H over those Ritz vectors gives the eigenpairs; if an
 * H residual near the window is still above tol the rho-tolerance is lowered
 * 100-fold and the iteration continues (at most four times).  Outputs as
 * pfe_solve_interval; stats->iterations counts restart cycles.  ECAPACITY if
 * more than m - 2b Ritz values exceed tau or the window holds more than nev.
 * A block Krylov space holds at most b directions of one eigenspace: an
 * eigenvalue of multiplicity above b is returned at most b times (subspace
 * iteration, pfe_solve_interval, has no such limit below its block size). */
pfe_status pfe_solve_lanczos(pfe_handle h, double lam_lo, double lam_hi, int32_t nev,
                             const pfe_lanczos_opts* opts, int32_t* n_found, double* evals,
                             double* evecs, double* resid, pfe_solve_stats* stats);

/* Spectrum slicing (end of Sec. 2.6; Sec. 6): eigenpairs in [lam_lo, lam_hi]
 * when they do not fit one subspace.  The window is cut into sub-windows
 * (explicit cuts, or where the count estimate of eq. eigval_count_estimator
 * from pfe_count_moments reaches equal shares), each solved like
 * pfe_solve_interval with opts (block, r, smoothing, tol, max_iter, precision,
 * locking, seed, refine_sweeps; degree, eps and x0 are ignored; with
 * refine_sweeps 0 the FP32 form's sub-solves may run up to 8 refinement
 * sweeps, since a sub-window that falls short is split and splitting does not
 * help the refinement) and a filter margin of
 * `margin` times its width (degree by eq. thresh).  Interior cuts are widened
 * by 1e-8 lam_ub on both sides; pairs within that guard are grouped by
 * eigenvalue (a gap above 1e-9 lam_ub starts a new group) and each group is
 * taken from the side that found more of it, so no pair is lost or returned
 * twice, also for degenerate eigenvalues on a cut.  A sub-window that returns
 * ECAPACITY or ENOCONV is split in two (up to 64 splits).
 * Outputs as pfe_solve_interval (evecs [nev][n], host or device by
 * opts->flags), plus the number of sub-windows used and their boundaries
 * cuts[n_slices + 1] (host, if cuts_cap is large enough).  Needs device
 * memory for nev + block eigenvectors. */
typedef struct {
  int32_t n_slices;       /* sub-windows; 0: ceil(estimated count / per_slice) */
  int32_t per_slice;      /* eigenvalues aimed for per sub-window (0: block / 2) */
  double margin;          /* filter margin / sub-window width (0: the widest margin, up
                             to 1.5 widths and at least 1/6, whose count estimated from
                             the moments stays within 85 % of the block; 1/6 when the
                             cuts are given and no moments are computed) */
  int32_t count_degree;   /* Jackson-damped series degree of the count (0: 1000) */
  int32_t count_samples;  /* probe vectors of the count (0: 32) */
  uint64_t count_seed;    /* probe vector seed */
  const double* cuts;     /* optional interior cuts [n_slices - 1] (host), ascending */
} pfe_slice_opts;

pfe_status pfe_solve_sliced(pfe_handle h, double lam_lo, double lam_hi, int32_t nev,
                            const pfe_solve_opts* opts, const pfe_slice_opts* slice_opts,
                            int32_t* n_found, double* evals, double* evecs, double* resid,
                            int32_t* n_slices, double* cuts, int32_t cuts_cap,
                            pfe_solve_stats* stats);

/* Chebyshev moments of the spectral density seen by M = nsamples unit probe
 * vectors (V [n][M] row-major if given, else drawn by the library from seed):
 * mu_k = (1/M) sum_l v_l^T T_k(H_hat) v_l for k = 0..K (host output
 * mu[K+1]), H_hat = (H - c I)/e from the stored bounds.  The count estimate
 * of eq. eigval_count_estimator for any window is n sum_k g_k gamma_k mu_k
 * with the window's characteristic-function coefficients gamma_k and damping
 * g_k. */
pfe_status pfe_count_moments(pfe_handle h, int32_t K, int32_t nsamples, const double* V,
                             uint64_t seed, uint32_t flags, double* mu);

/* Stochastic estimate of the number of eigenvalues in [lam_lo, lam_hi]
 * (Sec. 2.4, eq. eigval_count_estimator): (n/M) sum_l v_l^T psi(H_hat) v_l
 * with M = nsamples unit Gaussian vectors (V [n][M] row-major if given, else
 * drawn by the library) and psi the damped Chebyshev series of the
 * characteristic function of the mapped window, degree `degree`. */
pfe_status pfe_estimate_count(pfe_handle h, double lam_lo, double lam_hi, int32_t degree,
                              int32_t smoothing, int32_t nsamples, const double* V,
                              uint64_t seed, uint32_t flags, double* count);

/* Device memory held by the handle, in bytes (Hessian copies and workspaces). */
int64_t pfe_device_bytes(pfe_handle h);

#ifdef __cplusplus
}
#endif

#endif /* PFEIG_H */
