// C-ABI of libpfeig and its host driver: Hessian import and validation,
// Lanczos bounds, filter application (forward and reverse), filtered
// subspace iteration with CholQR2 and Rayleigh-Ritz, eigenvalue count,
// gradient chain rule.  Every numerical step runs in the library's HIP
// kernels; the host only sequences launches, designs the filter (O(d)
// scalars) and takes the convergence decisions from q Ritz values and
// residuals copied back per outer iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "lanczos_host.h"

using pfe::DevBuf;
using pfe::Err;

// Device scratch of pfe_apply_filter_noalloc: the second multivector of the
// Clenshaw recurrence (the first is the caller's output), for callers that
// cannot allocate.  Each device the library runs on holds its own copy until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: host code uses only the per-device address that
// hipGetSymbolAddress returns (scratch_addr below).
constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxScratchDevices] = {};

// Resolves the device address of `scratch` on `device`, which must be the
// current device; once per device (later calls return the stored address).
hipError_t init_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipSuccess;   // entry point refuses
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[device] = p;
  return hipSuccess;
}

void* scratch_addr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_addr[device];
}
}  // namespace

struct pfe_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // Hessian
  int64_t n_atoms = 0, nnzb = 0;
  bool has_h = false, has_masses = false;
  DevBuf row_ptr, col_idx, H, transpose, masses, H32;
  int tile_rows = 0;
  int64_t n_tiles = 0;
  DevBuf tile_ptr, tile_vptr, tile_cm, tile_row, tile_perm, Ht, H32row;
  // pattern the tiles were built for (a new value set on the same pattern
  // only re-permutes the values)
  std::vector<int64_t> tiled_rp;
  std::vector<int32_t> tiled_ci;
  int tiled_R = 0;
  bool tiled_local = false;   // rows in locality order
  int64_t tiled_window = 0;   // window of the regrouped order of tiles of 3+ rows (0: none)
  int tiled_mode = -1;        // order requested when the tiles were built
  int64_t tiled_span = 0;     // neighbour_span of the pattern
  double h32_c = NAN, h32_e = NAN;
  // Row tiles of the FP32 filter when its tile height differs from the FP64
  // one (same pattern and order; built at the first FP32 filter, kept while
  // the pattern stays): H32 is stored in their order.
  int tile32_rows = 0;
  int64_t n_tiles32 = 0;
  DevBuf t32_ptr, t32_vptr, t32_cm, t32_row, t32_perm;
  int h32_R = 0;              // tile height H32's order was made for
  // Row tiles of the FP64 filter for wide blocks (same pattern and order,
  // more rows per tile) and the block values in their order (refreshed after
  // every new value set, at the next wide filter).
  int tile64w_rows = 0;
  int64_t n_tiles64w = 0;
  DevBuf w64_ptr, w64_vptr, w64_cm, w64_row, w64_perm, Hw;
  bool hw_valid = false;
  // bounds
  bool has_bounds = false;
  double lam_lb = 0, lam_ub = 0;
  // workspaces kept between calls
  DevBuf flags;                 // int[4] + double[4]
  DevBuf wsA, wsB, wsC, wsD;    // multivectors
  DevBuf wsSmall;               // q x q matrices, vectors
  DevBuf wsRed;                 // reduction partials
  DevBuf wsOut;                 // eigenvector output staging
  DevBuf wsCk;                  // adjoint checkpoints
  DevBuf wsSlice;               // eigenvectors collected over the slices of a sliced solve
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // [0,1] phase timers, [2,3] MFMA kernels

  pfe::Bsr bsr() const {
    pfe::Bsr a;
    a.n_atoms = n_atoms;
    a.nnzb = nnzb;
    a.row_ptr = row_ptr.as<int64_t>();
    a.col_idx = col_idx.as<int32_t>();
    a.tile_rows = tile_rows;
    a.n_tiles = n_tiles;
    a.tile_ptr = tile_ptr.as<int64_t>();
    a.tile_vptr = tile_vptr.as<int64_t>();
    a.tile_cm = tile_cm.as<int2>();
    a.tile_row = tile_row.as<int32_t>();
    a.tile_local = tiled_local;
    a.span = tiled_span;
    return a;
  }
  // The pattern as the FP32 filter walks it: its own row tiles when built.
  pfe::Bsr bsr32() const {
    pfe::Bsr a = bsr();
    if (tile32_rows >= 2) {
      a.tile_rows = tile32_rows;
      a.n_tiles = n_tiles32;
      a.tile_ptr = t32_ptr.as<int64_t>();
      a.tile_vptr = t32_vptr.as<int64_t>();
      a.tile_cm = t32_cm.as<int2>();
      a.tile_row = t32_row.as<int32_t>();
    }
    return a;
  }
  pfe::Bsr bsr64w() const {
    pfe::Bsr a = bsr();
    a.tile_rows = tile64w_rows;
    a.n_tiles = n_tiles64w;
    a.tile_ptr = w64_ptr.as<int64_t>();
    a.tile_vptr = w64_vptr.as<int64_t>();
    a.tile_cm = w64_cm.as<int2>();
    a.tile_row = w64_row.as<int32_t>();
    return a;
  }
  void release_tiles64w() {
    tile64w_rows = 0;
    n_tiles64w = 0;
    hw_valid = false;
    w64_ptr.release();
    w64_vptr.release();
    w64_cm.release();
    w64_row.release();
    w64_perm.release();
    Hw.release();
  }
  void release_tiles32() {
    tile32_rows = 0;
    n_tiles32 = 0;
    t32_ptr.release();
    t32_vptr.release();
    t32_cm.release();
    t32_row.release();
    t32_perm.release();
  }
  // Block values as the fused step reads them (tile order when tiles are on).
  const double* step_vals64() const {
    return tile_rows >= 2 ? Ht.as<double>() : H.as<double>();
  }
  int64_t n() const { return 3 * n_atoms; }
};

namespace {

pfe_status finish(pfe_handle h, const Err& e) {
  if (h) h->err = e.st == PFE_OK ? std::string() : e.msg;
  return e.st;
}

// No C++ exception crosses the C-ABI: a failed host allocation (std::bad_alloc)
// becomes PFE_ENOMEM, anything else PFE_EHIP, each with a message.
template <class F>
pfe_status guarded(pfe_handle h, F&& body) {
  try {
    return finish(h, body());
  } catch (const std::bad_alloc&) {
    return finish(h, pfe::fail(PFE_ENOMEM, "host allocation failed"));
  } catch (const std::exception& ex) {
    return finish(h, pfe::fail(PFE_EHIP, std::string("internal error: ") + ex.what()));
  } catch (...) {
    return finish(h, pfe::fail(PFE_EHIP, "internal error"));
  }
}

// The same for entry points without a handle.
template <class F>
pfe_status host_guarded(F&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return PFE_ENOMEM;
  } catch (...) {
    return PFE_EHIP;
  }
}

Err select_device(pfe_handle h) {
  PFE_HIP(hipSetDevice(h->device));
  return pfe::ok();
}

// Copies n elements between host/device according to `device_ptrs`.
template <typename T>
Err upload(pfe_handle h, T* dst, const T* src, int64_t count, bool device_ptrs) {
  if (count == 0) return pfe::ok();
  PFE_HIP(hipMemcpyAsync(dst, src, count * sizeof(T),
                         device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         h->stream));
  return pfe::ok();
}
// Host block [n][q] into device rows of stride ld >= q: one contiguous copy
// (into `staging` when ld > q, at least n q doubles, which is left zeroed),
// then the strided placement on the device.  A 2-D copy from pageable host
// memory moves one row at a time (about 27 s for 3e6 rows of 160 columns).
Err upload_block(pfe_handle h, double* dst, int64_t ld, const double* src, int q, int64_t n,
                 double* staging) {
  if (n == 0 || q == 0) return pfe::ok();
  if (ld == q) {
    PFE_HIP(hipMemcpyAsync(dst, src, (size_t)n * q * sizeof(double), hipMemcpyHostToDevice,
                           h->stream));
    return pfe::ok();
  }
  PFE_HIP(hipMemcpyAsync(staging, src, (size_t)n * q * sizeof(double), hipMemcpyHostToDevice,
                         h->stream));
  PFE_HIP(pfe::copy_cols_f64(n, q, staging, q, dst, ld, h->stream));
  PFE_HIP(pfe::zero_f64(staging, n * q, h->stream));
  return pfe::ok();
}

template <typename T>
Err download(pfe_handle h, T* dst, const T* src, int64_t count, bool device_ptrs) {
  if (count == 0) return pfe::ok();
  PFE_HIP(hipMemcpyAsync(dst, src, count * sizeof(T),
                         device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         h->stream));
  return pfe::ok();
}
Err sync(pfe_handle h) {
  PFE_HIP(hipStreamSynchronize(h->stream));
  return pfe::ok();
}

int64_t round_up(int64_t v, int64_t m) { return ((v + m - 1) / m) * m; }

#ifndef PFE_TILE_ROWS
#define PFE_TILE_ROWS 2
#endif
constexpr int kDefaultTileRows = PFE_TILE_ROWS;
// FP32 filter: three-row tiles measured 4 % (1e5 atoms) and 8 % (1e6) faster
// steps at q = 96 than two-row ones, which FP64 keeps (three rows need 92
// VGPRs there).  Above kWideF32 columns (one 256-column pass, four floats per
// lane) four-row tiles share more gathers and win despite fewer waves: 4e6
// atoms, q = 256: 12.75 against 13.35 ms per step; at q = 160 and below they
// lose (9.40 against 8.86 ms), and five or six rows lose everywhere.  The
// height follows the block width of the solve (or of the filter call), so
// columns locked during a solve never rebuild the tiles.
// PFEIG_TILE_ROWS_F32 overrides.
constexpr int kDefaultTileRowsF32 = 3;
constexpr int kWideTileRowsF32 = 4;
constexpr int kWideF32 = 192;
// FP64 filter above kWideF64 columns (two 128-column passes): three-row tiles
// (one record per batch) measured 5 % faster steps on the 4e6-atom glass at
// q = 256 and slower ones at q = 160 (passes of 80) and q = 96; they get a
// tile set and a copy of the block values of their own, used by the wide
// filters only.  PFEIG_TILE_ROWS_F64W overrides (0: none).
constexpr int kWideTileRowsF64 = 3;
constexpr int kWideF64 = 192;
// Locality order of the row tiles: rows per leaf range of the bisection
// (best of 16..1024 in a per-XCD L2 model); a window of rows of the order of
// what the 256 MB Infinity Cache holds of T_in at q = 96 in FP64 (2304 B per
// atom row) next to the streamed data; and the largest fraction of
// neighbours beyond that window for which the given numbering is kept
// without comparing (1.2% on a lattice-numbered glass, 70-97% on randomly
// numbered ones).
constexpr int kOrderLeaf = 256;
constexpr int64_t kOrderWindow = 32768;
constexpr double kOrderFarMax = 0.05;

// Tile sets of three or more rows regroup the natural order inside windows
// of kGroupWindow rows (window_group_order), so that a tile's rows share
// more block columns (records per atom row on the 1e5-atom glass: 10.44 ->
// 9.06 for four-row tiles, 11.19 -> 10.18 for three-row tiles) while the
// order of work stays that of the rows.  4e6-atom glass, q = 256: FP32 step
// 12.41 -> 12.22 ms, FP64 (three-row wide tiles) 27.20 -> 26.87 ms; 1e5
// atoms, q = 96, FP32: 170.9 -> 161.9 us; 1e6 atoms FP32 at q = 160 2222 -> 2192 us.  The gain is smaller than the cut
// in gathers because the L2 hit rate falls with it (0.515 -> 0.448 at 4e6
// atoms).  Two-row tiles keep the natural order.  PFEIG_TILE_WINDOW
// overrides (0: natural order for every height).
constexpr int64_t kGroupWindow = 16384;

int64_t group_window() {
  const char* e = std::getenv("PFEIG_TILE_WINDOW");
  return e ? std::atoll(e) : kGroupWindow;
}

// Row order of tiles R rows high: the locality order when the handle's tiles
// use it, the natural order regrouped in windows for three or more rows,
// else the natural order (nullptr).
const int32_t* tile_order(int64_t na, const int64_t* rp, const int32_t* ci, bool local,
                          int64_t window, int R, std::vector<int32_t>& order) {
  if (local) {
    pfe::locality_order(na, rp, ci, kOrderLeaf, R, order);
    return order.data();
  }
  if (window > 0 && R >= 3) {
    pfe::window_group_order(na, rp, ci, window, R, order);
    return order.data();
  }
  return nullptr;
}
// Largest residual at which a plateau of the FP32-filter iterations is taken
// for their rounding floor (and answered by FP64 refinement, not by a higher
// degree).
constexpr double kFp32Floor = 1e-3;
// Most FP64 filter applications in one refinement sweep of the FP32 form.
constexpr int kMaxRefineApps = 16;
// Refinement sweeps a sub-window of a sliced FP32-form solve may run when the
// caller leaves refine_sweeps at 0.
constexpr int kSliceRefineSweeps = 8;

// Algorithmic HBM bytes of one filter application of degree d >= 1 by the
// Clenshaw recurrence (d launches): every launch reads the matrix values,
// column indices and row pointers once; the multivector streams are 2 in the
// first launch (X gathered and X), 3 in the second (b_{k+2} = 0 is not read)
// and 4 after (b_{k+1} gathered once, b_{k+2} and X read, b_k written).
double filter_bytes(int64_t n_atoms, int64_t nnzb, int q, int elem, int d) {
  if (d < 1) return 0.0;
  const double mat = (double)nnzb * (9.0 * elem + 4.0) + 8.0 * (n_atoms + 1);
  const double vec = 3.0 * n_atoms * q * elem;
  return d * mat + (4.0 * d - 3.0) * vec;
}

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  double* acc;
  bool on;
  // pair 0: phase timers; pair 1: the MFMA kernels inside a phase
  Timer(pfe_handle h, double* acc_, int pair = 0)
      : a(h->ev[2 * pair]), b(h->ev[2 * pair + 1]), s(h->stream), acc(acc_), on(acc_ != nullptr) {
    if (on) (void)hipEventRecord(a, s);
  }
  void stop() {
    if (!on) return;
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    *acc += ms * 1e-3;
    on = false;
  }
  ~Timer() { stop(); }
};

// ---------------------------------------------------------------- filter
// Y = p(A) X, A = a1 H + b1 I, by Clenshaw's backward recurrence for a
// Chebyshev series: b_{d+1} = b_{d+2} = 0, b_k = g_k X + 2 A b_{k+1} - b_{k+2}
// (k = d..1), Y = g_0 X + A b_1 - b_2.  It evaluates the same polynomial as
// the forward recurrence of Algorithm 2 with one multivector stream less per
// step (no running sum to read and write).  b_d = g_d X is never stored: it
// is folded into the first launch and into the X coefficient of the second.
// X is read only; the result lands in P, Q is scratch (P, Q, X distinct).
// d launches for d >= 1.
template <typename T>
Err run_filter(pfe_handle h, const T* vals, const double* g, int d, double a1, double b1,
               const T* X, T* P, T* Q, int q, int64_t ld, int64_t* steps,
               const pfe::Bsr* over = nullptr) {
  const pfe::Bsr A = over ? *over : (sizeof(T) == 4 ? h->bsr32() : h->bsr());
  auto step = [&](const T* tin, const T* prev, T* out, double al, double be, double de,
                  double ze) -> hipError_t {
    if constexpr (sizeof(T) == 8)
      return pfe::cheb_step_f64(A, (const double*)vals, (const double*)tin, (const double*)prev,
                                (const double*)X, (double*)out, q, ld, al, be, de, ze, h->stream);
    else
      return pfe::cheb_step_f32(A, (const float*)vals, (const float*)tin, (const float*)prev,
                                (const float*)X, (float*)out, q, ld, (float)al, (float)be,
                                (float)de, (float)ze, h->stream);
  };
  if (d == 0) {
    PFE_HIP(step(X, nullptr, P, 0.0, 0.0, 0.0, g[0]));
    if (steps) *steps += 1;
    return pfe::ok();
  }
  if (d == 1) {
    PFE_HIP(step(X, nullptr, P, g[1] * a1, g[1] * b1, 0.0, g[0]));
    if (steps) *steps += 1;
    return pfe::ok();
  }
  // outputs alternate between two buffers; pick the start so the result is P
  T* buf[2] = {((d - 1) % 2 == 0) ? P : Q, ((d - 1) % 2 == 0) ? Q : P};
  // b_{d-1} = g_{d-1} X + 2 A (g_d X)
  PFE_HIP(step(X, nullptr, buf[0], 2.0 * g[d] * a1, 2.0 * g[d] * b1, 0.0, g[d - 1]));
  if (d == 2) {
    // Y = g_0 X + A b_1 - b_2, b_2 = g_2 X
    PFE_HIP(step(buf[0], nullptr, buf[1], a1, b1, 0.0, g[0] - g[2]));
  } else {
    // b_{d-2} = g_{d-2} X + 2 A b_{d-1} - g_d X
    PFE_HIP(step(buf[0], nullptr, buf[1], 2.0 * a1, 2.0 * b1, 0.0, g[d - 2] - g[d]));
    T* cur = buf[1];   // b_{k+1}
    T* prv = buf[0];   // b_{k+2}
    for (int k = d - 3; k >= 1; --k) {
      PFE_HIP(step(cur, prv, prv, 2.0 * a1, 2.0 * b1, -1.0, g[k]));
      std::swap(cur, prv);
    }
    // Y = g_0 X + A b_1 - b_2, over b_2
    PFE_HIP(step(cur, prv, prv, a1, b1, -1.0, g[0]));
  }
  if (steps) *steps += d;
  return pfe::ok();
}

template <typename T>
Err run_filter(pfe_handle h, const T* vals, const std::vector<double>& g, double a1, double b1,
               const T* X, T* P, T* Q, int q, int64_t ld, int64_t* steps,
               const pfe::Bsr* over = nullptr) {
  return run_filter<T>(h, vals, g.data(), (int)g.size() - 1, a1, b1, X, P, Q, q, ld, steps, over);
}

// The pattern and block values an FP64 filter on blocks `width` columns wide
// walks: the wide tile set above kWideF64 (built at its first use, values
// re-permuted after every new value set), else the handle's own tiles.
Err filter_set64(pfe_handle h, int width, pfe::Bsr* A, const double** vals) {
  *A = h->bsr();
  *vals = h->step_vals64();
  int Rw = width > kWideF64 ? kWideTileRowsF64 : 0;
  if (const char* v = std::getenv("PFEIG_TILE_ROWS_F64W")) Rw = std::atoi(v);
  if (h->tile_rows < 2 || Rw < 2 || Rw > 4 || Rw == h->tile_rows) return pfe::ok();
  if (h->tile64w_rows != Rw) {
    h->release_tiles64w();
    const int64_t na = h->n_atoms;
    std::vector<int32_t> order;
    const int32_t* ord = tile_order(na, h->tiled_rp.data(), h->tiled_ci.data(), h->tiled_local,
                                    h->tiled_window, Rw, order);
    std::vector<int64_t> tp, tv, perm;
    std::vector<int32_t> tcm, trow;
    pfe::build_row_tiles(na, h->tiled_rp.data(), h->tiled_ci.data(), Rw, ord, tp, tv, tcm, trow,
                         perm);
    PFE_HIP(h->w64_ptr.ensure(tp.size() * sizeof(int64_t)));
    PFE_HIP(h->w64_vptr.ensure(tv.size() * sizeof(int64_t)));
    PFE_HIP(h->w64_cm.ensure(tcm.size() * sizeof(int32_t)));
    PFE_HIP(h->w64_row.ensure(trow.size() * sizeof(int32_t)));
    PFE_HIP(h->w64_perm.ensure(perm.size() * sizeof(int64_t)));
    PFE_HIP(hipMemcpy(h->w64_ptr.p, tp.data(), tp.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    PFE_HIP(hipMemcpy(h->w64_vptr.p, tv.data(), tv.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    PFE_HIP(hipMemcpy(h->w64_cm.p, tcm.data(), tcm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    PFE_HIP(hipMemcpy(h->w64_row.p, trow.data(), trow.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    PFE_HIP(hipMemcpy(h->w64_perm.p, perm.data(), perm.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    h->n_tiles64w = (int64_t)tp.size() - 1;
    h->tile64w_rows = Rw;
    h->hw_valid = false;
  }
  if (!h->hw_valid) {
    const int64_t nel = (h->nnzb + pfe::kBsrPad) * 9;
    PFE_HIP(h->Hw.ensure((size_t)nel * sizeof(double)));
    PFE_HIP(pfe::zero_f64(h->Hw.as<double>(), nel, h->stream));
    PFE_HIP(pfe::permute_blocks_f64(h->nnzb, h->w64_perm.as<int64_t>(), h->H.as<double>(),
                                    h->Hw.as<double>(), h->stream));
    h->hw_valid = true;
  }
  *A = h->bsr64w();
  *vals = h->Hw.as<double>();
  return pfe::ok();
}

// FP32 row tiles of height R32 over the FP64 tiles' pattern and order.
Err ensure_tiles32(pfe_handle h, int width) {
  int R32 = width > kWideF32 ? kWideTileRowsF32 : kDefaultTileRowsF32;
  if (const char* v = std::getenv("PFEIG_TILE_ROWS_F32")) R32 = std::atoi(v);
  if (h->tile_rows < 2 || R32 < 2 || R32 > 4 || R32 == h->tile_rows) {
    h->release_tiles32();   // the FP32 filter walks the FP64 tiles
    return pfe::ok();
  }
  if (h->tile32_rows == R32) return pfe::ok();
  h->release_tiles32();
  const int64_t na = h->n_atoms;
  std::vector<int32_t> order;
  const int32_t* ord = tile_order(na, h->tiled_rp.data(), h->tiled_ci.data(), h->tiled_local,
                                  h->tiled_window, R32, order);
  std::vector<int64_t> tp, tv, perm;
  std::vector<int32_t> tcm, trow;
  pfe::build_row_tiles(na, h->tiled_rp.data(), h->tiled_ci.data(), R32, ord, tp, tv, tcm, trow,
                       perm);
  PFE_HIP(h->t32_ptr.ensure(tp.size() * sizeof(int64_t)));
  PFE_HIP(h->t32_vptr.ensure(tv.size() * sizeof(int64_t)));
  PFE_HIP(h->t32_cm.ensure(tcm.size() * sizeof(int32_t)));
  PFE_HIP(h->t32_row.ensure(trow.size() * sizeof(int32_t)));
  PFE_HIP(h->t32_perm.ensure(perm.size() * sizeof(int64_t)));
  PFE_HIP(hipMemcpy(h->t32_ptr.p, tp.data(), tp.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  PFE_HIP(hipMemcpy(h->t32_vptr.p, tv.data(), tv.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  PFE_HIP(hipMemcpy(h->t32_cm.p, tcm.data(), tcm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  PFE_HIP(hipMemcpy(h->t32_row.p, trow.data(), trow.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  PFE_HIP(hipMemcpy(h->t32_perm.p, perm.data(), perm.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  h->n_tiles32 = (int64_t)tp.size() - 1;
  h->tile32_rows = R32;
  return pfe::ok();
}

// FP32 copy of H_hat in the order of the FP32 tiles for filters `width`
// columns wide.
Err ensure_h32(pfe_handle h, double c, double e, int width) {
  PFE_TRY(ensure_tiles32(h, width));
  const int R32 = h->tile32_rows >= 2 ? h->tile32_rows : h->tile_rows;
  if (h->H32.p && h->h32_c == c && h->h32_e == e && h->h32_R == R32) return pfe::ok();
  const int64_t nel = (h->nnzb + pfe::kBsrPad) * 9;
  PFE_HIP(h->H32.ensure((size_t)nel * sizeof(float)));
  PFE_HIP(pfe::zero_f32(h->H32.as<float>(), nel, h->stream));
  if (h->tile_rows >= 2) {
    // formed in row order (diagonal blocks known there), then put in the
    // order of the tiles the FP32 filter walks
    const DevBuf& perm = h->tile32_rows >= 2 ? h->t32_perm : h->tile_perm;
    PFE_HIP(h->H32row.ensure((size_t)nel * sizeof(float)));
    PFE_HIP(pfe::shift_scale_to_f32(h->bsr(), h->H.as<double>(), c, e, h->H32row.as<float>(),
                                    h->stream));
    PFE_HIP(pfe::permute_blocks_f32(h->nnzb, perm.as<int64_t>(), h->H32row.as<float>(),
                                    h->H32.as<float>(), h->stream));
    PFE_HIP(hipStreamSynchronize(h->stream));
    h->H32row.release();
  } else {
    PFE_HIP(pfe::shift_scale_to_f32(h->bsr(), h->H.as<double>(), c, e, h->H32.as<float>(),
                                    h->stream));
  }
  h->h32_c = c;
  h->h32_e = e;
  h->h32_R = R32;
  return pfe::ok();
}

Err check_filter(pfe_handle h, const pfe_filter* f) {
  if (!f || f->degree < 0 || !f->coef || !(f->e > 0) || !std::isfinite(f->c))
    return pfe::fail(PFE_EINVAL, "invalid filter (degree, coef, c, e)");
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  return pfe::ok();
}

// ------------------------------------------------------ small workspaces
struct Small {
  double* G;       // q*q
  double* Rinv;    // 2 q*q
  double* S;       // q*q
  double* Q;       // q*q
  double* jw;      // jacobi_work_bytes(q)
  double* theta;   // q
  double* res;     // q
  double* dmax;    // 4
  int* info;       // 4
  int* sel;        // q
};

Err alloc_small(pfe_handle h, int q, Small* s) {
  const size_t qq = (size_t)q * q;
  const size_t jwd = (pfe::jacobi_work_bytes(q) + sizeof(double) - 1) / sizeof(double);
  const size_t doubles = qq * 5 + jwd + 2 * (size_t)q + 4;
  const size_t bytes = doubles * sizeof(double) + 8 * sizeof(int) + (size_t)q * sizeof(int) + 256;
  PFE_HIP(h->wsSmall.ensure(bytes));
  double* p = h->wsSmall.as<double>();
  s->G = p;
  s->Rinv = s->G + qq;
  s->S = s->Rinv + 2 * qq;
  s->Q = s->S + qq;
  s->jw = s->Q + qq;
  s->theta = s->jw + jwd;
  s->res = s->theta + q;
  s->dmax = s->res + q;
  s->info = reinterpret_cast<int*>(s->dmax + 4);
  s->sel = s->info + 8;
  return pfe::ok();
}

Err ensure_red(pfe_handle h, int64_t n, int q) {
  size_t need = std::max(pfe::gram_work_bytes(n, q, q), pfe::colnorm_work_bytes(n, q));
  need = std::max(need, (size_t)q * 64 * 24 + 1024);
  PFE_HIP(h->wsRed.ensure(need));
  return pfe::ok();
}

// CholQR2 of X [n][ld] (q columns) in place.  If a factorisation breaks
// down, one shifted pass (shift 11 (n q + q (q + 1)) u tr(G) bound, the
// shifted CholeskyQR of Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa)
// is inserted and followed by the two plain passes.  That recovers blocks
// with a condition number up to about 1/u.  A block of lower rank (a start
// block with repeated columns, say) breaks down again after the shift: then
// with `refill` the column at the failed pivot, which the preceding columns
// span, is replaced by a seeded Gaussian one and the factorisation starts
// over (at most q times), as Householder QR would complete the basis
// (without, EBREAKDOWN: a caller that needs the block to stay orthogonal to
// other vectors refills and projects on its own).  On the first
// pass the largest squared column norm is compared with `norm_bound`^2
// (EBOUNDS).  Time and flops of the MFMA kernels (Gram and tall GEMM),
// 2 n q^2 each; `shifted` counts shifted passes and refilled columns.
struct GemmAcct {
  double t = 0, flops = 0;
  bool on = false;
};

Err cholqr2(pfe_handle h, const Small& sm, double* X, int64_t n, int q, int64_t ld,
            double norm_bound, GemmAcct* ga = nullptr, int* shifted = nullptr,
            bool refill = false) {
  const bool tg = ga && ga->on;
  const double f2 = 2.0 * (double)n * q * q;
  int passes = 2;
  bool shifted_done = false;
  int refills = 0;
  for (int pass = 0; pass < passes; ++pass) {
    {
      Timer tm(h, tg ? &ga->t : nullptr, 1);
      PFE_HIP(pfe::gram_f64(n, q, q, X, ld, X, ld, sm.G, h->wsRed.p, h->stream));
    }
    if (ga) ga->flops += f2;
    PFE_HIP(pfe::chol_inv_f64(q, sm.G, 0.0, sm.Rinv, sm.info, sm.dmax, h->stream));
    int info = 0;
    double dmax = 0;
    PFE_HIP(hipMemcpyAsync(&info, sm.info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    PFE_HIP(hipMemcpyAsync(&dmax, sm.dmax, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    PFE_TRY(sync(h));
    if (pass == 0 && norm_bound > 0 && !(dmax <= norm_bound * norm_bound))
      return pfe::fail(PFE_EBOUNDS,
                       "filtered vectors grew beyond the filter's bound on [-1, 1] (largest column "
                       "norm " + std::to_string(std::sqrt(dmax)) + " > " + std::to_string(norm_bound) +
                       "): the spectrum exceeds [lam_lb, lam_ub]");
    if (info != 0) {
      if (!(dmax > 0) || !std::isfinite(dmax))
        return pfe::fail(PFE_EBREAKDOWN, "CholQR breakdown (Gram matrix not positive definite)");
      if (shifted_done) {
        // rank deficient: refill the dependent column and start over
        if (!refill || refills >= q || info < 1 || info > q)
          return pfe::fail(PFE_EBREAKDOWN, "CholQR breakdown (rank-deficient block)");
        PFE_HIP(pfe::gaussian_fill_f64(n, 1, X + (info - 1), ld, 0x5EED0000ull + refills, h->stream));
        ++refills;
        if (shifted) ++*shifted;
        shifted_done = false;
        passes = 2;
        pass = -1;
        norm_bound = -1.0;
        continue;
      }
      const double u = std::ldexp(1.0, -53);
      const double shift = 11.0 * ((double)n * q + (double)q * (q + 1)) * u * (dmax * q);
      PFE_HIP(pfe::chol_inv_f64(q, sm.G, shift, sm.Rinv, sm.info, nullptr, h->stream));
      PFE_HIP(hipMemcpyAsync(&info, sm.info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
      PFE_TRY(sync(h));
      if (info != 0)
        return pfe::fail(PFE_EBREAKDOWN, "shifted CholQR breakdown");
      shifted_done = true;
      if (shifted) ++*shifted;
      passes += 1;
    }
    {
      Timer tm(h, tg ? &ga->t : nullptr, 1);
      PFE_HIP(pfe::gemm_tall_f64(n, q, q, X, ld, sm.Rinv, X, ld, h->stream));
    }
    if (ga) ga->flops += f2;
  }
  return pfe::ok();
}

// Rayleigh-Ritz on H: W = H X, S = X^T W, S = Q Theta Q^T, X <- X Q, W <- W Q,
// residuals ||W_j - theta_j X_j|| / lam_ub.  Theta and residuals to host.
Err rayleigh_ritz(pfe_handle h, const Small& sm, double* X, double* W, int64_t n, int q,
                  int64_t ld, std::vector<double>& theta, std::vector<double>& res,
                  double* t_rr, double* t_res, GemmAcct* ga = nullptr) {
  pfe::Bsr A;
  const double* vals = nullptr;
  PFE_TRY(filter_set64(h, q, &A, &vals));   // W = H X walks the filter's tiles for this width
  const bool tg = ga && ga->on;
  const double f2 = 2.0 * (double)n * q * q;
  {
    Timer tm(h, t_rr);
    PFE_HIP(pfe::cheb_step_f64(A, vals, X, nullptr, nullptr, W, q, ld, 1.0, 0.0, 0.0, 0.0,
                               h->stream));
    {
      Timer tg1(h, tg ? &ga->t : nullptr, 1);
      PFE_HIP(pfe::gram_f64(n, q, q, X, ld, W, ld, sm.S, h->wsRed.p, h->stream));
    }
    PFE_HIP(pfe::sym_eig_f64(q, sm.S, sm.theta, sm.Q, sm.jw, sm.info, h->stream));
    {
      Timer tg2(h, tg ? &ga->t : nullptr, 1);
      PFE_HIP(pfe::gemm_tall_f64(n, q, q, X, ld, sm.Q, X, ld, h->stream));
      PFE_HIP(pfe::gemm_tall_f64(n, q, q, W, ld, sm.Q, W, ld, h->stream));
    }
    if (ga) ga->flops += 3.0 * f2;
  }
  {
    Timer tm(h, t_res);
    PFE_HIP(pfe::resid_norms_f64(n, q, W, X, ld, sm.theta, 1.0 / h->lam_ub, sm.res, h->wsRed.p,
                                 h->stream));
    theta.resize(q);
    res.resize(q);
    int info = 0;
    PFE_HIP(hipMemcpyAsync(theta.data(), sm.theta, q * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    PFE_HIP(hipMemcpyAsync(res.data(), sm.res, q * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    PFE_HIP(hipMemcpyAsync(&info, sm.info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    PFE_TRY(sync(h));
    if (info < 0) return pfe::fail(PFE_EHIP, "Jacobi eigensolver did not converge");
  }
  return pfe::ok();
}

double coef_abs_sum(const std::vector<double>& c) {
  double s = 0;
  for (double v : c) s += std::fabs(v);
  return s;
}

}  // namespace

// =================================================================== C-ABI
extern "C" {

const char* pfe_version(void) { return "pfeig 0.1 (gfx950)"; }

static thread_local std::string g_create_err;

static pfe_status create_fail(pfe_ctx* h, pfe_status st, const std::string& msg) {
  g_create_err = msg;
  if (h) {
    for (auto& e : h->ev)
      if (e) (void)hipEventDestroy(e);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
  }
  return st;
}

pfe_status pfe_create(int device, void* hip_stream, pfe_handle* out) {
  if (!out) return create_fail(nullptr, PFE_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess)
    return create_fail(nullptr, PFE_EHIP, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
  if (device < 0 || device >= ndev)
    return create_fail(nullptr, PFE_EINVAL,
                       "device " + std::to_string(device) + " out of range (" + std::to_string(ndev) + " devices)");
  pfe_ctx* h = new (std::nothrow) pfe_ctx();
  if (!h) return create_fail(nullptr, PFE_ENOMEM, "host allocation failed");
  h->device = device;
  if ((e = hipSetDevice(device)) != hipSuccess)
    return create_fail(h, PFE_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  if ((e = init_scratch(device)) != hipSuccess)
    return create_fail(h, PFE_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  if (hip_stream) {
    h->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    // a blocking stream: work on it is ordered against the legacy default
    // stream, where a caller (torch's default stream included) may still be
    // writing the device arrays it passes
    if ((e = hipStreamCreate(&h->stream)) != hipSuccess)
      return create_fail(h, PFE_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    h->own_stream = true;
  }
  if ((e = hipEventCreate(&h->ev[0])) != hipSuccess || (e = hipEventCreate(&h->ev[1])) != hipSuccess ||
      (e = hipEventCreate(&h->ev[2])) != hipSuccess || (e = hipEventCreate(&h->ev[3])) != hipSuccess)
    return create_fail(h, PFE_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
  if ((e = h->flags.ensure(256)) != hipSuccess)
    return create_fail(h, PFE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  g_create_err.clear();
  *out = h;
  return PFE_OK;
}

void pfe_destroy(pfe_handle h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

const char* pfe_last_error(pfe_handle h) { return h ? h->err.c_str() : g_create_err.c_str(); }

int64_t pfe_device_bytes(pfe_handle h) {
  if (!h) return 0;
  const DevBuf* bufs[] = {&h->tile_ptr, &h->tile_vptr, &h->tile_cm, &h->tile_row, &h->tile_perm, &h->Ht,
                          &h->row_ptr, &h->col_idx, &h->H,    &h->transpose, &h->masses,
                          &h->H32,     &h->flags,   &h->wsA,  &h->wsB,       &h->wsC,
                          &h->wsD,     &h->wsSmall, &h->wsRed, &h->wsOut,    &h->wsCk, &h->wsSlice,
                          &h->t32_ptr, &h->t32_vptr, &h->t32_cm, &h->t32_row, &h->t32_perm,
                          &h->w64_ptr, &h->w64_vptr, &h->w64_cm, &h->w64_row, &h->w64_perm, &h->Hw};
  int64_t s = 0;
  for (auto* b : bufs) s += (int64_t)b->bytes;
  return s;
}

void pfe_solve_opts_default(pfe_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->r = std::pow(0.1, 0.25);
  o->smoothing = PFE_SMOOTH_NONE;
  o->tol = 0.0;   // 1e-10 (FP64) or 1e-8 (FP32 filter form)
  o->max_iter = 100;
  o->precision = PFE_FP64;
  o->seed = 11;
  o->locking = 1;
}

// ----------------------------------------------------------- set_hessian
// blocks_dev: `blocks` is device memory whatever PFE_DEVICE_PTRS says (the
// spring assembly hands over its own device buffer).
static Err set_hessian_impl(pfe_handle h, int64_t n_atoms, int64_t nnzb, const int64_t* row_ptr,
                            const int32_t* col_idx, const double* blocks, const double* masses,
                            uint32_t flags, bool blocks_dev = false) {
  PFE_TRY(select_device(h));
  if (n_atoms <= 0 || nnzb < n_atoms || !row_ptr || !col_idx || !blocks)
    return pfe::fail(PFE_EINVAL, "need n_atoms > 0, nnzb >= n_atoms and non-null arrays");
  if (n_atoms > (int64_t)INT32_MAX / 3 || nnzb >= (int64_t)INT32_MAX)
    return pfe::fail(PFE_EINVAL, "sizes exceed the 32-bit index range of the kernels");
  const bool weight = !(flags & PFE_BLOCKS_ARE_H);
  if (weight && !masses) return pfe::fail(PFE_EINVAL, "masses are required unless PFE_BLOCKS_ARE_H");
  const bool dev = (flags & PFE_DEVICE_PTRS) != 0;
  // row pointers checked on the host
  std::vector<int64_t> rp(n_atoms + 1);
  if (dev) {
    PFE_HIP(hipMemcpy(rp.data(), row_ptr, rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(rp.data(), row_ptr, rp.size() * sizeof(int64_t));
  }
  if (rp[0] != 0 || rp[n_atoms] != nnzb)
    return pfe::fail(PFE_EINVAL, "row_ptr must start at 0 and end at nnzb");
  for (int64_t i = 0; i < n_atoms; ++i)
    if (rp[i + 1] <= rp[i]) return pfe::fail(PFE_EINVAL, "every block row needs >= 1 block (the diagonal)");
  h->has_h = h->has_masses = h->has_bounds = false;
  h->h32_c = h->h32_e = NAN;
  h->H32.release();
  h->n_atoms = n_atoms;
  h->nnzb = nnzb;
  PFE_HIP(h->row_ptr.ensure((n_atoms + 1) * sizeof(int64_t)));
  PFE_HIP(h->col_idx.ensure((nnzb + pfe::kBsrPad) * sizeof(int32_t)));
  PFE_HIP(h->H.ensure((size_t)(nnzb + pfe::kBsrPad) * 9 * sizeof(double)));
  PFE_HIP(h->transpose.ensure(nnzb * sizeof(int32_t)));
  PFE_HIP(hipMemsetAsync(h->col_idx.p, 0, (nnzb + pfe::kBsrPad) * sizeof(int32_t), h->stream));
  PFE_HIP(pfe::zero_f64(h->H.as<double>(), (nnzb + pfe::kBsrPad) * 9, h->stream));
  PFE_HIP(hipMemcpyAsync(h->row_ptr.p, rp.data(), rp.size() * sizeof(int64_t),
                         hipMemcpyHostToDevice, h->stream));
  PFE_TRY(upload(h, h->col_idx.as<int32_t>(), col_idx, nnzb, dev));
  PFE_TRY(upload(h, h->H.as<double>(), blocks, nnzb * 9, dev || blocks_dev));
  int* eflag = h->flags.as<int>();
  PFE_HIP(hipMemsetAsync(eflag, 0, sizeof(int), h->stream));
  const pfe::Bsr A = h->bsr();
  PFE_HIP(pfe::validate_bsr(A, h->H.as<double>(), h->transpose.as<int32_t>(), eflag, h->stream));
  if (masses) {
    PFE_HIP(h->masses.ensure(n_atoms * sizeof(double)));
    PFE_TRY(upload(h, h->masses.as<double>(), masses, n_atoms, dev));
    PFE_HIP(pfe::validate_masses(n_atoms, h->masses.as<double>(), eflag, h->stream));
  }
  int ef = 0;
  PFE_HIP(hipMemcpyAsync(&ef, eflag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  PFE_TRY(sync(h));
  if (ef & 1) return pfe::fail(PFE_EINVAL, "column indices out of range, unsorted, or diagonal block missing");
  if (ef & 2) return pfe::fail(PFE_EINVAL, "non-finite block value");
  if (ef & 16) return pfe::fail(PFE_EINVAL, "masses must be finite and > 0");
  if (ef & 4) return pfe::fail(PFE_ENOTSYM, "a block has no transpose partner");
  if (ef & 8) return pfe::fail(PFE_ENOTSYM, "a block differs from its partner's transpose");
  if (weight) {
    PFE_HIP(pfe::mass_weight(A, h->H.as<double>(), h->masses.as<double>(), h->H.as<double>(),
                             h->stream));
  }
  // row tiles for the fused filter step (rows per tile: PFEIG_TILE_ROWS, else
  // the default measured best on MI355X)
  int R = kDefaultTileRows;
  if (const char* e = std::getenv("PFEIG_TILE_ROWS")) R = std::atoi(e);
  // processing order of the rows: PFEIG_ROW_ORDER=0 natural, 1 locality
  // order, unset: chosen from the pattern
  const char* ro = std::getenv("PFEIG_ROW_ORDER");
  const int order_mode = ro ? (std::atoi(ro) != 0 ? 1 : 0) : -1;
  if (R >= 2 && R <= 4) {
    std::vector<int32_t> ci((size_t)nnzb);
    if (dev) {
      PFE_HIP(hipMemcpy(ci.data(), col_idx, nnzb * sizeof(int32_t), hipMemcpyDeviceToHost));
    } else {
      std::memcpy(ci.data(), col_idx, nnzb * sizeof(int32_t));
    }
    const int64_t window = group_window();
    const bool same = h->tile_rows == R && h->tiled_R == R && h->tiled_mode == order_mode &&
                      h->tiled_window == window && h->tiled_rp == rp && h->tiled_ci == ci;
    if (!same) {
      h->tile_rows = 0;
      h->n_tiles = 0;
      h->tiled_R = 0;
      h->release_tiles32();
      h->release_tiles64w();
      std::vector<int64_t> tp, tv, perm;
      std::vector<int32_t> tcm, trow, order;
      // Rows whose neighbours lie far away in the given numbering (an MD
      // snapshot's atom ids, say) are taken in graph-locality order: on the
      // 1e5-atom glass with randomly relabelled atoms the filter step runs
      // 2.2x faster in that order, while a lattice-like numbering is left as
      // it is (its natural order measured 6% faster than the locality order).
      bool local = order_mode == 1;
      if (order_mode < 0) {
        const double far_nat =
            pfe::far_block_fraction(n_atoms, rp.data(), ci.data(), nullptr, kOrderWindow);
        if (far_nat > kOrderFarMax) {
          pfe::locality_order(n_atoms, rp.data(), ci.data(), kOrderLeaf, R, order);
          local = pfe::far_block_fraction(n_atoms, rp.data(), ci.data(), order.data(),
                                          kOrderWindow) < far_nat;
        }
      } else if (local) {
        pfe::locality_order(n_atoms, rp.data(), ci.data(), kOrderLeaf, R, order);
      }
      const int32_t* ord = local ? order.data() : nullptr;
      if (!local && window > 0 && R >= 3) {
        pfe::window_group_order(n_atoms, rp.data(), ci.data(), window, R, order);
        ord = order.data();
      }
      pfe::build_row_tiles(n_atoms, rp.data(), ci.data(), R, ord, tp, tv, tcm, trow, perm);
      PFE_HIP(h->tile_ptr.ensure(tp.size() * sizeof(int64_t)));
      PFE_HIP(h->tile_vptr.ensure(tv.size() * sizeof(int64_t)));
      PFE_HIP(h->tile_cm.ensure(tcm.size() * sizeof(int32_t)));
      PFE_HIP(h->tile_row.ensure(trow.size() * sizeof(int32_t)));
      PFE_HIP(h->tile_perm.ensure(perm.size() * sizeof(int64_t)));
      PFE_HIP(hipMemcpy(h->tile_ptr.p, tp.data(), tp.size() * sizeof(int64_t), hipMemcpyHostToDevice));
      PFE_HIP(hipMemcpy(h->tile_vptr.p, tv.data(), tv.size() * sizeof(int64_t), hipMemcpyHostToDevice));
      PFE_HIP(hipMemcpy(h->tile_cm.p, tcm.data(), tcm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      PFE_HIP(hipMemcpy(h->tile_row.p, trow.data(), trow.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      PFE_HIP(hipMemcpy(h->tile_perm.p, perm.data(), perm.size() * sizeof(int64_t), hipMemcpyHostToDevice));
      h->n_tiles = (int64_t)tp.size() - 1;
      h->tiled_rp = std::move(rp);
      h->tiled_ci = std::move(ci);
      h->tiled_R = R;
      h->tiled_local = local;
      h->tiled_mode = order_mode;
      h->tiled_window = window;
      h->tiled_span = local ? 0 : pfe::neighbour_span(n_atoms, h->tiled_rp.data(), h->tiled_ci.data());
    }
    PFE_HIP(h->Ht.ensure((size_t)(nnzb + pfe::kBsrPad) * 9 * sizeof(double)));
    PFE_HIP(pfe::zero_f64(h->Ht.as<double>(), (nnzb + pfe::kBsrPad) * 9, h->stream));
    PFE_HIP(pfe::permute_blocks_f64(nnzb, h->tile_perm.as<int64_t>(), h->H.as<double>(),
                                    h->Ht.as<double>(), h->stream));
    h->tile_rows = R;
    h->hw_valid = false;   // the wide tiles' values follow at their next use
  } else {
    h->tile_rows = 0;
    h->n_tiles = 0;
    h->tiled_R = 0;
    h->tiled_rp.clear();
    h->tiled_ci.clear();
    h->tile_ptr.release();
    h->tile_vptr.release();
    h->tile_cm.release();
    h->tile_row.release();
    h->tile_perm.release();
    h->Ht.release();
    h->release_tiles32();
    h->release_tiles64w();
  }
  PFE_TRY(sync(h));
  h->has_h = true;
  h->has_masses = masses != nullptr;
  return pfe::ok();
}

pfe_status pfe_set_hessian(pfe_handle h, int64_t n_atoms, int64_t nnzb, const int64_t* row_ptr,
                           const int32_t* col_idx, const double* blocks, const double* masses,
                           uint32_t flags) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return set_hessian_impl(h, n_atoms, nnzb, row_ptr, col_idx, blocks, masses, flags); });
}

// Spring network: K assembled on the device, then the same import as above.
static Err set_springs_impl(pfe_handle h, int64_t n_atoms, int64_t nnzb, const int64_t* row_ptr,
                            const int32_t* col_idx, int64_t P, const int64_t* pairs,
                            const double* unit, const double* k, const double* masses,
                            double* hblocks_out, uint32_t flags) {
  PFE_TRY(select_device(h));
  if (n_atoms <= 0 || P < 0 || !row_ptr || !col_idx || !masses || (P > 0 && (!pairs || !unit || !k)))
    return pfe::fail(PFE_EINVAL, "need n_atoms > 0, n_springs >= 0 and non-null arrays");
  if (nnzb != n_atoms + 2 * P)
    return pfe::fail(PFE_EINVAL, "the pattern must hold the diagonal and both orientations of every spring "
                                 "(nnzb = n_atoms + 2 n_springs)");
  if (n_atoms > (int64_t)INT32_MAX / 3 || nnzb >= (int64_t)INT32_MAX)
    return pfe::fail(PFE_EINVAL, "sizes exceed the 32-bit index range of the kernels");
  const bool dev = (flags & PFE_DEVICE_PTRS) != 0;
  std::vector<int64_t> rp(n_atoms + 1);
  if (dev) {
    PFE_HIP(hipMemcpy(rp.data(), row_ptr, rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(rp.data(), row_ptr, rp.size() * sizeof(int64_t));
  }
  if (rp[0] != 0 || rp[n_atoms] != nnzb)
    return pfe::fail(PFE_EINVAL, "row_ptr must start at 0 and end at nnzb");
  for (int64_t i = 0; i < n_atoms; ++i)
    if (rp[i + 1] < rp[i]) return pfe::fail(PFE_EINVAL, "row_ptr must be non-decreasing");
  // staging: K, and device copies of host inputs
  const size_t bK = (size_t)nnzb * 9 * sizeof(double);
  const size_t need = bK + (dev ? 0 : (size_t)(n_atoms + 1) * 8 + (size_t)nnzb * 4 + (size_t)P * 48) + 256;
  pfe::DevBuf stage;
  PFE_HIP(stage.ensure(need));
  char* base = stage.as<char>();
  double* K = (double*)base;
  const int64_t* rpd = row_ptr;
  const int32_t* cid = col_idx;
  const int64_t* prd = pairs;
  const double* und = unit;
  const double* kd = k;
  if (!dev) {
    int64_t* a = (int64_t*)(base + bK);
    int64_t* b = a + (n_atoms + 1);
    double* c = (double*)(b + 2 * P);
    double* d = c + 3 * P;
    int32_t* e = (int32_t*)(d + P);
    PFE_TRY(upload(h, a, row_ptr, n_atoms + 1, false));
    PFE_TRY(upload(h, b, pairs, 2 * P, false));
    PFE_TRY(upload(h, c, unit, 3 * P, false));
    PFE_TRY(upload(h, d, k, P, false));
    PFE_TRY(upload(h, e, col_idx, nnzb, false));
    rpd = a;
    prd = b;
    und = c;
    kd = d;
    cid = e;
  }
  int* eflag = h->flags.as<int>() + 8;
  PFE_HIP(hipMemsetAsync(eflag, 0, sizeof(int), h->stream));
  PFE_HIP(pfe::assemble_springs(n_atoms, rpd, cid, P, prd, und, kd, K, eflag, h->stream));
  int ef = 0;
  PFE_HIP(hipMemcpyAsync(&ef, eflag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  PFE_TRY(sync(h));
  if (ef & 32) return pfe::fail(PFE_EINVAL, "spring pairs must satisfy 0 <= i < j < n_atoms in strictly increasing order");
  if (ef & 64) return pfe::fail(PFE_EINVAL, "an off-diagonal block of the pattern has no spring");
  if (ef & 1) return pfe::fail(PFE_EINVAL, "diagonal block missing");
  PFE_TRY(set_hessian_impl(h, n_atoms, nnzb, row_ptr, col_idx, K, masses, flags & ~PFE_BLOCKS_ARE_H, true));
  if (hblocks_out) {
    PFE_TRY(download(h, hblocks_out, h->H.as<double>(), nnzb * 9, dev));
    PFE_TRY(sync(h));
  }
  return pfe::ok();
}

pfe_status pfe_set_springs(pfe_handle h, int64_t n_atoms, int64_t nnzb, const int64_t* row_ptr,
                           const int32_t* col_idx, int64_t n_springs, const int64_t* pairs,
                           const double* unit, const double* k, const double* masses,
                           double* hblocks_out, uint32_t flags) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return set_springs_impl(h, n_atoms, nnzb, row_ptr, col_idx, n_springs, pairs, unit, k,
                                    masses, hblocks_out, flags); });
}

// ----------------------------------------------------------------- bounds
static Err bounds_impl(pfe_handle h, int m, const double* v0, uint64_t seed, uint32_t flags,
                       double* lam_lb, double* lam_ub, double* theta_max) {
  PFE_TRY(select_device(h));
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  const int64_t n = h->n();
  if (m < 2 || m > 512 || m > n) return pfe::fail(PFE_EINVAL, "steps must be in [2, min(512, n)]");
  const bool dev = (flags & PFE_DEVICE_PTRS) != 0;
  PFE_HIP(h->wsA.ensure((size_t)(m + 2) * n * sizeof(double)));
  double* V = h->wsA.as<double>();
  double* w = V + (int64_t)(m + 1) * n;
  PFE_HIP(h->wsSmall.ensure((size_t)(4 * m + 8 + 3 * m * m) * sizeof(double) + 64));
  double* alpha = h->wsSmall.as<double>();
  double* beta = alpha + m;
  double* hv = beta + m;
  double* nrm = hv + m + 4;
  double* Tm = nrm + 4;
  double* evals = Tm + (int64_t)m * m;
  double* Qm = evals + m;
  PFE_HIP(h->wsRed.ensure(std::max(pfe::multidot_work_bytes(n, m + 1), pfe::colnorm_work_bytes(n, 1)) +
                          pfe::jacobi_work_bytes(m) + 64));
  double* red = h->wsRed.as<double>();
  double* jw = red + std::max(pfe::multidot_work_bytes(n, m + 1), pfe::colnorm_work_bytes(n, 1)) / sizeof(double);
  int* info = h->flags.as<int>() + 4;
  if (v0) {
    PFE_TRY(upload(h, V, v0, n, dev));
  } else {
    PFE_HIP(pfe::gaussian_fill_f64(n, 1, V, 1, seed, h->stream));
  }
  const pfe::Bsr A = h->bsr();
  const double* Hv = h->H.as<double>();
  PFE_HIP(pfe::col_norms_f64(n, 1, V, 1, nrm, red, h->stream));
  PFE_HIP(pfe::scale_by_inv_f64(n, V, nrm, V, h->stream));
  for (int j = 0; j < m; ++j) {
    double* vj = V + (int64_t)j * n;
    PFE_HIP(pfe::spmv_f64(A, Hv, vj, w, h->stream));
    PFE_HIP(pfe::multi_dot_f64(n, 1, vj, w, alpha + j, red, h->stream));
    PFE_HIP(pfe::multi_axpy_f64(n, 1, vj, alpha + j, w, h->stream));
    if (j > 0) PFE_HIP(pfe::multi_axpy_f64(n, 1, vj - n, beta + j - 1, w, h->stream));
    for (int pass = 0; pass < 2; ++pass) {
      PFE_HIP(pfe::multi_dot_f64(n, j + 1, V, w, hv, red, h->stream));
      PFE_HIP(pfe::multi_axpy_f64(n, j + 1, V, hv, w, h->stream));
    }
    PFE_HIP(pfe::col_norms_f64(n, 1, w, 1, beta + j, red, h->stream));
    PFE_HIP(pfe::scale_by_inv_f64(n, w, beta + j, vj + n, h->stream));
  }
  std::vector<double> ha(m), hb(m);
  PFE_HIP(hipMemcpyAsync(ha.data(), alpha, m * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  PFE_HIP(hipMemcpyAsync(hb.data(), beta, m * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  PFE_TRY(sync(h));
  // an invariant subspace ends the recurrence early
  int mm = m;
  for (int j = 0; j < m; ++j)
    if (!(hb[j] > 1e-300) || !std::isfinite(hb[j])) {
      mm = j + 1;
      break;
    }
  for (int j = 0; j < mm; ++j)
    if (!std::isfinite(ha[j])) return pfe::fail(PFE_EINVAL, "Lanczos produced non-finite values");
  std::vector<double> Th((size_t)mm * mm, 0.0);
  for (int j = 0; j < mm; ++j) {
    Th[(size_t)j * mm + j] = ha[j];
    if (j + 1 < mm) Th[(size_t)j * mm + j + 1] = Th[(size_t)(j + 1) * mm + j] = hb[j];
  }
  PFE_HIP(hipMemcpyAsync(Tm, Th.data(), Th.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
  PFE_HIP(pfe::sym_eig_f64(mm, Tm, evals, Qm, jw, info, h->stream));
  std::vector<double> ev(mm), Qh((size_t)mm * mm);
  PFE_HIP(hipMemcpyAsync(ev.data(), evals, mm * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  PFE_HIP(hipMemcpyAsync(Qh.data(), Qm, Qh.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  PFE_TRY(sync(h));
  const double th = ev[mm - 1];
  const double s_last = Qh[(size_t)(mm - 1) * mm + (mm - 1)];
  const double bm = (mm == m) ? hb[m - 1] : 0.0;
  const double ub = th + std::fabs(bm * s_last);
  h->lam_lb = 0.0;
  h->lam_ub = ub;
  h->has_bounds = true;
  if (lam_lb) *lam_lb = 0.0;
  if (lam_ub) *lam_ub = ub;
  if (theta_max) *theta_max = th;
  return pfe::ok();
}

pfe_status pfe_estimate_bounds(pfe_handle h, int32_t steps, const double* v0, uint64_t seed,
                               uint32_t flags, double* lam_lb, double* lam_ub, double* theta_max) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return bounds_impl(h, steps, v0, seed, flags, lam_lb, lam_ub, theta_max); });
}

pfe_status pfe_set_bounds(pfe_handle h, double lam_lb, double lam_ub) {
  if (!h) return PFE_EINVAL;
  if (!(lam_ub > lam_lb) || !std::isfinite(lam_lb) || !std::isfinite(lam_ub))
    return finish(h, pfe::fail(PFE_EINVAL, "need finite lam_lb < lam_ub"));
  h->lam_lb = lam_lb;
  h->lam_ub = lam_ub;
  h->has_bounds = true;
  return finish(h, pfe::ok());
}

// ---------------------------------------------------------------- design
pfe_status pfe_design_filter(double lam_lo, double lam_hi, double lam_lb, double lam_ub,
                             const pfe_filter_opts* opts, double* coef_out, int32_t coef_cap,
                             pfe_filter* out) {
  return host_guarded([&]() -> pfe_status {
    if (!opts || !out) return PFE_EINVAL;
    pfe::FilterDesign f;
    Err e = pfe::design_filter(lam_lo, lam_hi, lam_lb, lam_ub, opts->degree, opts->eps, opts->r,
                               opts->smoothing, &f);
    if (e) return e.st;
    out->degree = f.degree;
    out->smoothing = f.smoothing;
    out->c = f.c;
    out->e = f.e;
    out->xi = f.xi;
    out->eta = f.eta;
    out->eps = f.eps;
    out->coef = nullptr;
    if (!coef_out || coef_cap < f.degree + 1) return PFE_ECAPACITY;
    std::memcpy(coef_out, f.coef.data(), (f.degree + 1) * sizeof(double));
    out->coef = coef_out;
    return PFE_OK;
  });
}

// ----------------------------------------------------------- apply_filter
static Err apply_impl(pfe_handle h, const pfe_filter* f, int nvec, const void* X, void* Y,
                      int64_t ld, int precision, uint32_t flags) {
  PFE_TRY(select_device(h));
  PFE_TRY(check_filter(h, f));
  if (nvec < 1 || ld < nvec || !X || !Y) return pfe::fail(PFE_EINVAL, "need 1 <= nvec <= ld and arrays");
  if (precision != PFE_FP64 && precision != PFE_FP32) return pfe::fail(PFE_EINVAL, "precision");
  const bool dev = (flags & PFE_DEVICE_PTRS) != 0;
  const int64_t n = h->n();
  const size_t elem = precision == PFE_FP64 ? 8 : 4;
  const size_t mv = (size_t)n * ld * elem;
  std::vector<double> coef(f->coef, f->coef + f->degree + 1);
  PFE_HIP(h->wsA.ensure(mv));
  if (!dev) {
    PFE_HIP(h->wsC.ensure(mv));
    PFE_HIP(h->wsD.ensure(mv));
  }
  const void* Xd = X;
  void* Yd = Y;
  if (!dev) {
    PFE_HIP(hipMemcpyAsync(h->wsC.p, X, mv, hipMemcpyHostToDevice, h->stream));
    Xd = h->wsC.p;
    Yd = h->wsD.p;
  }
  if (precision == PFE_FP64) {
    pfe::Bsr A64;
    const double* v64 = nullptr;
    PFE_TRY(filter_set64(h, nvec, &A64, &v64));
    PFE_TRY(run_filter<double>(h, v64, coef, 1.0 / f->e, -f->c / f->e, (const double*)Xd,
                               (double*)Yd, h->wsA.as<double>(), nvec, ld, nullptr, &A64));
  } else {
    PFE_TRY(ensure_h32(h, f->c, f->e, nvec));
    PFE_TRY(run_filter<float>(h, h->H32.as<float>(), coef, 1.0, 0.0, (const float*)Xd,
                              (float*)Yd, h->wsA.as<float>(), nvec, ld, nullptr));
  }
  if (!dev) PFE_HIP(hipMemcpyAsync(Y, Yd, mv, hipMemcpyDeviceToHost, h->stream));
  PFE_TRY(sync(h));
  return pfe::ok();
}

pfe_status pfe_apply_filter(pfe_handle h, const pfe_filter* f, int32_t nvec, const void* X,
                            void* Y, int64_t ld, int32_t precision, uint32_t flags) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return apply_impl(h, f, nvec, X, Y, ld, precision, flags); });
}

// The FP64 filter of apply_impl on device arrays with the recurrence's
// scratch multivector in `scratch`: no allocation, no synchronisation.
static Err apply_noalloc_impl(pfe_handle h, const pfe_filter* f, int nvec, const double* X,
                              double* Y, int64_t ld) {
  PFE_TRY(select_device(h));
  PFE_TRY(check_filter(h, f));
  if (nvec < 1 || ld < nvec || !X || !Y) return pfe::fail(PFE_EINVAL, "need 1 <= nvec <= ld and arrays");
  double* Q = static_cast<double*>(scratch_addr(h->device));
  if (!Q) return pfe::fail(PFE_ESTATE, "no scratch address for this device");
  const int64_t n = h->n();
  const double bytes = (double)n * (double)ld * sizeof(double);
  if (bytes > (double)kNoAllocScratchBytes)
    return pfe::fail(PFE_EINVAL, "n * ld * 8 = " + std::to_string((long long)bytes) +
                                     " bytes exceeds the allocation-free scratch of " +
                                     std::to_string((long long)kNoAllocScratchBytes) + " bytes");
  const uintptr_t x0 = reinterpret_cast<uintptr_t>(X), y0 = reinterpret_cast<uintptr_t>(Y);
  const uintptr_t span = (uintptr_t)bytes;
  if (x0 < y0 + span && y0 < x0 + span) return pfe::fail(PFE_EINVAL, "X and Y overlap");
  PFE_TRY(run_filter<double>(h, h->step_vals64(), f->coef, f->degree, 1.0 / f->e, -f->c / f->e, X,
                             Y, Q, nvec, ld, nullptr));
  return pfe::ok();
}

pfe_status pfe_apply_filter_noalloc(pfe_handle h, const pfe_filter* f, int32_t nvec,
                                    const double* X, double* Y, int64_t ld) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return apply_noalloc_impl(h, f, nvec, X, Y, ld); });
}

// ------------------------------------------------------------------ solve
static Err solve_impl(pfe_handle h, double lam_lo, double lam_hi, int nev,
                      const pfe_solve_opts* o_in, int* n_found, double* evals, double* evecs,
                      double* resid, pfe_solve_stats* st_out) {
  const auto t0 = std::chrono::steady_clock::now();
  PFE_TRY(select_device(h));
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  if (!h->has_bounds) return pfe::fail(PFE_ESTATE, "no spectral bounds (estimate_bounds or set_bounds)");
  pfe_solve_opts o;
  pfe_solve_opts_default(&o);
  if (o_in) o = *o_in;
  if (o.tol <= 0) o.tol = (o.precision == PFE_FP32) ? 1e-8 : 1e-10;
  if (o.max_iter <= 0) o.max_iter = 100;
  if (o.r == 0) o.r = std::pow(0.1, 0.25);
  const int q = o.block;
  const int64_t n = h->n();
  if (q < 1 || q > 256 || q > n) return pfe::fail(PFE_EINVAL, "block must be in [1, min(256, n)]");
  if (nev < 0 || !n_found) return pfe::fail(PFE_EINVAL, "nev >= 0 and n_found required");
  if (o.precision != PFE_FP64 && o.precision != PFE_FP32) return pfe::fail(PFE_EINVAL, "precision");
  if (lam_lo < h->lam_lb || lam_hi > h->lam_ub)
    return pfe::fail(PFE_EINVAL, "window must lie inside [lam_lb, lam_ub]");
  pfe::FilterDesign fd;
  PFE_TRY(pfe::design_filter(lam_lo, lam_hi, h->lam_lb, h->lam_ub, o.degree, o.eps, o.r,
                             o.smoothing, &fd));
  pfe_solve_stats st;
  std::memset(&st, 0, sizeof(st));
  st.degree = fd.degree;
  st.eps = fd.eps;
  st.c = fd.c;
  st.e = fd.e;
  st.xi = fd.xi;
  st.eta = fd.eta;

  const bool mixed = o.precision == PFE_FP32;
  const char* tr_env = std::getenv("PFEIG_TRACE");
  const bool trace = tr_env && tr_env[0] && tr_env[0] != '0';
  const int64_t ld = round_up(q, 8);
  const size_t mv64 = (size_t)n * ld * sizeof(double);
  // FP64 form: X, W and one FP64 scratch.  Mixed form: X64, W64 and a
  // 12-byte/element region holding X32, P32, Q32 (or, for the refinement
  // sweep, one FP64 scratch).
  PFE_HIP(h->wsA.ensure(mv64));
  PFE_HIP(h->wsB.ensure(mv64));
  PFE_HIP(h->wsC.ensure(mixed ? (size_t)n * ld * 12 : mv64));
  double* X = h->wsA.as<double>();
  double* W = h->wsB.as<double>();
  char* R = h->wsC.as<char>();
  PFE_HIP(pfe::zero_f64(X, n * ld, h->stream));
  PFE_HIP(pfe::zero_f64(W, n * ld, h->stream));
  PFE_HIP(pfe::zero_f64((double*)R, (int64_t)(mixed ? n * ld * 12 : mv64) / 8, h->stream));
  Small sm;
  PFE_TRY(alloc_small(h, q, &sm));
  PFE_TRY(ensure_red(h, n, q));
  if (o.x0) {
    if (o.flags & PFE_DEVICE_PTRS) {
      PFE_HIP(pfe::copy_cols_f64(n, q, o.x0, q, X, ld, h->stream));
    } else {
      PFE_TRY(upload_block(h, X, ld, o.x0, q, n, W));
    }
  } else {
    PFE_HIP(pfe::gaussian_fill_f64(n, q, X, ld, o.seed, h->stream));
  }
  if (mixed) PFE_TRY(ensure_h32(h, fd.c, fd.e, q));
  double bound = 1.05 * coef_abs_sum(fd.coef) + 1e-12;
  int stall = 0;
  const int max_degree = std::min(200000, 8 * std::max(fd.degree, 1));
  {
    Timer tm(h, &st.t_orth);
    PFE_TRY(cholqr2(h, sm, X, n, q, ld, -1.0, nullptr, &st.shifted_passes, true));
  }
  const double delta = 1e-6 * h->lam_ub;
  std::vector<double> theta, res;
  int prev_cnt = -1;
  bool converged = false;
  bool fp64_phase = !mixed;
  double prev_max = HUGE_VAL;
  const pfe::Bsr A = h->bsr();
  std::vector<int> perm(q);
  GemmAcct ga;
  ga.on = true;
  const int max_sweeps = o.refine_sweeps > 0 ? o.refine_sweeps : 1;
  int refine_m = 1;         // filter applications of the current refinement sweep
  double refine_kap = 0.0;  // contraction per application it was sized for
  double good_ratio = 0.0;  // the FP32 phase's last contraction below 0.5 per iteration
  for (int it = 1; it <= o.max_iter; ++it) {
    // Locking: the Ritz vectors of the last Rayleigh-Ritz step that lie in the
    // window with residual <= tol are not filtered.  The others (rounded up
    // to a multiple of 8 columns, so the filter keeps its wide aligned loads)
    // come first; the locked ones follow unfiltered.  Orthonormalisation and
    // Rayleigh-Ritz act on the span of all q columns.
    // A pair locks at a tenth of tol: the Rayleigh-Ritz step on the full span
    // moves a locked vector's residual a little, and one locked just below
    // tol would cross it again and hold up the stop rule.
    int nf = q;
    if (o.locking && !theta.empty() && !(fp64_phase && mixed)) {
      const double lock_tol = 0.1 * o.tol;
      auto locked = [&](int j) {
        return theta[j] >= lam_lo && theta[j] <= lam_hi && res[j] <= lock_tol;
      };
      int na = 0;
      for (int j = 0; j < q; ++j)
        if (!locked(j)) perm[na++] = j;
      int nl = na;
      for (int j = 0; j < q; ++j)
        if (locked(j)) perm[nl++] = j;
      nf = std::min<int>(q, (int)round_up(std::max(na, 1), 8));
    }
    // Y = p(H_hat) X into W (X is read only), then Y is orthonormalised in
    // place and becomes the next basis: the X and W buffers swap roles.
    // With locked columns, X is first permuted into W, the filter runs from
    // W's leading nf columns into X, and the locked columns are copied after
    // them; then no swap is needed.
    double* Fin = X;
    double* Fout = W;
    if (nf < q) {
      PFE_HIP(hipMemcpyAsync(sm.sel, perm.data(), q * sizeof(int), hipMemcpyHostToDevice, h->stream));
      PFE_HIP(pfe::permute_cols_f64(n, q, X, ld, sm.sel, W, h->stream));
      PFE_HIP(pfe::copy_cols_f64(n, q - nf, W + nf, ld, X + nf, ld, h->stream));
      Fin = W;
      Fout = X;
    }
    st.filter_columns += nf;
    if (fp64_phase) {
      // A refinement sweep of the FP32 form applies the filter refine_m
      // times, orthonormalising between applications (Algorithm 4's QR after
      // every filter step, its Rayleigh-Ritz step only after the last);
      // otherwise once.
      const int reps = (mixed && st.refined) ? refine_m : 1;
      for (int rep = 0; rep < reps; ++rep) {
        if (rep > 0) {
          {
            Timer tm(h, &st.t_orth);
            PFE_TRY(cholqr2(h, sm, Fout, n, q, ld, bound, &ga, &st.shifted_passes));
          }
          std::swap(Fin, Fout);
          st.filter_columns += nf;
        }
        pfe::Bsr A64;
        const double* v64 = nullptr;
        PFE_TRY(filter_set64(h, q, &A64, &v64));
        Timer tm(h, &st.t_filter);
        PFE_TRY(run_filter<double>(h, v64, fd.coef, 1.0 / fd.e, -fd.c / fd.e, Fin, Fout,
                                   (double*)R, nf, ld, &st.filter_steps, &A64));
        st.filter_bytes += filter_bytes(h->n_atoms, h->nnzb, nf, 8, fd.degree);
        if (mixed) st.refine_applications++;
        if (trace && reps > 1) {
          PFE_TRY(sync(h));
          std::fprintf(stderr, "[pfeig]   FP64 application %d of %d done t=%.3fs\n", rep + 1, reps,
                       std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
        }
      }
      st.fp64_iterations++;
    } else {
      float* X32 = (float*)R;
      float* P32 = X32 + n * ld;
      float* Q32 = P32 + n * ld;
      Timer tm(h, &st.t_filter);
      PFE_HIP(pfe::cast_f64_to_f32(n, nf, Fin, ld, X32, ld, h->stream));
      PFE_TRY(run_filter<float>(h, h->H32.as<float>(), fd.coef, 1.0, 0.0, X32, P32, Q32, nf, ld,
                                &st.filter_steps));
      PFE_HIP(pfe::cast_f32_to_f64(n, nf, P32, ld, Fout, ld, h->stream));
      st.filter_bytes += filter_bytes(h->n_atoms, h->nnzb, nf, 4, fd.degree);
    }
    {
      // Filtered columns obey the filter's bound; locked ones were carried
      // over unfiltered with unit norm, so with any locked column the bound
      // on the largest column norm is at least 1.
      const double nbound = nf < q ? std::max(bound, 1.0 + 1e-9) : bound;
      Timer tm(h, &st.t_orth);
      PFE_TRY(cholqr2(h, sm, Fout, n, q, ld, nbound, &ga, &st.shifted_passes));
    }
    if (Fout == W) {
      std::swap(h->wsA.p, h->wsB.p);
      std::swap(h->wsA.bytes, h->wsB.bytes);
      X = h->wsA.as<double>();
      W = h->wsB.as<double>();
    }
    PFE_TRY(rayleigh_ritz(h, sm, X, W, n, q, ld, theta, res, &st.t_rr, &st.t_resid, &ga));
    st.iterations = it;
    int cnt = 0;
    bool ok_all = true;
    double mx = 0.0;
    for (int j = 0; j < q; ++j) {
      if (theta[j] >= lam_lo - delta && theta[j] <= lam_hi + delta) {
        ok_all = ok_all && res[j] <= o.tol;
        mx = std::max(mx, res[j]);
      }
      if (theta[j] >= lam_lo && theta[j] <= lam_hi) ++cnt;
    }
    // Contraction of the slowest wanted Ritz vector per filter application:
    // its error along an eigenvector outside the subspace shrinks by
    // |pi(lambda)| / |pi(theta_i)| per application, and every eigenvalue
    // outside the subspace has |pi| at most the smallest |pi| of the q Ritz
    // values (the subspace holds the q largest), so min_j |pi(theta_j)| over
    // the smallest near-window |pi(theta_i)| bounds the rate.
    auto rate_bound = [&]() {
      double pall = HUGE_VAL, pwin = HUGE_VAL;
      for (int j = 0; j < q; ++j) {
        const double x = std::min(1.0, std::max(-1.0, (theta[j] - fd.c) / fd.e));
        const double v = std::fabs(pfe::cheb_value(fd.coef, x));
        pall = std::min(pall, v);
        if (theta[j] >= lam_lo - delta && theta[j] <= lam_hi + delta) pwin = std::min(pwin, v);
      }
      if (!(pwin > 0) || !std::isfinite(pwin)) return 0.0;
      return std::min(pall / pwin, 1.0);
    };
    // Filter applications a refinement sweep needs to take the largest
    // near-window residual from rho to tol at rate kap (at most
    // kMaxRefineApps).
    auto sweep_apps = [&](double rho, double kap) {
      kap = std::min(kap, 0.95);
      if (!(rho > o.tol) || !(kap > 0)) return 1;
      const double m = std::ceil(std::log(o.tol / rho) / std::log(kap));
      return (int)std::min<double>(kMaxRefineApps, std::max(1.0, m));
    };
    if (trace)
      std::fprintf(stderr, "[pfeig] it %d %s in-window %d max-resid(near) %.3e rate-bound %.3e t=%.3fs\n",
                   it, fp64_phase ? "fp64" : "fp32", cnt, mx, rate_bound(),
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    if (fp64_phase && mixed) {
      // after the FP64 refinement sweep: done, or ENOCONV with the converged
      // pairs, unless the caller allows further sweeps
      if (ok_all) {
        converged = true;
        break;
      }
      if (st.refined >= max_sweeps) break;
      ++st.refined;
      // the sweep just run measured the rate (its first application also
      // removed the FP32 rounding, so the measured rate can be too low)
      const double measured = std::pow(mx / prev_max, 1.0 / refine_m);
      refine_kap = std::max({refine_kap, rate_bound(), measured});
      refine_m = sweep_apps(mx, refine_kap);
      if (trace) std::fprintf(stderr, "[pfeig] refinement sweep %d: %d FP64 filter applications\n",
                              st.refined, refine_m);
      prev_cnt = cnt;
      prev_max = mx;
      continue;
    }
    // Stop as Algorithm 4 does once the wanted pairs have converged: every
    // Ritz value near the window meets tol, and the in-window count is the
    // one of the previous iteration (the count is the only sign of a pair
    // still entering the window).
    if (ok_all && cnt == prev_cnt && it >= 3) {
      converged = true;
      break;
    }
    // A plateau far above the FP32 rounding level means the filter cannot
    // separate the window from eigenvalues in its margin (the block holds
    // fewer vectors than [xi - eps, eta + eps] has eigenvalues, Sec. 2.6):
    // raise the degree 1.5-fold, which shrinks eps by eq. thresh.
    // In the FP32 phase only a plateau above kFp32Floor counts: FP32 rounding
    // floors lie below it (2.1e-6 at degree 400 on 1e5 atoms, 1.1e-5 at degree
    // 1200 on 1e6), and a higher degree would only raise them.
    const bool plateau = it >= 3 && cnt == prev_cnt && mx > 0.7 * prev_max;
    stall = plateau ? stall + 1 : 0;
    const double stall_floor = fp64_phase ? o.tol : kFp32Floor;
    if (stall >= 3 && mx > stall_floor && fd.degree < max_degree) {
      const int nd = std::min(max_degree, (int)std::ceil(1.5 * fd.degree));
      PFE_TRY(pfe::design_filter(lam_lo, lam_hi, h->lam_lb, h->lam_ub, nd, 0.0, o.r, o.smoothing, &fd));
      bound = 1.05 * coef_abs_sum(fd.coef) + 1e-12;
      st.degree = fd.degree;
      st.eps = fd.eps;
      stall = 0;
      if (trace) std::fprintf(stderr, "[pfeig] plateau: degree raised to %d (eps %.3e)\n", fd.degree, fd.eps);
    }
    const bool have_prev = prev_max > 0 && std::isfinite(prev_max);
    if (!fp64_phase && have_prev && mx > 0 && mx < 0.5 * prev_max) good_ratio = mx / prev_max;
    if (!fp64_phase && it >= 2 && std::abs(cnt - prev_cnt) <= std::max(2, cnt / 50) &&
        ((have_prev && mx > 0.5 * prev_max && mx <= kFp32Floor) || mx <= 30.0 * o.tol)) {
      // FP32 iterations have stalled at their rounding level (or are within
      // reach of tol): the FP64 refinement sweep from here.  The in-window
      // count need not have settled: on a large instance the FP32 plateau can
      // leave Ritz values off by about the window's width (4e6 atoms,
      // q = 256: residuals of 1.3e-4 of lam_ub against a window 1.4e-4 of it
      // wide), so the count may still drift by a few (at most 2 % of it)
      // until the sweep, after which the stop test takes it as it is.  The
      // sweep's rate is the larger of the Ritz values' bound and the last
      // contraction the FP32
      // iterations showed before the plateau, i.e. the last one below 0.5
      // (the plateau's own ratios are near 1; the bound can come out low
      // when the block holds many more vectors than the window, whose Ritz
      // values are poor).  The plateau is FP32 rounding spread over every
      // eigendirection, most of which the first FP64 application removes;
      // what decays at the slow rate is at most the previous iteration's
      // residual times that rate.
      fp64_phase = true;
      st.refined = 1;
      refine_kap = std::max(rate_bound(), good_ratio);
      refine_m = sweep_apps(std::min(mx, refine_kap * prev_max), refine_kap);
      if (trace) std::fprintf(stderr, "[pfeig] refinement sweep 1: %d FP64 filter applications\n",
                              refine_m);
    }
    prev_cnt = cnt;
    prev_max = mx;
  }
  st.gemm_flops = ga.flops;
  st.t_gemm = ga.t;
  // in-window selection (ascending theta)
  std::vector<int> sel;
  for (int j = 0; j < q; ++j)
    if (theta[j] >= lam_lo && theta[j] <= lam_hi && (converged || res[j] <= o.tol)) sel.push_back(j);
  int total_in = 0;
  for (int j = 0; j < q; ++j)
    if (theta[j] >= lam_lo && theta[j] <= lam_hi) ++total_in;
  st.n_window = total_in;
  const auto t1 = std::chrono::steady_clock::now();
  st.t_total = std::chrono::duration<double>(t1 - t0).count();
  if (st_out) *st_out = st;
  if (total_in > nev) {
    *n_found = total_in;
    return pfe::fail(PFE_ECAPACITY, "more eigenvalues in the window than nev");
  }
  if (total_in >= q && q < n) {
    // every Ritz value lies in the window: the subspace cannot show that the
    // window holds no more eigenvalues (Sec. 2.6 asks q above the count)
    *n_found = total_in;
    return pfe::fail(PFE_ECAPACITY, "block too small: every Ritz value lies in the window");
  }
  const int ns = (int)sel.size();
  *n_found = ns;
  double maxr = 0;
  for (int s = 0; s < ns; ++s) {
    if (evals) evals[s] = theta[sel[s]];
    if (resid) resid[s] = res[sel[s]];
    maxr = std::max(maxr, res[sel[s]]);
  }
  if (evecs && ns > 0) {
    PFE_HIP(hipMemcpyAsync(sm.sel, sel.data(), ns * sizeof(int), hipMemcpyHostToDevice, h->stream));
    const bool dev_out = (o.flags & PFE_DEVICE_PTRS) != 0;
    double* dst = evecs;
    if (!dev_out) {
      PFE_HIP(h->wsOut.ensure((size_t)ns * n * sizeof(double)));
      dst = h->wsOut.as<double>();
    }
    PFE_HIP(pfe::gather_transpose_signfix(n, ns, X, ld, sm.sel, dst, h->wsRed.p, h->stream));
    if (!dev_out)
      PFE_HIP(hipMemcpyAsync(evecs, dst, (size_t)ns * n * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    PFE_TRY(sync(h));
  }
  st.max_resid = maxr;
  st.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st_out) *st_out = st;
  (void)A;
  if (!converged) return pfe::fail(PFE_ENOCONV, "not converged within max_iter (or after the refinement sweep)");
  return pfe::ok();
}

pfe_status pfe_solve_interval(pfe_handle h, double lam_lo, double lam_hi, int32_t nev,
                              const pfe_solve_opts* opts, int32_t* n_found, double* evals,
                              double* evecs, double* resid, pfe_solve_stats* stats) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return solve_impl(h, lam_lo, lam_hi, nev, opts, n_found, evals, evecs, resid, stats); });
}

// ------------------------------------------------------------------ count
static Err count_impl(pfe_handle h, double lam_lo, double lam_hi, int degree, int smoothing,
                      int M, const double* V, uint64_t seed, uint32_t flags, double* count) {
  PFE_TRY(select_device(h));
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  if (!h->has_bounds) return pfe::fail(PFE_ESTATE, "no spectral bounds");
  if (degree < 0 || M < 1 || !count || smoothing < 0 || smoothing > 2)
    return pfe::fail(PFE_EINVAL, "degree >= 0, nsamples >= 1, smoothing, count");
  const int64_t n = h->n();
  const double c = 0.5 * (h->lam_ub + h->lam_lb), e = 0.5 * (h->lam_ub - h->lam_lb);
  std::vector<double> coef = pfe::chi_coefficients((lam_lo - c) / e, (lam_hi - c) / e, degree, smoothing);
  const int64_t ld = round_up(M, 8);
  const size_t mv = (size_t)n * ld * sizeof(double);
  PFE_HIP(h->wsA.ensure(mv));
  PFE_HIP(h->wsB.ensure(mv));
  PFE_HIP(h->wsC.ensure(mv));
  double* Vd = h->wsA.as<double>();
  PFE_HIP(pfe::zero_f64(Vd, n * ld, h->stream));
  if (V) {
    if (flags & PFE_DEVICE_PTRS) {
      PFE_HIP(pfe::copy_cols_f64(n, M, V, M, Vd, ld, h->stream));
    } else {
      PFE_TRY(upload_block(h, Vd, ld, V, M, n, h->wsB.as<double>()));
    }
  } else {
    PFE_HIP(pfe::gaussian_fill_f64(n, M, Vd, ld, seed, h->stream));
  }
  PFE_TRY(ensure_red(h, n, M));
  PFE_HIP(h->wsSmall.ensure((size_t)2 * M * sizeof(double) + 64));
  double* nrm = h->wsSmall.as<double>();
  double* dots = nrm + M;
  PFE_HIP(pfe::col_norms_f64(n, M, Vd, ld, nrm, h->wsRed.p, h->stream));
  PFE_HIP(pfe::col_scale_inv_f64(n, M, Vd, ld, nrm, h->stream));
  double* Y = h->wsB.as<double>();
  PFE_TRY(run_filter<double>(h, h->step_vals64(), coef, 1.0 / e, -c / e, Vd, Y,
                             h->wsC.as<double>(), M, ld, nullptr));
  PFE_HIP(pfe::col_dots_f64(n, M, Vd, Y, ld, dots, h->wsRed.p, h->stream));
  std::vector<double> hd(M);
  PFE_HIP(hipMemcpyAsync(hd.data(), dots, M * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  PFE_TRY(sync(h));
  double s = 0;
  for (double v : hd) s += v;
  *count = (double)n / M * s;
  return pfe::ok();
}

pfe_status pfe_estimate_count(pfe_handle h, double lam_lo, double lam_hi, int32_t degree,
                              int32_t smoothing, int32_t nsamples, const double* V, uint64_t seed,
                              uint32_t flags, double* count) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return count_impl(h, lam_lo, lam_hi, degree, smoothing, nsamples, V, seed, flags,
                              count); });
}

// ---------------------------------------------------------------- moments
// mu_k = (1/M) sum_l v_l^T T_k(H_hat) v_l, k = 0..K, for M unit probe vectors,
// by the three-term recurrence (eq. 3-term-recurrence) with one column-dot
// reduction per step.  Any window's count estimate of eq.
// eigval_count_estimator is then n sum_k chi_k mu_k.
static Err moments_impl(pfe_handle h, int K, int M, const double* V, uint64_t seed, uint32_t flags,
                        std::vector<double>* mu) {
  PFE_TRY(select_device(h));
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  if (!h->has_bounds) return pfe::fail(PFE_ESTATE, "no spectral bounds");
  if (K < 0 || K > 100000 || M < 1 || M > 256) return pfe::fail(PFE_EINVAL, "need 0 <= K <= 100000, 1 <= nsamples <= 256");
  const int64_t n = h->n();
  const double c = 0.5 * (h->lam_ub + h->lam_lb), e = 0.5 * (h->lam_ub - h->lam_lb);
  const int64_t ld = round_up(M, 8);
  const size_t mv = (size_t)n * ld * sizeof(double);
  PFE_HIP(h->wsA.ensure(mv));
  PFE_HIP(h->wsB.ensure(mv));
  PFE_HIP(h->wsC.ensure(mv));
  double* Vd = h->wsA.as<double>();
  double* Ta = h->wsB.as<double>();
  double* Tb = h->wsC.as<double>();
  PFE_HIP(pfe::zero_f64(Vd, n * ld, h->stream));
  if (V) {
    if (flags & PFE_DEVICE_PTRS) {
      PFE_HIP(pfe::copy_cols_f64(n, M, V, M, Vd, ld, h->stream));
    } else {
      PFE_TRY(upload_block(h, Vd, ld, V, M, n, h->wsB.as<double>()));
    }
  } else {
    PFE_HIP(pfe::gaussian_fill_f64(n, M, Vd, ld, seed, h->stream));
  }
  PFE_TRY(ensure_red(h, n, M));
  PFE_HIP(h->wsSmall.ensure((size_t)(M + (int64_t)(K + 1) * M) * sizeof(double) + 64));
  double* nrm = h->wsSmall.as<double>();
  double* dots = nrm + M;
  PFE_HIP(pfe::col_norms_f64(n, M, Vd, ld, nrm, h->wsRed.p, h->stream));
  PFE_HIP(pfe::col_scale_inv_f64(n, M, Vd, ld, nrm, h->stream));
  const pfe::Bsr A = h->bsr();
  const double* Hv = h->step_vals64();
  const double a1 = 1.0 / e, b1 = -c / e;
  PFE_HIP(pfe::col_dots_f64(n, M, Vd, Vd, ld, dots, h->wsRed.p, h->stream));
  if (K >= 1) {
    PFE_HIP(pfe::cheb_step_f64(A, Hv, Vd, nullptr, nullptr, Ta, M, ld, a1, b1, 0.0, 0.0, h->stream));
    PFE_HIP(pfe::col_dots_f64(n, M, Vd, Ta, ld, dots + M, h->wsRed.p, h->stream));
  }
  // t_{k+1} = 2 H_hat t_k - t_{k-1}, written over t_{k-1}
  const double* tprev = Vd;
  double* tcur = Ta;
  double* spare = Tb;
  for (int k = 1; k < K; ++k) {
    double* tnext = (tprev == Vd) ? spare : const_cast<double*>(tprev);
    PFE_HIP(pfe::cheb_step_f64(A, Hv, tcur, tprev, nullptr, tnext, M, ld, 2.0 * a1, 2.0 * b1, -1.0,
                               0.0, h->stream));
    PFE_HIP(pfe::col_dots_f64(n, M, Vd, tnext, ld, dots + (int64_t)(k + 1) * M, h->wsRed.p, h->stream));
    tprev = tcur;
    tcur = tnext;
  }
  std::vector<double> hd((size_t)(K + 1) * M);
  PFE_HIP(hipMemcpyAsync(hd.data(), dots, hd.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  PFE_TRY(sync(h));
  mu->assign(K + 1, 0.0);
  for (int k = 0; k <= K; ++k) {
    double sm = 0;
    for (int l = 0; l < M; ++l) sm += hd[(size_t)k * M + l];
    (*mu)[k] = sm / M;
  }
  return pfe::ok();
}

pfe_status pfe_count_moments(pfe_handle h, int32_t K, int32_t nsamples, const double* V,
                             uint64_t seed, uint32_t flags, double* mu) {
  if (!h) return PFE_EINVAL;
  if (!mu) return finish(h, pfe::fail(PFE_EINVAL, "mu output required"));
  return guarded(h, [&] {
    std::vector<double> m;
    Err e = moments_impl(h, K, nsamples, V, seed, flags, &m);
    if (e.st == PFE_OK) std::copy(m.begin(), m.end(), mu);
    return e;
  });
}

// ---------------------------------------------------------------- slicing
// Spectrum slicing (end of Sec. 2.6; Sec. 6): [lam_lo, lam_hi] is cut where
// the moment-based count estimate reaches equal shares, every sub-window is
// solved by the filtered subspace iteration with a margin proportional to its
// width (degree by eq. thresh), and the results are merged.  Interior cuts get
// a guard g on both sides, so an eigenvalue near a cut is found by both
// neighbours; there the pairs are grouped by eigenvalue (gap > tau starts a
// new group) and each group is taken from the side that found more of it,
// which removes duplicates also for degenerate clusters.  A sub-window that
// overflows the block or does not converge is split in two.
static Err sliced_impl(pfe_handle h, double lam_lo, double lam_hi, int nev,
                       const pfe_solve_opts* o_in, const pfe_slice_opts* so_in, int* n_found,
                       double* evals, double* evecs, double* resid, int* n_slices_out,
                       double* cuts_out, int cuts_cap, pfe_solve_stats* st_out) {
  const auto t0 = std::chrono::steady_clock::now();
  PFE_TRY(select_device(h));
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  if (!h->has_bounds) return pfe::fail(PFE_ESTATE, "no spectral bounds (estimate_bounds or set_bounds)");
  pfe_solve_opts o;
  pfe_solve_opts_default(&o);
  if (o_in) o = *o_in;
  pfe_slice_opts so;
  std::memset(&so, 0, sizeof(so));
  so.count_seed = 13;
  if (so_in) so = *so_in;
  const int q = o.block;
  const int64_t n = h->n();
  if (q < 1 || q > 256 || q > n) return pfe::fail(PFE_EINVAL, "block must be in [1, min(256, n)]");
  if (nev < 0 || !n_found) return pfe::fail(PFE_EINVAL, "nev >= 0 and n_found required");
  if (!(lam_lo < lam_hi) || lam_lo < h->lam_lb || lam_hi > h->lam_ub)
    return pfe::fail(PFE_EINVAL, "window must satisfy lam_lb <= lam_lo < lam_hi <= lam_ub");
  if (so.n_slices < 0 || so.per_slice < 0 || so.margin < 0 || so.count_degree < 0 || so.count_samples < 0)
    return pfe::fail(PFE_EINVAL, "slice options must be >= 0");
  const double margin = so.margin > 0 ? so.margin : 1.0 / 6.0;
  const int per = so.per_slice > 0 ? so.per_slice : std::max(1, q / 2);
  const int K = so.count_degree > 0 ? so.count_degree : 1000;
  const int M = so.count_samples > 0 ? so.count_samples : 32;
  const double c = 0.5 * (h->lam_ub + h->lam_lb), e = 0.5 * (h->lam_ub - h->lam_lb);
  const double g = 1e-8 * h->lam_ub;
  const double tau = 1e-9 * h->lam_ub;
  // ---- cut points
  std::vector<double> mu;
  auto count_to = [&](double x) {
    const std::vector<double> chi =
        pfe::chi_coefficients((lam_lo - c) / e, (x - c) / e, K, PFE_SMOOTH_JACKSON);
    double acc = 0;
    for (int k = 0; k <= K; ++k) acc += chi[k] * mu[k];
    return (double)n * acc;
  };
  std::vector<double> bnd{lam_lo};
  if (so.cuts && so.n_slices > 1) {
    for (int i = 0; i < so.n_slices - 1; ++i) {
      const double x = so.cuts[i];
      if (!(x > bnd.back() && x < lam_hi)) return pfe::fail(PFE_EINVAL, "cuts must increase strictly inside the window");
      bnd.push_back(x);
    }
  } else if (so.n_slices != 1) {
    PFE_TRY(moments_impl(h, K, M, nullptr, so.count_seed, 0, &mu));
    const double total = count_to(lam_hi);
    int ns = so.n_slices > 0 ? so.n_slices : std::max(1, (int)std::ceil(total / per));
    ns = std::min(ns, 4096);
    if (ns > 1) {
      const int G = 4096;
      std::vector<double> xs(G + 1), Ns(G + 1);
      for (int i = 0; i <= G; ++i) {
        xs[i] = lam_lo + (lam_hi - lam_lo) * i / G;
        Ns[i] = i == 0 ? 0.0 : std::max(Ns[i - 1], count_to(xs[i]));
      }
      int gi = 1;
      for (int i = 1; i < ns; ++i) {
        const double target = Ns[G] * i / ns;
        while (gi < G && Ns[gi] < target) ++gi;
        const double f = (Ns[gi] > Ns[gi - 1]) ? (target - Ns[gi - 1]) / (Ns[gi] - Ns[gi - 1]) : 0.5;
        const double x = xs[gi - 1] + f * (xs[gi] - xs[gi - 1]);
        if (x > bnd.back() + 1e-6 * (lam_hi - lam_lo) && x < lam_hi - 1e-6 * (lam_hi - lam_lo))
          bnd.push_back(x);
      }
    }
  }
  bnd.push_back(lam_hi);
  // ---- slices, lowest first; a failed slice is replaced by its two halves
  std::vector<std::pair<double, double>> todo;
  for (size_t i = bnd.size() - 1; i >= 1; --i) todo.emplace_back(bnd[i - 1], bnd[i]);
  struct Pair {
    double th, res;
  };
  std::vector<Pair> kept;                  // ascending; vector i in slot i of VB
  const int cap = nev + q;
  PFE_HIP(h->wsSlice.ensure((size_t)cap * n * sizeof(double)));
  double* VB = h->wsSlice.as<double>();
  pfe_solve_stats agg;
  std::memset(&agg, 0, sizeof(agg));
  std::vector<double> used{lam_lo};
  int splits = 0, slice_no = 0;
  std::vector<double> ev(q), rs(q);
  while (!todo.empty()) {
    const double a = todo.back().first, b = todo.back().second;
    todo.pop_back();
    const bool first = a == lam_lo, last = b == lam_hi;
    const double wa = first ? a : std::max(h->lam_lb, a - g);
    const double wb = last ? b : std::min(h->lam_ub, b + g);
    pfe_solve_opts os = o;
    os.degree = 0;
    os.eps = margin * (wb - wa) / e;
    if (so.margin <= 0 && !mu.empty()) {
      // The filter's work for a slice scales with 1/eps whatever its rate r
      // (degree ~ log(1/r)/eps, iterations ~ log(tol)/log(r)), and Sec. 2.6
      // only asks the block to hold the eigenvalues of [xi - eps, eta + eps]:
      // take the widest margin (up to 1.5 widths) whose estimated count from
      // the moments stays within 85 % of the block.
      auto count_in = [&](double u, double v) {
        u = std::max(u, h->lam_lb);
        v = std::min(v, h->lam_ub);
        const std::vector<double> chi =
            pfe::chi_coefficients((u - c) / e, (v - c) / e, K, PFE_SMOOTH_JACKSON);
        double acc = 0;
        for (int k = 0; k <= K; ++k) acc += chi[k] * mu[k];
        return (double)n * acc;
      };
      const double w = wb - wa, cap_q = 0.85 * q;
      double mlo = margin, mhi = 1.5;
      if (count_in(wa - mlo * w, wb + mlo * w) <= cap_q) {
        if (count_in(wa - mhi * w, wb + mhi * w) <= cap_q) {
          mlo = mhi;
        } else {
          for (int it = 0; it < 24; ++it) {
            const double mm = 0.5 * (mlo + mhi);
            (count_in(wa - mm * w, wb + mm * w) <= cap_q ? mlo : mhi) = mm;
          }
        }
        os.eps = mlo * w / e;
      }
    }
    os.x0 = nullptr;
    // a sub-window of the FP32 form whose one refinement sweep falls short
    // would be split, which narrows it without helping the refinement: the
    // sub-solves may run further sweeps unless the caller set a number
    if (os.refine_sweeps <= 0) os.refine_sweeps = kSliceRefineSweeps;
    os.seed = o.seed + 7919ull * (uint64_t)slice_no;
    os.flags = PFE_DEVICE_PTRS;
    const int base = (int)kept.size();
    if (base + q > cap) {
      *n_found = base;
      return pfe::fail(PFE_ECAPACITY, "more eigenvalues in the window than nev");
    }
    int nf = 0;
    pfe_solve_stats ss;
    std::memset(&ss, 0, sizeof(ss));
    const Err r = solve_impl(h, wa, wb, q, &os, &nf, ev.data(), VB + (size_t)base * n, rs.data(), &ss);
    ++slice_no;
    agg.iterations += ss.iterations;
    agg.fp64_iterations += ss.fp64_iterations;
    agg.refined += ss.refined;
    agg.refine_applications += ss.refine_applications;
    agg.shifted_passes += ss.shifted_passes;
    agg.degree = std::max(agg.degree, ss.degree);
    agg.filter_steps += ss.filter_steps;
    agg.filter_bytes += ss.filter_bytes;
    agg.filter_columns += ss.filter_columns;
    agg.t_filter += ss.t_filter;
    agg.t_orth += ss.t_orth;
    agg.t_rr += ss.t_rr;
    agg.t_resid += ss.t_resid;
    agg.t_gemm += ss.t_gemm;
    agg.gemm_flops += ss.gemm_flops;
    agg.c = ss.c;
    agg.e = ss.e;
    if (r.st == PFE_ECAPACITY || r.st == PFE_ENOCONV) {
      // too many eigenvalues for the block, or no convergence: halve the
      // sub-window
      if (++splits > 64 || (b - a) < 1e-6 * (lam_hi - lam_lo))
        return pfe::fail(r.st, "sub-window [" + std::to_string(a) + ", " + std::to_string(b) +
                                   "] failed after splitting: " + r.msg);
      double mid = 0.5 * (a + b);
      if (!mu.empty()) {
        const double na = count_to(a), nb = count_to(b);
        if (nb - na > 1.0) {
          double lo2 = a, hi2 = b;
          for (int it = 0; it < 40; ++it) {
            const double m2 = 0.5 * (lo2 + hi2);
            (count_to(m2) < 0.5 * (na + nb) ? lo2 : hi2) = m2;
          }
          const double cand = 0.5 * (lo2 + hi2);
          if (cand > a + 0.05 * (b - a) && cand < b - 0.05 * (b - a)) mid = cand;
        }
      }
      todo.emplace_back(mid, b);
      todo.emplace_back(a, mid);
      continue;
    }
    if (r)
      return pfe::fail(r.st, "sub-window [" + std::to_string(a) + ", " + std::to_string(b) +
                                 "] (margin " + std::to_string(os.eps) + ", degree " +
                                 std::to_string(ss.degree) + "): " + r.msg);
    used.push_back(b);
    // merge the pairs near the cut a: old ones (end of `kept`) and new ones
    std::vector<int> order;          // final sequence of (negative: old slot, else new index)
    int zone0 = base;
    if (!first) {
      while (zone0 > 0 && kept[zone0 - 1].th >= a - g) --zone0;
    }
    struct Z {
      double th;
      int src;   // 0 old, 1 new
      int idx;
    };
    std::vector<Z> z;
    for (int i = zone0; i < base; ++i) z.push_back({kept[i].th, 0, i});
    int nz_new = 0;
    if (!first)
      while (nz_new < nf && ev[nz_new] <= a + g) ++nz_new;
    for (int i = 0; i < nz_new; ++i) z.push_back({ev[i], 1, i});
    std::stable_sort(z.begin(), z.end(), [](const Z& x, const Z& y) { return x.th < y.th; });
    std::vector<char> keep(z.size(), 1);
    for (size_t g0 = 0; g0 < z.size();) {
      size_t g1 = g0 + 1;
      while (g1 < z.size() && z[g1].th - z[g1 - 1].th <= tau) ++g1;
      int c0 = 0, c1 = 0;
      for (size_t i = g0; i < g1; ++i) (z[i].src ? c1 : c0)++;
      if (c0 > 0 && c1 > 0) {
        const int drop = (c1 > c0) ? 0 : 1;
        for (size_t i = g0; i < g1; ++i)
          if (z[i].src == drop) keep[i] = 0;
      }
      g0 = g1;
    }
    // new layout from slot zone0: kept zone entries in theta order, then the
    // remaining new pairs
    std::vector<std::pair<int, Pair>> seq;   // (source slot, pair)
    for (size_t i = 0; i < z.size(); ++i)
      if (keep[i]) {
        if (z[i].src == 0)
          seq.push_back({z[i].idx, kept[z[i].idx]});
        else
          seq.push_back({base + z[i].idx, Pair{ev[z[i].idx], rs[z[i].idx]}});
      }
    for (int i = nz_new; i < nf; ++i) seq.push_back({base + i, Pair{ev[i], rs[i]}});
    // sources are not in ascending slot order inside the zone (old and new
    // interleave by theta): stage through wsOut when any move is out of order
    bool monotone = true;
    for (size_t i = 1; i < seq.size(); ++i) monotone = monotone && seq[i].first > seq[i - 1].first;
    if (!monotone) {
      PFE_HIP(h->wsOut.ensure(seq.size() * (size_t)n * sizeof(double)));
      double* tmp = h->wsOut.as<double>();
      for (size_t i = 0; i < seq.size(); ++i)
        PFE_HIP(hipMemcpyAsync(tmp + i * (size_t)n, VB + (size_t)seq[i].first * n, n * sizeof(double),
                               hipMemcpyDeviceToDevice, h->stream));
      PFE_HIP(hipMemcpyAsync(VB + (size_t)zone0 * n, tmp, seq.size() * (size_t)n * sizeof(double),
                             hipMemcpyDeviceToDevice, h->stream));
    } else {
      for (size_t i = 0; i < seq.size(); ++i) {
        const int dst = zone0 + (int)i;
        if (dst != seq[i].first)
          PFE_HIP(hipMemcpyAsync(VB + (size_t)dst * n, VB + (size_t)seq[i].first * n,
                                 n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
      }
    }
    kept.resize(zone0);
    for (auto& sp : seq) kept.push_back(sp.second);
  }
  PFE_TRY(sync(h));
  const int total = (int)kept.size();
  agg.n_window = total;
  for (auto& kp : kept) agg.max_resid = std::max(agg.max_resid, kp.res);
  if (n_slices_out) *n_slices_out = (int)used.size() - 1;
  if (cuts_out && cuts_cap >= (int)used.size())
    std::copy(used.begin(), used.end(), cuts_out);
  agg.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st_out) *st_out = agg;
  *n_found = total;
  if (total > nev) return pfe::fail(PFE_ECAPACITY, "more eigenvalues in the window than nev");
  for (int i = 0; i < total; ++i) {
    if (evals) evals[i] = kept[i].th;
    if (resid) resid[i] = kept[i].res;
  }
  if (evecs && total > 0) {
    const bool dev_out = (o.flags & PFE_DEVICE_PTRS) != 0;
    PFE_HIP(hipMemcpyAsync(evecs, VB, (size_t)total * n * sizeof(double),
                           dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
    PFE_TRY(sync(h));
  }
  agg.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st_out) *st_out = agg;
  return pfe::ok();
}

pfe_status pfe_solve_sliced(pfe_handle h, double lam_lo, double lam_hi, int32_t nev,
                            const pfe_solve_opts* opts, const pfe_slice_opts* slice_opts,
                            int32_t* n_found, double* evals, double* evecs, double* resid,
                            int32_t* n_slices, double* cuts, int32_t cuts_cap,
                            pfe_solve_stats* stats) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return sliced_impl(h, lam_lo, lam_hi, nev, opts, slice_opts, n_found, evals, evecs,
                               resid, n_slices, cuts, cuts_cap, stats); });
}

// ------------------------------------------------------ thick-restart Lanczos
// Eigenpairs in [lam_lo, lam_hi] by block Lanczos with thick restart on the
// Dirac-delta filter rho_k(H_hat) (Sec. 2.5 and Sec. 3): the eigenvectors of
// rho_k(H_hat) with eigenvalue >= tau = rho_k(xi) = rho_k(eta) span the wanted
// eigenvectors of H, which a Rayleigh-Ritz step on H extracts.
//
// Basis V [n][ldv] of up to m + b columns.  Each expansion step filters the
// last block into the next b columns, keeps a copy, projects the new block
// against the basis twice and orthonormalises it (full re-orthogonalisation),
// and takes the new block column of T = V^T rho(H_hat) V from one Gram
// product with the kept copy, so T is computed, not assumed tridiagonal.  With m columns the Ritz pairs of T_m
// give residuals ||B s_last||; a thick restart keeps the k largest Ritz
// vectors (X <- V S_k), moves the residual block after them and restarts T as
// diag(theta) with the arrow coupling B S_last,k.
static Err lanczos_impl(pfe_handle h, double lam_lo, double lam_hi, int nev,
                        const pfe_lanczos_opts* o_in, int* n_found, double* evals, double* evecs,
                        double* resid, pfe_solve_stats* st_out) {
  const auto t0 = std::chrono::steady_clock::now();
  PFE_TRY(select_device(h));
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  if (!h->has_bounds) return pfe::fail(PFE_ESTATE, "no spectral bounds (estimate_bounds or set_bounds)");
  pfe_lanczos_opts o;
  pfe_lanczos_opts_default(&o);
  if (o_in) o = *o_in;
  const int64_t n = h->n();
  const int b = o.block;
  if (b < 1 || b > 64) return pfe::fail(PFE_EINVAL, "block must be in [1, 64]");
  if (nev < 0 || !n_found) return pfe::fail(PFE_EINVAL, "nev >= 0 and n_found required");
  const int64_t m_req = o.max_basis > 0 ? (int64_t)o.max_basis : std::max<int64_t>(4 * b, 3 * (int64_t)std::max(nev, 1));
  pfe::LanczosShape shp;
  if (m_req > 511 || pfe::lanczos_shape((int)round_up(m_req, b), b, &shp) != 0)
    return pfe::fail(PFE_EINVAL, "max_basis must give 3 block <= m and m + block <= 511");
  const int m = shp.m;
  if (m + b > n) return pfe::fail(PFE_EINVAL, "basis larger than the matrix");
  if (lam_lo < h->lam_lb || lam_hi > h->lam_ub)
    return pfe::fail(PFE_EINVAL, "window must lie inside [lam_lb, lam_ub]");
  const double tol = o.tol > 0 ? o.tol : 1e-10;
  const int max_restarts = o.max_restarts > 0 ? o.max_restarts : 200;
  pfe::DiracDesign dd;
  PFE_TRY(pfe::design_dirac(lam_lo, lam_hi, h->lam_lb, h->lam_ub, o.degree, o.phi > 0 ? o.phi : 0.8,
                            o.smoothing, &dd));
  pfe_solve_stats st;
  std::memset(&st, 0, sizeof(st));
  st.degree = dd.degree;
  st.c = dd.c;
  st.e = dd.e;
  st.xi = dd.xi;
  st.eta = dd.eta;
  const int64_t ldv = round_up(m + b, 8);
  const size_t mvb = (size_t)n * ldv * sizeof(double);
  PFE_HIP(h->wsA.ensure(mvb));                                   // V
  PFE_HIP(h->wsB.ensure(mvb));                                   // filter scratch / Ritz vectors
  PFE_HIP(h->wsC.ensure(mvb));                                   // H X in the extraction
  PFE_HIP(h->wsD.ensure((size_t)n * round_up(b, 8) * sizeof(double)));   // kept rho(H) V_j
  double* V = h->wsA.as<double>();
  double* Scr = h->wsB.as<double>();
  double* Wx = h->wsC.as<double>();
  double* Wk = h->wsD.as<double>();
  const int64_t ldk = round_up(b, 8);
  PFE_HIP(pfe::zero_f64(V, n * ldv, h->stream));
  PFE_HIP(pfe::zero_f64(Scr, n * ldv, h->stream));
  PFE_HIP(pfe::zero_f64(Wk, n * ldk, h->stream));
  Small sm;
  PFE_TRY(alloc_small(h, m + b, &sm));
  PFE_TRY(ensure_red(h, n, m + b));
  // Orthonormalise block B (b columns at ld ldv) against V[:, 0:p] (two
  // projection passes, classical Gram-Schmidt) and in itself (CholQR2).  A
  // block that has (numerically) no part outside span(V) is replaced by
  // random directions, projected the same way: the Krylov space has then
  // closed over those directions, and T stays exact because it is formed
  // from the kept filtered block.
  int refills = 0;
  auto project = [&](double* B, int p0) -> Err {
    for (int pass = 0; pass < 2 && p0 > 0; ++pass) {
      PFE_HIP(pfe::gram_f64(n, p0, b, V, ldv, B, ldv, sm.G, h->wsRed.p, h->stream));
      PFE_HIP(pfe::gemm_tall_f64(n, p0, b, V, ldv, sm.G, Scr, ldv, h->stream));
      PFE_HIP(pfe::sub_cols_f64(n, b, Scr, ldv, B, ldv, h->stream));
    }
    return pfe::ok();
  };
  auto orth_block = [&](double* Vb, int p0, double* B) -> Err {
    (void)Vb;
    PFE_TRY(project(B, p0));
    Err e = cholqr2(h, sm, B, n, b, ldv, -1.0);
    for (int tries = 0; e.st == PFE_EBREAKDOWN && tries < 3; ++tries) {
      ++refills;
      PFE_HIP(pfe::gaussian_fill_f64(n, b, B, ldv, o.seed + 1000003ull * (uint64_t)(refills + 1), h->stream));
      PFE_TRY(project(B, p0));
      e = cholqr2(h, sm, B, n, b, ldv, -1.0);
    }
    return e;
  };
  PFE_HIP(pfe::gaussian_fill_f64(n, b, V, ldv, o.seed, h->stream));
  {
    Timer tm(h, &st.t_orth);
    PFE_TRY(orth_block(V, 0, V));
  }
  const int M1 = shp.M1;
  std::vector<double> T((size_t)M1 * M1, 0.0), Cf((size_t)M1 * b), th(m), Q((size_t)m * m);
  std::vector<double> Tm((size_t)m * m), rA(m), Mh;
  // host matrices copied into sm.Rinv (2 (m + b)^2 doubles)
  const size_t rinv_cap = 2 * (size_t)M1 * M1;
  int p = b;                       // columns [p - b, p) still need their filtered image
  double epsA = 0.1 * tol;         // A-residual target relative to rho(gamma)
  int prev_nw = -1, cycles = 0, tightened = 0;
  const double delta = 1e-6 * h->lam_ub;
  std::vector<double> theta, res;
  bool done = false;
  int ns_final = 0;
  std::vector<int> sel;
  while (!done) {
    // ---- expansion to m columns plus the residual block
    while (p < m + b) {
      if (p % b != 0 || p + b > M1)
        return pfe::fail(PFE_EHIP, "internal: Lanczos block outside the basis");
      {
        Timer tm(h, &st.t_filter);
        PFE_TRY(run_filter<double>(h, h->step_vals64(), dd.coef, 1.0 / dd.e, -dd.c / dd.e,
                                   V + (p - b), V + p, Scr, b, ldv, &st.filter_steps));
      }
      st.filter_columns += b;
      PFE_HIP(pfe::copy_cols_f64(n, b, V + p, ldv, Wk, ldk, h->stream));
      {
        Timer tm(h, &st.t_orth);
        PFE_TRY(orth_block(V, p, V + p));
        PFE_HIP(pfe::gram_f64(n, p + b, b, V, ldv, Wk, ldk, sm.G, h->wsRed.p, h->stream));
        PFE_HIP(hipMemcpyAsync(Cf.data(), sm.G, (size_t)(p + b) * b * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
        PFE_TRY(sync(h));
      }
      if (pfe::lanczos_store_block(shp, p, Cf, T) != 0)
        return pfe::fail(PFE_EHIP, "internal: Lanczos Gram block outside T");
      p += b;
    }
    // ---- Ritz pairs of T_m (device Jacobi)
    if (pfe::lanczos_leading(shp, T, Tm) != 0) return pfe::fail(PFE_EHIP, "internal: Lanczos T shape");
    int info = 0;
    {
      Timer tm(h, &st.t_rr);
      PFE_HIP(hipMemcpyAsync(sm.S, Tm.data(), Tm.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
      PFE_HIP(pfe::sym_eig_f64(m, sm.S, sm.theta, sm.Q, sm.jw, sm.info, h->stream));
      PFE_HIP(hipMemcpyAsync(th.data(), sm.theta, m * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      PFE_HIP(hipMemcpyAsync(Q.data(), sm.Q, Q.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      PFE_HIP(hipMemcpyAsync(&info, sm.info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
      PFE_TRY(sync(h));
    }
    if (info < 0) return pfe::fail(PFE_EHIP, "Jacobi eigensolver did not converge");
    ++cycles;
    st.iterations = cycles;
    // residual norms ||B s_i||, B = T[m:m+b, m-b:m]
    if (pfe::lanczos_ritz_residuals(shp, T, Q, rA) != 0)
      return pfe::fail(PFE_EHIP, "internal: Lanczos residual shape");
    // wanted: theta >= tau, largest first (theta ascending from Jacobi)
    std::vector<int> want;
    for (int i = m - 1; i >= 0; --i)
      if (th[i] >= dd.tau) want.push_back(i);
    const int nw = (int)want.size();
    const int k = pfe::lanczos_keep(shp, nw);
    if (k < 0) {
      *n_found = nw;
      return pfe::fail(PFE_ECAPACITY, "max_basis too small for the eigenvalues above tau");
    }
    bool conv = true;
    for (int i : want) conv = conv && rA[i] <= epsA * dd.peak;
    const char* tr_env = std::getenv("PFEIG_TRACE");
    if (tr_env && tr_env[0] && tr_env[0] != '0') {
      double mx = 0;
      for (int i : want) mx = std::max(mx, rA[i] / dd.peak);
      std::fprintf(stderr, "[pfeig] lanczos cycle %d wanted %d max rel A-resid %.3e\n", cycles, nw, mx);
    }
    if (conv && nw == prev_nw && cycles >= 2) {
      // ---- extraction: Rayleigh-Ritz on H over the wanted Ritz vectors
      if (nw == 0) {
        theta.clear();
        res.clear();
        done = true;
        break;
      }
      if (pfe::lanczos_select_columns(shp, Q, want, Mh) != 0 || Mh.size() > rinv_cap)
        return pfe::fail(PFE_EHIP, "internal: Lanczos wanted columns");
      PFE_HIP(hipMemcpyAsync(sm.Rinv, Mh.data(), Mh.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
      PFE_TRY(sync(h));
      PFE_HIP(pfe::gemm_tall_f64(n, m, nw, V, ldv, sm.Rinv, Scr, ldv, h->stream));
      {
        Timer tm(h, &st.t_orth);
        PFE_TRY(cholqr2(h, sm, Scr, n, nw, ldv, -1.0));
      }
      PFE_TRY(rayleigh_ritz(h, sm, Scr, Wx, n, nw, ldv, theta, res, &st.t_rr, &st.t_resid));
      bool ok = true;
      for (int j = 0; j < nw; ++j)
        if (theta[j] >= lam_lo - delta && theta[j] <= lam_hi + delta) ok = ok && res[j] <= tol;
      if (ok) {
        done = true;
        break;
      }
      if (++tightened > 4) return pfe::fail(PFE_ENOCONV, "H residuals above tol after tightening");
      epsA *= 0.01;
    }
    prev_nw = nw;
    if (cycles >= max_restarts) return pfe::fail(PFE_ENOCONV, "not converged within max_restarts");
    // ---- thick restart: keep the k largest Ritz vectors, k a multiple of b
    // so that the expansion fills the basis exactly up to m + b columns
    std::vector<int> keep(k);
    for (int c = 0; c < k; ++c) keep[c] = m - 1 - c;
    if (pfe::lanczos_select_columns(shp, Q, keep, Mh) != 0 || Mh.size() > rinv_cap)
      return pfe::fail(PFE_EHIP, "internal: Lanczos kept columns");
    PFE_HIP(hipMemcpyAsync(sm.Rinv, Mh.data(), Mh.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    PFE_HIP(pfe::gemm_tall_f64(n, m, k, V, ldv, sm.Rinv, V, ldv, h->stream));
    PFE_HIP(pfe::copy_cols_f64(n, b, V + m, ldv, V + k, ldv, h->stream));
    PFE_TRY(sync(h));
    if (pfe::lanczos_restart(shp, k, th, Q, T) != 0)
      return pfe::fail(PFE_EHIP, "internal: Lanczos restart shape");
    p = k + b;
  }
  // ---- selection and output (theta ascending)
  sel.clear();
  int total_in = 0;
  for (size_t j = 0; j < theta.size(); ++j)
    if (theta[j] >= lam_lo && theta[j] <= lam_hi) {
      ++total_in;
      sel.push_back((int)j);
    }
  st.n_window = total_in;
  st.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st_out) *st_out = st;
  if (total_in > nev) {
    *n_found = total_in;
    return pfe::fail(PFE_ECAPACITY, "more eigenvalues in the window than nev");
  }
  ns_final = (int)sel.size();
  *n_found = ns_final;
  double maxr = 0;
  for (int s2 = 0; s2 < ns_final; ++s2) {
    if (evals) evals[s2] = theta[sel[s2]];
    if (resid) resid[s2] = res[sel[s2]];
    maxr = std::max(maxr, res[sel[s2]]);
  }
  if (evecs && ns_final > 0) {
    PFE_HIP(hipMemcpyAsync(sm.sel, sel.data(), ns_final * sizeof(int), hipMemcpyHostToDevice, h->stream));
    const bool dev_out = (o.flags & PFE_DEVICE_PTRS) != 0;
    double* dst = evecs;
    if (!dev_out) {
      PFE_HIP(h->wsOut.ensure((size_t)ns_final * n * sizeof(double)));
      dst = h->wsOut.as<double>();
    }
    PFE_HIP(pfe::gather_transpose_signfix(n, ns_final, Scr, ldv, sm.sel, dst, h->wsRed.p, h->stream));
    if (!dev_out)
      PFE_HIP(hipMemcpyAsync(evecs, dst, (size_t)ns_final * n * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    PFE_TRY(sync(h));
  }
  st.max_resid = maxr;
  st.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st_out) *st_out = st;
  return pfe::ok();
}

void pfe_lanczos_opts_default(pfe_lanczos_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->block = 16;
  o->phi = 0.8;
  o->smoothing = PFE_SMOOTH_NONE;
  o->max_restarts = 200;
  o->seed = 11;
}

pfe_status pfe_solve_lanczos(pfe_handle h, double lam_lo, double lam_hi, int32_t nev,
                             const pfe_lanczos_opts* opts, int32_t* n_found, double* evals,
                             double* evecs, double* resid, pfe_solve_stats* stats) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return lanczos_impl(h, lam_lo, lam_hi, nev, opts, n_found, evals, evecs, resid, stats); });
}

pfe_status pfe_locality_order(int64_t n_atoms, int64_t nnzb, const int64_t* row_ptr,
                              const int32_t* col_idx, int32_t leaf, int32_t group, int64_t window,
                              int32_t* order, double* far_in, double* far_out) {
  return host_guarded([&]() -> pfe_status {
    if (n_atoms <= 0 || n_atoms > (int64_t)INT32_MAX || nnzb < 0 || !row_ptr || !col_idx ||
        !order || group < 1 || group > 4 || leaf < 2 * group || window < 0)
      return PFE_EINVAL;
    if (row_ptr[0] != 0 || row_ptr[n_atoms] != nnzb) return PFE_EINVAL;
    for (int64_t i = 0; i < n_atoms; ++i)
      if (row_ptr[i + 1] < row_ptr[i]) return PFE_EINVAL;
    for (int64_t k = 0; k < nnzb; ++k)
      if (col_idx[k] < 0 || col_idx[k] >= n_atoms) return PFE_EINVAL;
    std::vector<int32_t> ord;
    pfe::locality_order(n_atoms, row_ptr, col_idx, leaf, group, ord);
    std::memcpy(order, ord.data(), (size_t)n_atoms * sizeof(int32_t));
    if (far_in) *far_in = pfe::far_block_fraction(n_atoms, row_ptr, col_idx, nullptr, window);
    if (far_out) *far_out = pfe::far_block_fraction(n_atoms, row_ptr, col_idx, ord.data(), window);
    return PFE_OK;
  });
}

pfe_status pfe_design_dirac(double lam_lo, double lam_hi, double lam_lb, double lam_ub,
                            int32_t degree, double phi, int32_t smoothing, double* coef_out,
                            int32_t coef_cap, pfe_dirac_filter* out) {
  return host_guarded([&]() -> pfe_status {
    if (!out) return PFE_EINVAL;
    pfe::DiracDesign dd;
    const Err e = pfe::design_dirac(lam_lo, lam_hi, lam_lb, lam_ub, degree, phi, smoothing, &dd);
    if (e) return e.st;
    out->degree = dd.degree;
    out->smoothing = dd.smoothing;
    out->c = dd.c;
    out->e = dd.e;
    out->xi = dd.xi;
    out->eta = dd.eta;
    out->gamma = dd.gamma;
    out->tau = dd.tau;
    out->peak = dd.peak;
    out->coef = coef_out;
    if (!coef_out || coef_cap < dd.degree + 1) return PFE_ECAPACITY;
    std::copy(dd.coef.begin(), dd.coef.end(), coef_out);
    return PFE_OK;
  });
}

// ---------------------------------------------------------------- adjoint
static Err adjoint_impl(pfe_handle h, const pfe_filter* f, int nvec, const double* X,
                        const double* dY, double* dX, double* dblocks, int64_t ld, int stride,
                        uint32_t flags) {
  PFE_TRY(select_device(h));
  PFE_TRY(check_filter(h, f));
  if (nvec < 1 || nvec > 256 || ld < nvec || !X || !dY || !dX || !dblocks)
    return pfe::fail(PFE_EINVAL, "need 1 <= nvec <= 256, nvec <= ld and non-null arrays");
  const bool dev = (flags & PFE_DEVICE_PTRS) != 0;
  const int64_t n = h->n();
  const int d = f->degree;
  const double c = f->c, e = f->e;
  const int s = stride > 0 ? stride : std::max(1, (int)std::ceil(std::sqrt((double)std::max(d, 1))));
  const int nseg = d > 0 ? (d + s - 1) / s : 0;
  const size_t mv = (size_t)n * ld * sizeof(double);
  const int64_t nel = n * ld;
  // Default: the sweep keeps a checkpoint pair (t_k, t_{k+1}) at the start
  // of every segment of s steps and regenerates the segment's forward
  // vectors from it on the way back (2 ceil(d/s) + 2 s + 2 vectors).
  // PFE_ADJOINT_RESIDENT (stride left to the library): the whole forward
  // trajectory (t_k for k < d) stays on the device instead when it fits in
  // half the free memory: no checkpoint copies and no recomputation.  The
  // adjoint recurrence does not depend on the forward one (only the block
  // gradient joins them) and both steps share alpha, beta and delta: when
  // both trajectories fit, slot k of one buffer holds [t_k | a_{d-k+1}]
  // side by side (2 ld columns) and one fused step advances both, the added
  // stream being [0 | Ybar].  Segments keep length s for the block gradient
  // and every element sees the same arithmetic, so all three give identical
  // bits.  A resident workspace that cannot be allocated falls back to
  // checkpoints.
  bool keep = false, pair = false;
  if ((flags & PFE_ADJOINT_RESIDENT) && stride <= 0 && d >= 2) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
      pair = nvec == ld && 2 * mv * (size_t)(d + 2) <= fr / 2 + h->wsCk.bytes;
      keep = pair || mv * (size_t)d <= fr / 2 + h->wsCk.bytes;
    }
  }
  // device: X, Ybar and either the paired slots, or the adjoint vectors of
  // one segment with the forward trajectory or with a segment buffer (s
  // vectors) and checkpoints (2 per segment)
  PFE_HIP(h->wsA.ensure(mv * 2));                 // X, Ybar (device copies when host inputs)
  PFE_HIP(h->wsSmall.ensure((size_t)std::max(d, 1) * sizeof(double) + 64));
  if (pair) {
    if (h->wsCk.ensure(2 * mv * (size_t)(d + 1)) != hipSuccess ||   // slots 0 .. d
        h->wsC.ensure(2 * mv) != hipSuccess) {                      // [0 | Ybar]
      (void)hipGetLastError();   // clear the failed allocation's error
      h->wsCk.release();
      pair = false;
    }
  }
  if (!pair && keep) {
    if (h->wsCk.ensure(mv * (size_t)d) != hipSuccess) {
      (void)hipGetLastError();
      h->wsCk.release();
      keep = false;
    }
  }
  if (!pair) PFE_HIP(h->wsB.ensure(mv * (size_t)(s + 2)));   // adjoint vectors of one segment
  if (!pair && !keep) {
    PFE_HIP(h->wsC.ensure(mv * (size_t)std::max(s, 1)));
    PFE_HIP(h->wsCk.ensure(mv * (size_t)std::max(2 * nseg, 1)));
  }
  PFE_HIP(h->wsD.ensure((size_t)(h->nnzb + 1) * 9 * sizeof(double)));
  const double* Xd = X;
  const double* Yb = dY;
  if (!dev) {
    PFE_HIP(hipMemcpyAsync(h->wsA.p, X, mv, hipMemcpyHostToDevice, h->stream));
    PFE_HIP(hipMemcpyAsync(h->wsA.as<double>() + nel, dY, mv, hipMemcpyHostToDevice, h->stream));
    Xd = h->wsA.as<double>();
    Yb = h->wsA.as<double>() + nel;
  }
  double* aA = h->wsB.as<double>();
  double* seg = h->wsC.as<double>();
  double* ck = h->wsCk.as<double>();
  double* G = h->wsD.as<double>();
  const pfe::Bsr A = h->bsr();
  const double* Hs = h->step_vals64();       // as the fused step reads it
  PFE_HIP(pfe::zero_f64(G, h->nnzb * 9, h->stream));
  const double a1 = 1.0 / e, b1 = -c / e, a2 = 2.0 / e, b2 = -2.0 * c / e;
  auto fwd = [&](const double* tin, const double* prev, double* out, bool first) -> hipError_t {
    return pfe::cheb_step_f64(A, Hs, tin, prev, nullptr, out, nvec, ld, first ? a1 : a2,
                              first ? b1 : b2, first ? 0.0 : -1.0, 0.0, h->stream);
  };
  if (pair) {
    const int64_t ld2 = 2 * ld, nel2 = 2 * nel;
    double* Z = h->wsCk.as<double>();      // slot k at Z + k nel2: [t_k | a_{d-k+1}]
    double* Yc = h->wsC.as<double>();      // [0 | Ybar]
    auto slot = [&](int k) { return Z + (size_t)k * nel2; };
    PFE_HIP(pfe::zero_f64(Yc, nel2, h->stream));
    PFE_HIP(pfe::copy_cols_f64(n, (int)ld, Yb, ld, Yc + ld, ld2, h->stream));
    PFE_HIP(pfe::zero_f64(slot(0), nel2, h->stream));                     // a_{d+1} = 0
    PFE_HIP(pfe::copy_cols_f64(n, (int)ld, Xd, ld, slot(0), ld2, h->stream));   // t_0 = X
    // t_1 = H_hat X;  a_d = g_d Ybar (no matrix term)
    PFE_HIP(pfe::cheb_step_f64(A, Hs, slot(0), nullptr, nullptr, slot(1), nvec, ld2, a1, b1, 0.0,
                               0.0, h->stream));
    PFE_HIP(pfe::cheb_step_f64(A, Hs, Yc + ld, nullptr, Yc + ld, slot(1) + ld, nvec, ld2, 0.0, 0.0,
                               0.0, f->coef[d], h->stream));
    // t_{s+1} = 2 H_hat t_s - t_{s-1} beside a_{d-s} = g_{d-s} Ybar + 2 H_hat a_{d-s+1} - a_{d-s+2}
    for (int st = 1; st <= d - 1; ++st)
      PFE_HIP(pfe::cheb_step_f64(A, Hs, slot(st), slot(st - 1), Yc, slot(st + 1), (int)ld2, ld2, a2,
                                 b2, -1.0, f->coef[d - st], h->stream));
    // a_0 = g_0 Ybar + H_hat a_1 - a_2, into the spent a_{d+1}
    PFE_HIP(pfe::cheb_step_f64(A, Hs, slot(d) + ld, slot(d - 1) + ld, Yc + ld, slot(0) + ld, nvec,
                               ld2, a1, b1, -1.0, f->coef[0], h->stream));
    double* wdv = h->wsSmall.as<double>();
    std::vector<double> wv((size_t)d, 2.0);
    wv[0] = 1.0;
    PFE_HIP(hipMemcpyAsync(wdv, wv.data(), d * sizeof(double), hipMemcpyHostToDevice, h->stream));
    // block gradient by segments, last first: t_k in slot k, a_{k+1} in slot d - k
    for (int j = nseg - 1; j >= 0; --j) {
      const int k0 = j * s, w1 = std::min(k0 + s, d) - k0;
      PFE_HIP(pfe::sddmm_seg_f64(A, nvec, w1, slot(d - k0) + ld, -nel2, slot(k0), nel2, ld2,
                                 wdv + k0, G, h->stream));
    }
    PFE_HIP(pfe::scale_f64(h->nnzb * 9, 1.0 / e, G, h->stream));
    if (dev) {
      PFE_HIP(pfe::copy_cols_f64(n, (int)ld, slot(0) + ld, ld2, dX, ld, h->stream));
      PFE_HIP(hipMemcpyAsync(dblocks, G, h->nnzb * 9 * sizeof(double), hipMemcpyDeviceToDevice,
                             h->stream));
    } else {
      double* a0 = h->wsA.as<double>();   // X's copy is spent
      PFE_HIP(pfe::copy_cols_f64(n, (int)ld, slot(0) + ld, ld2, a0, ld, h->stream));
      PFE_HIP(hipMemcpyAsync(dX, a0, mv, hipMemcpyDeviceToHost, h->stream));
      PFE_HIP(hipMemcpyAsync(dblocks, G, h->nnzb * 9 * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    }
    PFE_TRY(sync(h));
    return pfe::ok();
  }
  double* traj = h->wsCk.as<double>();   // trajectory: t_k in slot k
  if (keep) {
    PFE_HIP(pfe::copy_cols_f64(n, (int)ld, Xd, ld, traj, ld, h->stream));
    PFE_HIP(fwd(traj, nullptr, traj + nel, true));   // t_1
    for (int k = 1; k <= d - 2; ++k)
      PFE_HIP(fwd(traj + (size_t)k * nel, traj + (size_t)(k - 1) * nel, traj + (size_t)(k + 1) * nel,
                  false));
  } else if (d >= 1) {
    // forward sweep storing (t_{js}, t_{js+1}) for every segment j
    double* t_prev = seg;                         // rolling pair in seg[0], seg[1] (s >= 1)
    double* t_cur = (s >= 2) ? seg + nel : aA;
    PFE_HIP(pfe::copy_cols_f64(n, (int)ld, Xd, ld, t_prev, ld, h->stream));
    PFE_HIP(fwd(Xd, nullptr, t_cur, true));       // t_1
    for (int k = 1; k <= d - 1; ++k) {
      // invariant: t_prev = t_{k-1}, t_cur = t_k
      if ((k - 1) % s == 0) {
        const int j = (k - 1) / s;
        PFE_HIP(pfe::copy_cols_f64(n, (int)ld, t_prev, ld, ck + (2 * j) * nel, ld, h->stream));
        PFE_HIP(pfe::copy_cols_f64(n, (int)ld, t_cur, ld, ck + (2 * j + 1) * nel, ld, h->stream));
      }
      PFE_HIP(fwd(t_cur, t_prev, t_prev, false));  // t_{k+1} over t_{k-1}
      std::swap(t_prev, t_cur);
    }
    if ((d - 1) % s == 0) {   // last segment starts at d-1 (only t_{d-1} is needed)
      const int j = (d - 1) / s;
      PFE_HIP(pfe::copy_cols_f64(n, (int)ld, t_prev, ld, ck + (2 * j) * nel, ld, h->stream));
      PFE_HIP(pfe::copy_cols_f64(n, (int)ld, t_cur, ld, ck + (2 * j + 1) * nel, ld, h->stream));
    }
  }
  // reverse sweep: a_d = g_d Ybar; a_k = g_k Ybar + 2 A a_{k+1} - a_{k+2};
  // a_0 = g_0 Ybar + A a_1 - a_2; G += w_k a_{k+1} t_k^T (w_0 = 1, else 2).
  // One checkpoint segment at a time: slot i of segA holds a_{k0+i} for
  // i = 0 .. k1-k0+1, the steps run on the fused filter kernel (the adjoint
  // recurrence is the forward one with Ybar as the added stream, since H_hat
  // is symmetric), and the segment's block gradient is one batched SDDMM.
  double* segA = aA;
  // gradient weights w_k (1 for k = 0, else 2), uploaded once: the host
  // vector outlives every copy that reads it
  double* wdev = h->wsSmall.as<double>();
  std::vector<double> wv((size_t)std::max(d, 1), 2.0);
  wv[0] = 1.0;
  if (d >= 1)
    PFE_HIP(hipMemcpyAsync(wdev, wv.data(), d * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if (d == 0) {
    PFE_HIP(pfe::copy_cols_f64(n, (int)ld, Yb, ld, segA, ld, h->stream));
    PFE_HIP(pfe::scale_f64(nel, f->coef[0], segA, h->stream));
  }
  for (int j = nseg - 1; j >= 0; --j) {
    const int k0 = j * s;
    const int k1 = std::min(k0 + s, d);          // segment covers t_k, k0 <= k < k1
    const int w1 = k1 - k0;
    if (j == nseg - 1) {                          // a_{d+1} = 0, a_d = g_d Ybar
      PFE_HIP(pfe::zero_f64(segA + (size_t)(w1 + 1) * nel, nel, h->stream));
      PFE_HIP(pfe::copy_cols_f64(n, (int)ld, Yb, ld, segA + (size_t)w1 * nel, ld, h->stream));
      PFE_HIP(pfe::scale_f64(nel, f->coef[d], segA + (size_t)w1 * nel, h->stream));
    } else {                                      // a_{k1}, a_{k1+1} from the segment above
      PFE_HIP(pfe::copy_cols_f64(n, (int)ld, segA + nel, ld, segA + (size_t)(w1 + 1) * nel, ld, h->stream));
      PFE_HIP(pfe::copy_cols_f64(n, (int)ld, segA, ld, segA + (size_t)w1 * nel, ld, h->stream));
    }
    // t_{k0} .. t_{k1-1}: in the trajectory, or regenerated into seg[0 .. k1-k0-1]
    const double* segT = keep ? traj + (size_t)k0 * nel : seg;
    if (!keep) {
      PFE_HIP(pfe::copy_cols_f64(n, (int)ld, ck + (2 * j) * nel, ld, seg, ld, h->stream));
      if (w1 >= 2)
        PFE_HIP(pfe::copy_cols_f64(n, (int)ld, ck + (2 * j + 1) * nel, ld, seg + nel, ld, h->stream));
      for (int k = k0 + 2; k < k1; ++k)
        PFE_HIP(pfe::cheb_step_f64(A, Hs, seg + (k - 1 - k0) * nel, seg + (k - 2 - k0) * nel,
                                   nullptr, seg + (k - k0) * nel, nvec, ld, a2, b2, -1.0, 0.0,
                                   h->stream));
    }
    for (int k = k1 - 1; k >= k0; --k) {
      const bool last = (k == 0);
      PFE_HIP(pfe::cheb_step_f64(A, Hs, segA + (size_t)(k + 1 - k0) * nel,
                                 segA + (size_t)(k + 2 - k0) * nel, Yb, segA + (size_t)(k - k0) * nel,
                                 nvec, ld, last ? a1 : a2, last ? b1 : b2, -1.0, f->coef[k],
                                 h->stream));
    }
    PFE_HIP(pfe::sddmm_seg_f64(A, nvec, w1, segA + nel, nel, segT, nel, ld, wdev + k0, G, h->stream));
  }
  double* a_mid = segA;   // a_0 (or g_0 Ybar when d == 0)
  PFE_HIP(pfe::scale_f64(h->nnzb * 9, 1.0 / e, G, h->stream));
  if (dev) {
    PFE_HIP(pfe::copy_cols_f64(n, (int)ld, a_mid, ld, dX, ld, h->stream));
    PFE_HIP(hipMemcpyAsync(dblocks, G, h->nnzb * 9 * sizeof(double), hipMemcpyDeviceToDevice,
                           h->stream));
  } else {
    PFE_HIP(hipMemcpyAsync(dX, a_mid, mv, hipMemcpyDeviceToHost, h->stream));
    PFE_HIP(hipMemcpyAsync(dblocks, G, h->nnzb * 9 * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
  }
  PFE_TRY(sync(h));
  return pfe::ok();
}

pfe_status pfe_apply_filter_adjoint(pfe_handle h, const pfe_filter* f, int32_t nvec,
                                    const double* X, const double* dY, double* dX,
                                    double* dblocks, int64_t ld, int32_t ckpt_stride,
                                    uint32_t flags) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return adjoint_impl(h, f, nvec, X, dY, dX, dblocks, ld, ckpt_stride, flags); });
}

// ----------------------------------------------------- gradient helpers
static Err eigvec_grad_impl(pfe_handle h, int nvec, const double* V, const double* w,
                            double* dblocks, uint32_t flags) {
  PFE_TRY(select_device(h));
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  if (nvec < 1 || nvec > 256 || !V || !dblocks) return pfe::fail(PFE_EINVAL, "1 <= nvec <= 256");
  const bool dev = (flags & PFE_DEVICE_PTRS) != 0;
  const int64_t n = h->n();
  const int64_t ld = round_up(nvec, 8);
  PFE_HIP(h->wsA.ensure((size_t)n * nvec * sizeof(double)));
  PFE_HIP(h->wsB.ensure((size_t)n * ld * sizeof(double)));
  PFE_HIP(h->wsD.ensure((size_t)(h->nnzb + 1) * 9 * sizeof(double)));
  PFE_HIP(h->wsSmall.ensure((size_t)nvec * sizeof(double) + 64));
  const double* Vd = V;
  if (!dev) {
    PFE_HIP(hipMemcpyAsync(h->wsA.p, V, (size_t)n * nvec * sizeof(double), hipMemcpyHostToDevice,
                           h->stream));
    Vd = h->wsA.as<double>();
  }
  double* Vr = h->wsB.as<double>();
  PFE_HIP(pfe::zero_f64(Vr, n * ld, h->stream));
  PFE_HIP(pfe::transpose_to_rows(nvec, n, Vd, Vr, ld, h->stream));
  const double* wd = nullptr;
  if (w) {
    PFE_TRY(upload(h, h->wsSmall.as<double>(), w, nvec, dev));
    wd = h->wsSmall.as<double>();
  }
  double* G = dev ? dblocks : h->wsD.as<double>();
  PFE_HIP(pfe::sddmm_f64(h->bsr(), nvec, Vr, Vr, ld, wd, G, false, h->stream));
  if (!dev)
    PFE_HIP(hipMemcpyAsync(dblocks, G, h->nnzb * 9 * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
  PFE_TRY(sync(h));
  return pfe::ok();
}

pfe_status pfe_eigvec_block_gradient(pfe_handle h, int32_t nvec, const double* V, const double* w,
                                     double* dblocks, uint32_t flags) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return eigvec_grad_impl(h, nvec, V, w, dblocks, flags); });
}

static Err spring_grad_impl(pfe_handle h, int64_t P, const int64_t* pairs, const double* unit,
                            const double* dblocks, double* dk, double* dm, uint32_t flags) {
  PFE_TRY(select_device(h));
  if (!h->has_h) return pfe::fail(PFE_ESTATE, "no Hessian set");
  if (!h->has_masses) return pfe::fail(PFE_ESTATE, "masses were not given to set_hessian");
  if (P < 0 || (P > 0 && (!pairs || !unit || !dk)) || !dblocks || !dm)
    return pfe::fail(PFE_EINVAL, "arrays");
  const bool dev = (flags & PFE_DEVICE_PTRS) != 0;
  const int64_t N = h->n_atoms;
  // host pairs are checked here; device pairs by the kernel's block lookup
  if (!dev)
    for (int64_t p = 0; p < P; ++p)
      if (pairs[2 * p] < 0 || pairs[2 * p] >= N || pairs[2 * p + 1] < 0 || pairs[2 * p + 1] >= N ||
          pairs[2 * p] == pairs[2 * p + 1])
        return pfe::fail(PFE_EINVAL, "spring pair out of range");
  const size_t bG = (size_t)h->nnzb * 9 * sizeof(double);
  const size_t need = bG + (size_t)P * (16 + 24 + 8) + (size_t)N * 8 + 256;
  PFE_HIP(h->wsA.ensure(need));
  char* base = h->wsA.as<char>();
  double* G = (double*)base;
  int64_t* pr = (int64_t*)(base + bG);
  double* un = (double*)(pr + 2 * P);
  double* dkd = un + 3 * P;
  double* dmd = dkd + P;
  const int64_t* prs = pairs;
  const double* uns = unit;
  const double* Gs = dblocks;
  if (!dev) {
    PFE_TRY(upload(h, pr, pairs, 2 * P, false));
    PFE_TRY(upload(h, un, unit, 3 * P, false));
    PFE_TRY(upload(h, G, dblocks, h->nnzb * 9, false));
    prs = pr;
    uns = un;
    Gs = G;
  }
  int* eflag = h->flags.as<int>();
  PFE_HIP(hipMemsetAsync(eflag, 0, sizeof(int), h->stream));
  PFE_HIP(pfe::spring_chain(h->bsr(), h->transpose.as<int32_t>(), h->H.as<double>(),
                            h->masses.as<double>(), Gs, P, prs, uns, dev ? dk : dkd,
                            dev ? dm : dmd, eflag, h->stream));
  int ef = 0;
  PFE_HIP(hipMemcpyAsync(&ef, eflag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  if (!dev) {
    PFE_TRY(download(h, dk, dkd, P, false));
    PFE_TRY(download(h, dm, dmd, N, false));
  }
  PFE_TRY(sync(h));
  if (ef & 2) return pfe::fail(PFE_EINVAL, "spring pair out of range");
  if (ef) return pfe::fail(PFE_EINVAL, "a spring's blocks are not stored in the Hessian");
  return pfe::ok();
}

pfe_status pfe_spring_gradient(pfe_handle h, int64_t n_springs, const int64_t* pairs,
                               const double* unit, const double* dblocks, double* dk, double* dm,
                               uint32_t flags) {
  if (!h) return PFE_EINVAL;
  return guarded(h, [&] { return spring_grad_impl(h, n_springs, pairs, unit, dblocks, dk, dm, flags); });
}

}  // extern "C"
