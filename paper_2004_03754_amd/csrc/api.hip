// C ABI of the yeepic library: validation, buffers, dispatch, the step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <climits>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "yeepic_internal.h"

// Per-species buffers of the tile-sorted plasma path (grow-only).
struct SortState {
  int64_t cap = 0;
  int nbins = 0;  // sort keys (tiles times their bins: x3 planes and pairs of x2 rows)
  int* keys = nullptr;
  int* counts = nullptr;
  int* offsets = nullptr;
  int* cursors = nullptr;
  int* segsum = nullptr;  // per-segment sums of the count scan
  double* xs[3] = {nullptr, nullptr, nullptr};
  double* us[3] = {nullptr, nullptr, nullptr};
  int64_t* ids = nullptr;
  int* perm = nullptr;  // a sort's permutation (sorted position -> source index)
};

struct pic_grid {
  int ndim = 0;
  int64_t n[3] = {0, 0, 0};
  double dx[3] = {0, 0, 0};
  double dt = 0;
  int M = 0;
  double CE[PIC_MAX_M] = {};
  double CB[PIC_MAX_M] = {};
  int ME = 0, MB = 0;  // widths after trimming negligible trailing coefficients
  int prec = 0;
  size_t elem = 0;
  void* E[3] = {nullptr, nullptr, nullptr};
  void* B[3] = {nullptr, nullptr, nullptr};
  void* J[3] = {nullptr, nullptr, nullptr};
  void* alt[6] = {};  // second field set for the out-of-place sweep
  hipStream_t stream = nullptr;
  int* d_flag = nullptr;
  int* d_noconv = nullptr;  // exact pushes whose proper-time solve hit the iteration cap
  int deposit_mode = PIC_DEPOSIT_ATOMIC;
  double* stage = nullptr;  // deterministic mode: the tiles' staged currents (grow-only)
  size_t stage_cap = 0;
  SortState dsort;  // tile sort of (x_old, x_new) for pic_deposit_J on a 3D grid
  double* xo[3] = {nullptr, nullptr, nullptr};  // x^n scratch of the unsorted deposit path (grow-only)
  int64_t xo_cap = 0;
  int sort_every = 3;  // 3: the 64-bit tile current then fits three workgroups per CU
  std::vector<SortState> sorts;
  // vacuum step loop: two tile-ordered copies per species (re-sort ping-pong)
  std::vector<SortState> vsort_a, vsort_b;
  double* partial = nullptr;  // per-block partial sums of the coefficient gradients
  int64_t partial_cap = 0;
  double* noalloc = nullptr;  // device address of the static adjoint scratch on the grid's device
  // x1 current correction for a non-Yee C^B (Sec. 3.3): taps of the periodic
  // kernel, zero-padded to corr_kw + 1, and the corrected x1 current
  int corr_status = 0;     // PIC_OK, or why no kernel could be built
  int corr_kw = 0;         // tap half-width used by the kernel (8, 16, 32, 64)
  int corr_w = 0;          // last nonzero tap
  double* corr_taps = nullptr;
  void* Jc = nullptr;
  // moving window: array column of window cell 0, cells moved so far, and
  // the compaction scratch (grow-only)
  int64_t win_origin = 0, win_moved = 0;
  int absorb_w = 0;  // absorbing layers at the x1 ends: width in cells (0: none) and strength
  double absorb_sigma = 0.0;
  int* win_counts = nullptr;
  int64_t* win_offs = nullptr;
  int64_t win_nb_cap = 0;
  double* win_data = nullptr;  // x[3], u[3], id: 7 arrays of win_cap
  int64_t win_cap = 0;
  yeepic::Mesh mesh = {};
};

namespace yeepic {

static thread_local char g_err[512] = "no error";

// Device scratch of the allocation-free adjoint step: the per-block partial
// sums of the coefficient gradients (PIC_MAX_M doubles per reduction block).
// Each device holds its own copy until the process ends.  Host code never
// passes ``scratch`` itself to a kernel: it uses the device address that
// hipGetSymbolAddress returns for the current device (scratch_on_device).
constexpr int64_t kNoAllocDoubles = (int64_t)1 << 17;  // 1 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// The address of ``scratch`` on the current device, looked up once per
// device; nullptr with the error recorded when the lookup fails.
static double* scratch_on_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error(PIC_EHIP, "no usable current device for the adjoint scratch");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    double* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(PIC_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// vacuum step loop: species of at least kVacSortMin particles are pushed as a
// tile-ordered copy, re-sorted every kVacSortEvery steps (|v| < c moves a
// particle at most kVacSortEvery dt / dx1 = 8 cells at dt = dx1/2, one tile)
constexpr int64_t kVacSortMin = 1 << 15;
constexpr int kVacSortEvery = 16;

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

static int hip_fail(hipError_t e, const char* what) {
  return set_error(PIC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Last index whose trailing tail is not negligible: sum_{q>m} |C_q| <= 2^-70 sum|C|.
static int effective_width(const double* C, int M) {
  double total = 0;
  for (int q = 0; q < M; ++q) total += std::fabs(C[q]);
  const double tol = std::ldexp(total, -70);
  double tail = 0;
  int m = M;
  while (m > 1) {
    tail += std::fabs(C[m - 1]);
    if (tail > tol) break;
    --m;
  }
  return m;
}

static int swap_into_caller(pic_grid* g) {
  // copy the alt set back into the caller's arrays
  const size_t bytes = (size_t)g->n[0] * g->n[1] * g->n[2] * g->elem;
  for (int c = 0; c < 3; ++c) {
    hipError_t e = hipMemcpyAsync(g->E[c], g->alt[c], bytes, hipMemcpyDeviceToDevice, g->stream);
    if (e != hipSuccess) return hip_fail(e, "sweep copy-back");
    e = hipMemcpyAsync(g->B[c], g->alt[3 + c], bytes, hipMemcpyDeviceToDevice, g->stream);
    if (e != hipSuccess) return hip_fail(e, "sweep copy-back");
  }
  return PIC_OK;
}

static bool ampere_is_yee(const pic_grid* g) { return g->MB == 1 && g->CB[0] == 1.0; }

// Taps of the x1 current correction (Sec. 3.3, Eq. correction): the periodic
// kernel h whose discrete Fourier transform on the n1 modes of the x1 axis is
//   R(theta) = [k]_Yee/[k]_B1 = sin(theta/2) / sum_j C^B_j sin((2j-1) theta/2),
// theta = k1 dx1, with R(0) = 1/sum_j (2j-1) C^B_j.  h[m] = (1/N) sum_q
// R(theta_q) cos(m theta_q), theta_q = 2 pi q/N, evaluated in long double with
// N = n1 (exactly the mesh's periodic kernel) up to 16384; for longer rows
// N = 16384, whose aliases lie 16384 cells away (negligible for any kernel
// that passes the decay test).  The taps are cut after the last one above
// 2^-56 (FP64 fields) or 2^-32 (FP32 fields, well below the output's rounding)
// of their absolute sum, looking 128 cells out; the cut must fall within 64
// cells and below n1/2.
static int build_correction(pic_grid* g) {
  const int MB = g->MB;
  const int n1 = (int)g->n[0];
  const int N = n1 < 16384 ? n1 : 16384;
  const int mmax = std::min(128, N / 2);
  std::vector<long double> h(mmax + 1, 0.0L);
  long double csum = 0, kmax = 0;
  for (int j = 0; j < MB; ++j) csum += (2 * j + 1) * (long double)g->CB[j];
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<long double> kb(N), R(N);
  for (int q = 0; q < N; ++q) {
    const long double th = 2 * pi * q / N;
    long double v = 0;
    for (int j = 0; j < MB; ++j) v += g->CB[j] * sinl((2 * j + 1) * th / 2);
    kb[q] = v;
    kmax = std::max(kmax, fabsl(v));
  }
  for (int q = 1; q < N; ++q)
    if (fabsl(kb[q]) <= 1e-12L * kmax) return PIC_EUNSUPPORTED;  // [k]_B1 vanishes at a mode
  R[0] = 1.0L / csum;
  for (int q = 1; q < N; ++q) R[q] = sinl(pi * q / N) / kb[q];
  for (int q = 0; q < N; ++q) {
    // cos(m theta) by the three-term recurrence
    const long double c1 = cosl(2 * pi * q / N);
    long double cm1 = c1, cm = 1;  // cos(-theta), cos(0)
    for (int mm = 0; mm <= mmax; ++mm) {
      h[mm] += R[q] * cm;
      const long double nx = 2 * c1 * cm - cm1;
      cm1 = cm;
      cm = nx;
    }
  }
  long double asum = 0;
  for (int mm = 0; mm <= mmax; ++mm) {
    h[mm] /= N;
    asum += (mm ? 2 : 1) * fabsl(h[mm]);
  }
  int W = 0;
  const int cut = g->prec == PIC_FP64 ? -56 : -32;
  for (int mm = 1; mm <= mmax; ++mm)
    if (fabsl(h[mm]) > ldexpl(asum, cut)) W = mm;
  if (W > 64 || 2 * W >= n1) return PIC_EUNSUPPORTED;
  const int kw = W <= 8 ? 8 : W <= 16 ? 16 : W <= 24 ? 24 : W <= 32 ? 32 : W <= 40 ? 40 : W <= 48 ? 48 : 64;
  std::vector<double> taps(kw + 1, 0.0);
  for (int mm = 0; mm <= W; ++mm) taps[mm] = (double)h[mm];
  if (hipMalloc((void**)&g->corr_taps, taps.size() * sizeof(double)) != hipSuccess) return PIC_ENOMEM;
  if (hipMemcpy(g->corr_taps, taps.data(), taps.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return PIC_EHIP;
  g->corr_kw = kw;
  g->corr_w = W;
  return PIC_OK;
}

static int correction_error(const pic_grid* g) {
  if (g->corr_status == PIC_ENOMEM) return set_error(PIC_ENOMEM, "cannot allocate the current-correction buffers");
  if (g->corr_status == PIC_EHIP) return set_error(PIC_EHIP, "cannot upload the current-correction taps");
  return set_error(PIC_EUNSUPPORTED,
                   "x1 current correction: [k]_B1 vanishes at a mode or its kernel is wider than 64 cells");
}

// The corrected x1 current's buffer, for a grid with a current and a non-Yee
// C^B (allocated once, when J is first set).
static int ensure_jc(pic_grid* g) {
  if (g->Jc || !g->J[0] || ampere_is_yee(g) || g->corr_status) return PIC_OK;
  const size_t bytes = (size_t)g->n[0] * g->n[1] * g->n[2] * g->elem;
  if (hipMalloc(&g->Jc, bytes) != hipSuccess) {
    g->Jc = nullptr;
    return set_error(PIC_ENOMEM, "cannot allocate the corrected x1 current");
  }
  return PIC_OK;
}

// The current Ampere's law uses: J, with its x1 component replaced by the
// corrected one (written to g->Jc) when C^B is not the Yee stencil.
static int ampere_current(pic_grid* g, void* Ja[3]) {
  for (int c = 0; c < 3; ++c) Ja[c] = g->J[c];
  if (ampere_is_yee(g)) return PIC_OK;
  if (g->corr_status) return correction_error(g);
  int rc = ensure_jc(g);
  if (rc == PIC_OK) rc = launch_correct_j1(g->prec, g->mesh, g->J[0], g->Jc, g->corr_taps, g->corr_kw, g->stream);
  if (rc == PIC_OK) Ja[0] = g->Jc;
  return rc;
}

static int check_particles(const pic_grid* g, const pic_particles* p) {
  if (!p) return set_error(PIC_EINVAL, "particles is NULL");
  if (p->np < 0) return set_error(PIC_EINVAL, "negative particle count");
  if (p->np == 0) return PIC_OK;
  for (int d = 0; d < 3; ++d)
    if (!p->u[d]) return set_error(PIC_EINVAL, "particle momentum u[%d] is NULL", d);
  for (int d = 0; d < g->ndim; ++d)
    if (!p->x[d]) return set_error(PIC_EINVAL, "particle position x[%d] is NULL", d);
  if (g->ndim == 2 && g->n[2] > 1 && !p->x[2])
    return set_error(PIC_EINVAL, "a stack of 2D meshes needs x[2] (the plane index)");
  if (!(p->m > 0) || !std::isfinite(p->q) || !std::isfinite(p->w))
    return set_error(PIC_EINVAL, "bad species constants");
  if (p->np > ((int64_t)1 << 31) * 256) return set_error(PIC_EINVAL, "too many particles");
  return PIC_OK;
}

static void free_sort(SortState& st) {
  void* ptrs[] = {st.keys, st.counts, st.offsets, st.cursors, st.segsum, st.xs[0], st.xs[1], st.xs[2],
                  st.us[0], st.us[1], st.us[2], st.ids, st.perm};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  st = SortState();
}

// Sort buffers for np particles: keys, counts and scan state; with
// ``payload`` the second particle set (x, u, and ids with ``ids``); with
// ``perm`` the permutation.
static int ensure_sort(pic_grid* g, SortState& st, int64_t np, int nbins, bool ids, bool perm = false,
                       bool payload = true) {
  if (np <= st.cap && nbins == st.nbins && (!ids || st.ids) && (!perm || st.perm) && (!payload || st.xs[0]))
    return PIC_OK;
  (void)hipStreamSynchronize(g->stream);
  free_sort(st);
  const size_t n = (size_t)(np > 0 ? np : 1);
  bool ok = hipMalloc((void**)&st.keys, n * sizeof(int)) == hipSuccess &&
            hipMalloc((void**)&st.counts, (size_t)nbins * sizeof(int)) == hipSuccess &&
            hipMalloc((void**)&st.offsets, ((size_t)nbins + 1) * sizeof(int)) == hipSuccess &&
            hipMalloc((void**)&st.cursors, (size_t)nbins * sizeof(int)) == hipSuccess &&
            hipMalloc((void**)&st.segsum, (size_t)scan_segments(nbins) * sizeof(int)) == hipSuccess;
  for (int d = 0; d < 3 && ok && payload; ++d)
    ok = hipMalloc((void**)&st.xs[d], n * sizeof(double)) == hipSuccess &&
         hipMalloc((void**)&st.us[d], n * sizeof(double)) == hipSuccess;
  if (ok && ids) ok = hipMalloc((void**)&st.ids, n * sizeof(int64_t)) == hipSuccess;
  if (ok && perm) ok = hipMalloc((void**)&st.perm, n * sizeof(int)) == hipSuccess;
  if (!ok) {
    free_sort(st);
    return set_error(PIC_ENOMEM, "cannot allocate particle sort buffers for %lld particles", (long long)np);
  }
  st.cap = np;
  st.nbins = nbins;
  return PIC_OK;
}

// Deterministic deposit mode: staging for every tile's current, and the
// limits of the fixed-order node reduction (tiles and periodic images per
// direction that may cover one node).
static int ensure_stage(pic_grid* g, const TileGeom& tg) {
  const int n[3] = {(int)g->n[0], (int)g->n[1], (int)g->n[2]};
  for (int d = 0; d < 3; ++d) {
    const int reach = (tg.m[d] + 2 + tg.t[d] - 1) / tg.t[d] + 1;
    const int cand = std::min(tg.nt[d], 2 * reach + 1);
    if (cand > 16 || cand * (tg.r[d] / n[d] + 1) > 64)
      return set_error(PIC_EUNSUPPORTED, "deterministic deposit: tile window too wide for the mesh along x%d", d + 1);
  }
  const size_t need = stage_doubles(tg);
  if (need <= g->stage_cap) return PIC_OK;
  (void)hipStreamSynchronize(g->stream);
  if (g->stage) (void)hipFree(g->stage);
  g->stage = nullptr;
  g->stage_cap = 0;
  if (hipMalloc((void**)&g->stage, need * sizeof(double)) != hipSuccess)
    return set_error(PIC_ENOMEM, "cannot allocate %zu bytes of current staging", need * sizeof(double));
  g->stage_cap = need;
  return PIC_OK;
}

// Tile sorts index particles with 32-bit offsets.
static int check_sortable(const pic_particles* p) {
  if (p->np > (int64_t)INT32_MAX)
    return set_error(PIC_EUNSUPPORTED, "a tile-sorted species holds at most 2^31 - 1 particles (got %lld)",
                     (long long)p->np);
  return PIC_OK;
}

}  // namespace yeepic

using namespace yeepic;

extern "C" {

const char* pic_last_error(void) { return g_err; }

int pic_init_grid(const pic_grid_desc* d, pic_grid** out) {
  if (!d || !out) return set_error(PIC_EINVAL, "pic_init_grid: NULL argument");
  *out = nullptr;
  if (d->ndim != 2 && d->ndim != 3) return set_error(PIC_EINVAL, "ndim must be 2 or 3");
  if (d->prec != PIC_FP64 && d->prec != PIC_FP32_FIELDS) return set_error(PIC_EINVAL, "bad precision");
  if (d->M < 1 || d->M > PIC_MAX_M) return set_error(PIC_EINVAL, "M must be in 1..16");
  if (!d->CE || !d->CB) return set_error(PIC_EINVAL, "coefficient arrays are NULL");
  for (int a = 0; a < 3; ++a)
    if (d->n[a] < 1 || d->n[a] > (1 << 20)) return set_error(PIC_ESHAPE, "mesh size n[%d] out of range", a);
  if (d->n[0] % 64 != 0) return set_error(PIC_ESHAPE, "n1 must be a multiple of 64");
  if (d->n[0] < 2 * d->M) return set_error(PIC_ESHAPE, "n1 must be at least 2M");
  const int64_t cells = d->n[0] * d->n[1] * d->n[2];
  if (cells > ((int64_t)1 << 31) - 1) return set_error(PIC_ESHAPE, "mesh larger than 2^31 cells");
  for (int a = 0; a < d->ndim; ++a)
    if (!(d->dx[a] > 0) || !std::isfinite(d->dx[a])) return set_error(PIC_EINVAL, "bad cell size");
  if (!(d->dt > 0) || !std::isfinite(d->dt)) return set_error(PIC_EINVAL, "bad time step");
  for (int c = 0; c < 3; ++c) {
    if (!d->E[c] || !d->B[c]) return set_error(PIC_EINVAL, "field pointer is NULL");
    if (((uintptr_t)d->E[c] | (uintptr_t)d->B[c]) & 15) return set_error(PIC_ESHAPE, "fields must be 16-byte aligned");
  }
  double sE = 0, sB = 0;
  for (int q = 0; q < d->M; ++q) {
    if (!std::isfinite(d->CE[q]) || !std::isfinite(d->CB[q])) return set_error(PIC_EINVAL, "non-finite coefficient");
    sE += std::fabs(d->CE[q]);
    sB += std::fabs(d->CB[q]);
  }
  // Sec. 3.2 sufficient CFL bound (3D adds the x3 term)
  double lim = sB * sE / (d->dx[0] * d->dx[0]) + 1.0 / (d->dx[1] * d->dx[1]);
  if (d->ndim == 3) lim += 1.0 / (d->dx[2] * d->dx[2]);
  if (d->dt > 1.0 / std::sqrt(lim))
    return set_error(PIC_ECFL, "dt = %g exceeds the CFL bound %g", d->dt, 1.0 / std::sqrt(lim));

  pic_grid* g = new pic_grid();
  g->ndim = d->ndim;
  for (int a = 0; a < 3; ++a) {
    g->n[a] = d->n[a];
    g->dx[a] = (a < d->ndim) ? d->dx[a] : 1.0;
  }
  g->dt = d->dt;
  g->M = d->M;
  for (int q = 0; q < d->M; ++q) {
    g->CE[q] = d->CE[q];
    g->CB[q] = d->CB[q];
  }
  g->ME = effective_width(g->CE, g->M);
  g->MB = effective_width(g->CB, g->M);
  g->prec = d->prec;
  g->elem = d->prec == PIC_FP64 ? sizeof(double) : sizeof(float);
  for (int c = 0; c < 3; ++c) {
    g->E[c] = d->E[c];
    g->B[c] = d->B[c];
    g->J[c] = d->J[c];
  }
  g->stream = (hipStream_t)d->stream;
  Mesh& m = g->mesh;
  m.n1 = (int)g->n[0];
  m.n2 = (int)g->n[1];
  m.n3 = (int)g->n[2];
  m.ndim = g->ndim;
  m.order = 1;
  m.dx1 = g->dx[0];
  m.dx2 = g->dx[1];
  m.dx3 = g->dx[2];
  m.idx1 = 1.0 / m.dx1;
  m.idx2 = 1.0 / m.dx2;
  m.idx3 = 1.0 / m.dx3;
  m.L1 = m.n1 * m.dx1;
  m.L2 = m.n2 * m.dx2;
  m.L3 = m.n3 * m.dx3;
  m.exact_iters = 100;
  m.noconv = nullptr;
  const size_t bytes = (size_t)cells * g->elem;
  for (int c = 0; c < 6; ++c) {
    if (hipMalloc(&g->alt[c], bytes) != hipSuccess) {
      pic_destroy(g);
      return set_error(PIC_ENOMEM, "cannot allocate %zu bytes for the sweep buffers", 6 * bytes);
    }
  }
  if (hipMalloc((void**)&g->d_flag, sizeof(int)) != hipSuccess) {
    pic_destroy(g);
    return set_error(PIC_ENOMEM, "cannot allocate the flag word");
  }
  if (hipMalloc((void**)&g->d_noconv, sizeof(int)) != hipSuccess ||
      hipMemset(g->d_noconv, 0, sizeof(int)) != hipSuccess) {
    pic_destroy(g);
    return set_error(PIC_ENOMEM, "cannot allocate the pusher convergence counter");
  }
  m.noconv = g->d_noconv;
  g->noalloc = scratch_on_device();
  if (!g->noalloc) {
    const int rc = PIC_EHIP;
    pic_destroy(g);
    return rc;
  }
  if (!ampere_is_yee(g)) {
    g->corr_status = build_correction(g);
    int rc = g->corr_status == PIC_ENOMEM || g->corr_status == PIC_EHIP ? correction_error(g) : ensure_jc(g);
    if (rc) {
      pic_destroy(g);
      return rc;
    }
  }
  *out = g;
  return PIC_OK;
}

int pic_set_fields(pic_grid* g, void* const E[3], void* const B[3], void* const J[3]) {
  if (!g || !E || !B) return set_error(PIC_EINVAL, "pic_set_fields: NULL argument");
  for (int c = 0; c < 3; ++c) {
    if (!E[c] || !B[c]) return set_error(PIC_EINVAL, "field pointer is NULL");
    if (((uintptr_t)E[c] | (uintptr_t)B[c]) & 15) return set_error(PIC_ESHAPE, "fields must be 16-byte aligned");
  }
  for (int c = 0; c < 3; ++c) {
    g->E[c] = E[c];
    g->B[c] = B[c];
    g->J[c] = J ? J[c] : nullptr;
  }
  return ensure_jc(g);
}

int pic_grid_widths(const pic_grid* g, int* ME, int* MB) {
  if (!g || !ME || !MB) return set_error(PIC_EINVAL, "pic_grid_widths: NULL argument");
  *ME = g->ME;
  *MB = g->MB;
  return PIC_OK;
}

int pic_advance_B_half(pic_grid* g) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  return launch_advance_b(g->prec, g->mesh, g->E, g->B, g->B, g->CE, g->ME, 0.5 * g->dt, g->stream);
}

int pic_advance_E(pic_grid* g, int use_J) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (use_J && !(g->J[0] && g->J[1] && g->J[2])) return set_error(PIC_EINVAL, "use_J set but J is not");
  void* Ja[3] = {nullptr, nullptr, nullptr};
  if (use_J) {
    const int rc = ampere_current(g, Ja);
    if (rc) return rc;
  }
  return launch_advance_e(g->prec, g->mesh, g->E, g->B, Ja, g->CB, g->MB, g->dt, g->stream);
}

static int sweep_once(pic_grid* g, void* const inE[3], void* const inB[3], void* const outE[3],
                      void* const outB[3], int use_J, void* const half[3] = nullptr) {
  void* Ja[3] = {nullptr, nullptr, nullptr};
  if (use_J) {
    const int rc = ampere_current(g, Ja);
    if (rc) return rc;
  }
  return launch_sweep(g->prec, g->mesh, inE, inB, Ja, outE, outB, half, g->CE, g->ME, g->CB, g->MB, g->dt,
                      g->stream);
}

int pic_current_correction(pic_grid* g, void* J1_out) {
  if (!g || !J1_out) return set_error(PIC_EINVAL, "pic_current_correction: NULL argument");
  if (!g->J[0]) return set_error(PIC_EINVAL, "grid has no current arrays");
  if ((uintptr_t)J1_out & 15) return set_error(PIC_ESHAPE, "J1_out must be 16-byte aligned");
  const size_t bytes = (size_t)g->n[0] * g->n[1] * g->n[2] * g->elem;
  const uintptr_t a = (uintptr_t)J1_out, b = (uintptr_t)g->J[0];
  if (a < b + bytes && b < a + bytes) return set_error(PIC_EINVAL, "J1_out overlaps J[0]");
  if (ampere_is_yee(g))
    return hipMemcpyAsync(J1_out, g->J[0], bytes, hipMemcpyDeviceToDevice, g->stream) == hipSuccess
               ? PIC_OK
               : set_error(PIC_EHIP, "current copy");
  if (g->corr_status) return correction_error(g);
  return launch_correct_j1(g->prec, g->mesh, g->J[0], J1_out, g->corr_taps, g->corr_kw, g->stream);
}

// The absorbing layers (if set) on the fields of a finished step.
static int absorb_after_step(pic_grid* g, void* const E[3], void* const B[3]) {
  return launch_damp_columns(g->prec, g->mesh, E, B, g->win_origin, g->absorb_w, g->absorb_sigma, g->stream);
}

int pic_field_sweep(pic_grid* g, int use_J) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (use_J && !(g->J[0] && g->J[1] && g->J[2])) return set_error(PIC_EINVAL, "use_J set but J is not");
  int rc = sweep_once(g, g->E, g->B, g->alt, g->alt + 3, use_J);
  if (rc == PIC_OK) rc = absorb_after_step(g, g->alt, g->alt + 3);
  if (rc) return rc;
  return swap_into_caller(g);
}

int pic_set_absorber(pic_grid* g, int width, double sigma) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (width < 0 || 2 * (int64_t)width > g->n[0]) return set_error(PIC_EINVAL, "absorber width must be in 0..n1/2");
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) return set_error(PIC_EINVAL, "absorber strength must be >= 0");
  g->absorb_w = width;
  g->absorb_sigma = sigma;
  return PIC_OK;
}

int pic_gather_push(pic_grid* g, pic_particles* p, int pusher, double* const x_old[3]) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  int rc = check_particles(g, p);
  if (rc) return rc;
  if (pusher != PIC_PUSH_BORIS && pusher != PIC_PUSH_ANALYTIC && pusher != PIC_PUSH_HC)
    return set_error(PIC_EINVAL, "bad pusher");
  if (x_old)
    for (int d = 0; d < g->ndim; ++d)
      if (!x_old[d]) return set_error(PIC_EINVAL, "x_old[%d] is NULL", d);
  return launch_gather_push(g->prec, g->mesh, g->E, g->B, *p, pusher, g->dt, x_old, g->stream);
}

int pic_deposit_J(pic_grid* g, const pic_particles* p, double* const x_old[3], int zero_first) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  int rc = check_particles(g, p);
  if (rc) return rc;
  if (!(g->J[0] && g->J[1] && g->J[2])) return set_error(PIC_EINVAL, "grid has no current arrays");
  if (!x_old) return set_error(PIC_EINVAL, "x_old is NULL");
  for (int d = 0; d < g->ndim; ++d)
    if (!x_old[d]) return set_error(PIC_EINVAL, "x_old[%d] is NULL", d);
  if (g->ndim != 3) {
    if (g->deposit_mode == PIC_DEPOSIT_DETERMINISTIC)
      return set_error(PIC_EUNSUPPORTED, "the deterministic deposit covers 3D grids");
  } else {
    rc = check_sortable(p);
    if (rc) return rc;
  }
  if (zero_first) {
    const size_t bytes = (size_t)g->n[0] * g->n[1] * g->n[2] * g->elem;
    for (int c = 0; c < 3; ++c) {
      hipError_t e = hipMemsetAsync(g->J[c], 0, bytes, g->stream);
      if (e != hipSuccess) return hip_fail(e, "clear J");
    }
  }
  if (g->ndim != 3 || p->np == 0) return launch_deposit(g->prec, g->mesh, g->J, *p, x_old, g->dt, g->stream);
  // 3D: counting sort of (x_old, x) by the tile of x_old, as a permutation
  // the tile kernel reads the pairs through; it accumulates each tile's
  // current on chip (moves below one cell, so the window needs no drift
  // margin)
  const TileGeom tg = make_tile_geom(g->mesh, g->dt, 1);
  rc = ensure_sort(g, g->dsort, p->np, tg.nbins, false, true, false);
  double* stage = nullptr;
  if (rc == PIC_OK && g->deposit_mode == PIC_DEPOSIT_DETERMINISTIC) {
    rc = ensure_stage(g, tg);
    stage = g->stage;
  }
  if (rc) return rc;
  pic_particles pairs = *p;  // keys from x_old; x_new read beside it
  for (int d = 0; d < 3; ++d) {
    pairs.x[d] = x_old[d];
    pairs.u[d] = p->x[d];
  }
  pairs.id = nullptr;
  SortState& st = g->dsort;
  rc = launch_tile_sort(g->mesh, tg, pairs, pairs, st.keys, st.counts, st.offsets, st.cursors, st.segsum, g->stream,
                        false, st.perm);
  if (rc) return rc;
  return launch_tile_deposit(g->prec, g->mesh, tg, g->J, st.offsets, pairs, g->dt, stage, g->stream, st.perm);
}

int pic_step_n(pic_grid* g, pic_particles* const* species, int nspecies, int nsteps, int pusher, int deposit) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (nsteps < 0 || nspecies < 0) return set_error(PIC_EINVAL, "negative count");
  if (nspecies > 0 && !species) return set_error(PIC_EINVAL, "species is NULL");
  if (pusher != PIC_PUSH_BORIS && pusher != PIC_PUSH_ANALYTIC && pusher != PIC_PUSH_HC)
    return set_error(PIC_EINVAL, "bad pusher");
  for (int s = 0; s < nspecies; ++s) {
    int rc = check_particles(g, species[s]);
    if (rc) return rc;
  }
  if (deposit) {
    if (!(g->J[0] && g->J[1] && g->J[2])) return set_error(PIC_EINVAL, "deposit requested without J");
    if (!ampere_is_yee(g) && g->corr_status) return correction_error(g);
    if (g->ndim != 3 && g->deposit_mode == PIC_DEPOSIT_DETERMINISTIC)
      return set_error(PIC_EUNSUPPORTED, "the deterministic deposit covers 3D grids");
  }
  // scratch for x^n of the largest species (kept across calls)
  int64_t npmax = 0;
  for (int s = 0; s < nspecies; ++s) npmax = species[s]->np > npmax ? species[s]->np : npmax;
  double* xo[3] = {nullptr, nullptr, nullptr};
  if (deposit && g->ndim != 3 && npmax > 0) {
    if (npmax > g->xo_cap) {
      (void)hipStreamSynchronize(g->stream);
      for (int d = 0; d < 3; ++d) {
        (void)hipFree(g->xo[d]);
        g->xo[d] = nullptr;
      }
      g->xo_cap = 0;
      for (int d = 0; d < g->ndim; ++d)
        if (hipMalloc((void**)&g->xo[d], (size_t)npmax * sizeof(double)) != hipSuccess)
          return set_error(PIC_ENOMEM, "cannot allocate position scratch");
      g->xo_cap = npmax;
    }
    for (int d = 0; d < 3; ++d) xo[d] = g->xo[d];
  }
  void* cur[6] = {g->E[0], g->E[1], g->E[2], g->B[0], g->B[1], g->B[2]};
  void* nxt[6] = {g->alt[0], g->alt[1], g->alt[2], g->alt[3], g->alt[4], g->alt[5]};
  int rc = PIC_OK;
  const size_t jbytes = (size_t)g->n[0] * g->n[1] * g->n[2] * g->elem;
  // 3D plasma: particles sorted by tile, current accumulated on chip
  const bool tiled = deposit && g->ndim == 3;
  TileGeom tg = {};
  double* stage = nullptr;
  if (tiled) {
    tg = make_tile_geom(g->mesh, g->dt, g->sort_every);
    for (int s = 0; s < nspecies && rc == PIC_OK; ++s) rc = check_sortable(species[s]);
    if ((int)g->sorts.size() < nspecies) g->sorts.resize(nspecies);
    for (int s = 0; s < nspecies && rc == PIC_OK; ++s)
      rc = ensure_sort(g, g->sorts[s], species[s]->np, tg.nbins, species[s]->id != nullptr, true);
    if (rc == PIC_OK && g->deposit_mode == PIC_DEPOSIT_DETERMINISTIC) {
      rc = ensure_stage(g, tg);
      stage = g->stage;
    }
    if (rc) return rc;
  }
  // 3D vacuum: each large species is pushed as a tile-ordered copy, so that
  // the eight-node gathers of a wave share cache lines; the copy is re-sorted
  // every kVacSortEvery steps and scattered back to the caller's order at the
  // end.  Every particle's arithmetic is the same as in place.
  const bool vac = !deposit && g->ndim == 3 && nsteps >= 2;
  std::vector<pic_particles> vcur, valt;
  std::vector<char> vuse;
  if (vac) {
    tg = make_tile_geom(g->mesh, g->dt, 1);
    if ((int)g->vsort_a.size() < nspecies) {
      g->vsort_a.resize(nspecies);
      g->vsort_b.resize(nspecies);
    }
    vcur.resize(nspecies);
    valt.resize(nspecies);
    vuse.assign(nspecies, 0);
    for (int s = 0; s < nspecies && rc == PIC_OK; ++s) {
      if (species[s]->np < kVacSortMin) continue;
      rc = check_sortable(species[s]);
      if (rc) break;
      SortState& A = g->vsort_a[s];
      SortState& B = g->vsort_b[s];
      rc = ensure_sort(g, A, species[s]->np, tg.nbins, true);
      if (rc == PIC_OK) rc = ensure_sort(g, B, species[s]->np, tg.nbins, true);
      if (rc) break;
      vuse[s] = 1;
      vcur[s] = valt[s] = *species[s];
      for (int d = 0; d < 3; ++d) {
        vcur[s].x[d] = A.xs[d];
        vcur[s].u[d] = A.us[d];
        valt[s].x[d] = B.xs[d];
        valt[s].u[d] = B.us[d];
      }
      vcur[s].id = A.ids;
      valt[s].id = B.ids;
      // original indices (in B's id array) travel with the first sort into A
      pic_particles src = *species[s];
      src.id = B.ids;
      rc = launch_iota(B.ids, species[s]->np, g->stream);
      if (rc == PIC_OK)
        rc = launch_tile_sort(g->mesh, tg, src, vcur[s], A.keys, A.counts, A.offsets, A.cursors, A.segsum,
                                  g->stream);
    }
    if (rc) return rc;
  }
  // 3D plasma: a species' particles live in its own arrays or in the sort
  // scratch.  A sort only ranks them (a permutation), and the push after it
  // reads them through the permutation from one set and writes them sorted
  // into the other; steps between sorts push in place.  A call with an odd
  // number of sorts moves the particles at its first sort instead (scatter
  // into scratch, push back), so that every call ends with the particles in
  // the species' own arrays.
  const int nsorts = tiled ? (nsteps + g->sort_every - 1) / g->sort_every : 0;
  std::vector<char> in_scratch(tiled ? nspecies : 0, 0);
  for (int step = 0; step < nsteps && rc == PIC_OK; ++step) {
    if (deposit)
      for (int c = 0; c < 3 && rc == PIC_OK; ++c)
        if (hipMemsetAsync(g->J[c], 0, jbytes, g->stream) != hipSuccess) rc = set_error(PIC_EHIP, "clear J");
    for (int s = 0; s < nspecies && rc == PIC_OK; ++s) {
      if (tiled) {
        SortState& st = g->sorts[s];
        pic_particles scr = *species[s];
        for (int d = 0; d < 3; ++d) {
          scr.x[d] = st.xs[d];
          scr.u[d] = st.us[d];
        }
        scr.id = species[s]->id ? st.ids : nullptr;
        const pic_particles here = in_scratch[s] ? scr : *species[s];
        pic_particles src = here, dst = here;
        const int* perm = nullptr;
        if (step % g->sort_every == 0) {
          // after the first step of the call, the push before counted the tiles
          if (step == 0 && nsorts % 2 == 1) {
            rc = launch_tile_sort(g->mesh, tg, *species[s], scr, st.keys, st.counts, st.offsets, st.cursors,
                                  st.segsum, g->stream, false);
            src = scr;
            dst = *species[s];
          } else {
            rc = launch_tile_sort(g->mesh, tg, here, scr, st.keys, st.counts, st.offsets, st.cursors, st.segsum,
                                  g->stream, step > 0, st.perm);
            perm = st.perm;
            dst = in_scratch[s] ? *species[s] : scr;
            in_scratch[s] = !in_scratch[s];
          }
        }
        // the push before a sort writes the sort's keys and tile counts
        const bool count_next = (step + 1) % g->sort_every == 0 && step + 1 < nsteps;
        if (rc == PIC_OK)
          rc = launch_tile_push(g->prec, g->mesh, tg, cur, cur + 3, g->J, st.offsets, src, dst, pusher, g->dt,
                                stage, g->stream, count_next ? st.keys : nullptr, count_next ? st.counts : nullptr,
                                perm);
        continue;
      }
      if (vac && vuse[s]) {
        if (step > 0 && step % kVacSortEvery == 0) {
          SortState& D = (vcur[s].x[0] == g->vsort_a[s].xs[0]) ? g->vsort_b[s] : g->vsort_a[s];
          rc = launch_tile_sort(g->mesh, tg, vcur[s], valt[s], D.keys, D.counts, D.offsets, D.cursors, D.segsum,
                                g->stream);
          std::swap(vcur[s], valt[s]);
        }
        if (rc == PIC_OK) rc = launch_gather_push(g->prec, g->mesh, cur, cur + 3, vcur[s], pusher, g->dt, nullptr,
                                                  g->stream);
        continue;
      }
      rc = launch_gather_push(g->prec, g->mesh, cur, cur + 3, *species[s], pusher, g->dt, deposit ? xo : nullptr,
                              g->stream);
      if (rc == PIC_OK && deposit) rc = launch_deposit(g->prec, g->mesh, g->J, *species[s], xo, g->dt, g->stream);
    }
    if (rc == PIC_OK) rc = sweep_once(g, cur, cur + 3, nxt, nxt + 3, deposit);
    if (rc == PIC_OK) rc = absorb_after_step(g, nxt, nxt + 3);
    for (int c = 0; c < 6; ++c) std::swap(cur[c], nxt[c]);
  }
  if (vac)
    for (int s = 0; s < nspecies && rc == PIC_OK; ++s)
      if (vuse[s]) rc = launch_unsort(vcur[s], vcur[s].id, *species[s], g->stream);
  if (rc == PIC_OK && cur[0] != g->E[0]) {
    // odd number of steps: the state is in the alt set
    const size_t bytes = jbytes;
    for (int c = 0; c < 3 && rc == PIC_OK; ++c) {
      if (hipMemcpyAsync(g->E[c], cur[c], bytes, hipMemcpyDeviceToDevice, g->stream) != hipSuccess ||
          hipMemcpyAsync(g->B[c], cur[3 + c], bytes, hipMemcpyDeviceToDevice, g->stream) != hipSuccess)
        rc = set_error(PIC_EHIP, "step_n copy-back");
    }
  }
  return rc;
}

int pic_step_to(pic_grid* g, pic_particles* const* species, int nspecies, int pusher, void* const Eout[3],
                void* const Bout[3], void* const Bhalf[3]) {
  if (!g || !Eout || !Bout) return set_error(PIC_EINVAL, "pic_step_to: NULL argument");
  if (nspecies < 0) return set_error(PIC_EINVAL, "negative count");
  if (nspecies > 0 && !species) return set_error(PIC_EINVAL, "species is NULL");
  if (pusher != PIC_PUSH_BORIS && pusher != PIC_PUSH_ANALYTIC && pusher != PIC_PUSH_HC)
    return set_error(PIC_EINVAL, "bad pusher");
  for (int c = 0; c < 3; ++c) {
    if (!Eout[c] || !Bout[c]) return set_error(PIC_EINVAL, "output field pointer is NULL");
    if (((uintptr_t)Eout[c] | (uintptr_t)Bout[c]) & 15) return set_error(PIC_ESHAPE, "fields must be 16-byte aligned");
    for (int q = 0; q < 3; ++q)
      if (Eout[c] == g->E[q] || Eout[c] == g->B[q] || Bout[c] == g->E[q] || Bout[c] == g->B[q])
        return set_error(PIC_EINVAL, "pic_step_to: output aliases the grid's fields");
  }
  if (Bhalf)
    for (int c = 0; c < 3; ++c) {
      if (!Bhalf[c]) return set_error(PIC_EINVAL, "half-step field pointer is NULL");
      if ((uintptr_t)Bhalf[c] & 15) return set_error(PIC_ESHAPE, "fields must be 16-byte aligned");
      for (int q = 0; q < 3; ++q)
        if (Bhalf[c] == g->E[q] || Bhalf[c] == g->B[q] || Bhalf[c] == Eout[q] || Bhalf[c] == Bout[q])
          return set_error(PIC_EINVAL, "pic_step_to: half-step output aliases another field");
    }
  for (int s = 0; s < nspecies; ++s) {
    int rc = check_particles(g, species[s]);
    if (rc) return rc;
  }
  for (int s = 0; s < nspecies; ++s) {
    int rc = launch_gather_push(g->prec, g->mesh, g->E, g->B, *species[s], pusher, g->dt, nullptr, g->stream);
    if (rc) return rc;
  }
  int rc = sweep_once(g, g->E, g->B, Eout, Bout, 0, Bhalf);
  if (rc) return rc;
  return absorb_after_step(g, Eout, Bout);
}

// Argument checks shared by the two adjoint entry points.
static int adjoint_args(pic_grid* g, const pic_adjoint* adj, const pic_particles* const* species,
                        pic_particles* const* lambda, int nspecies, int pusher) {
  if (!g || !adj) return set_error(PIC_EINVAL, "pic_adjoint_step: NULL argument");
  if (g->prec != PIC_FP64) return set_error(PIC_EUNSUPPORTED, "the adjoint is built for FP64 grids only");
  if (pusher == PIC_PUSH_HC) return set_error(PIC_EUNSUPPORTED, "the adjoint covers the Boris and exact pushers");
  if (g->mesh.order != 1) return set_error(PIC_EUNSUPPORTED, "the adjoint covers the linear particle shape");
  if (g->absorb_w > 0) return set_error(PIC_EUNSUPPORTED, "the adjoint does not cover the absorbing layers");
  if (pusher != PIC_PUSH_BORIS && pusher != PIC_PUSH_ANALYTIC) return set_error(PIC_EINVAL, "bad pusher");
  if (nspecies < 0) return set_error(PIC_EINVAL, "negative count");
  if (nspecies > 0 && (!species || !lambda)) return set_error(PIC_EINVAL, "species or lambda is NULL");
  for (int c = 0; c < 3; ++c) {
    if (!adj->lE[c] || !adj->lB[c]) return set_error(PIC_EINVAL, "adjoint field pointer is NULL");
    if (((uintptr_t)adj->lE[c] | (uintptr_t)adj->lB[c]) & 15)
      return set_error(PIC_ESHAPE, "adjoint fields must be 16-byte aligned");
  }
  if (!adj->gCE || !adj->gCB) return set_error(PIC_EINVAL, "coefficient-gradient pointer is NULL");
  const bool outs = adj->lEo[0] || adj->lEo[1] || adj->lEo[2] || adj->lBo[0] || adj->lBo[1] || adj->lBo[2];
  if (outs) {
    const void* others[] = {adj->lE[0], adj->lE[1], adj->lE[2], adj->lB[0], adj->lB[1], adj->lB[2],
                            adj->En[0], adj->En[1], adj->En[2], adj->Bn[0], adj->Bn[1], adj->Bn[2],
                            adj->Bh[0], adj->Bh[1], adj->Bh[2], g->E[0], g->E[1], g->E[2],
                            g->B[0], g->B[1], g->B[2]};
    void* const o[6] = {adj->lEo[0], adj->lEo[1], adj->lEo[2], adj->lBo[0], adj->lBo[1], adj->lBo[2]};
    for (int c = 0; c < 6; ++c) {
      if (!o[c]) return set_error(PIC_EINVAL, "output cotangents: all six or none");
      if ((uintptr_t)o[c] & 15) return set_error(PIC_ESHAPE, "adjoint fields must be 16-byte aligned");
      for (const void* q : others)
        if (q == o[c]) return set_error(PIC_EINVAL, "an output cotangent aliases another array");
      for (int d = 0; d < c; ++d)
        if (o[d] == o[c]) return set_error(PIC_EINVAL, "output cotangents alias each other");
    }
  }
  for (int s = 0; s < nspecies; ++s) {
    int rc = check_particles(g, species[s]);
    if (rc) return rc;
    const pic_particles* l = lambda[s];
    if (!l || l->np != species[s]->np) return set_error(PIC_ESHAPE, "lambda[%d] does not match species[%d]", s, s);
    if (l->np > 0)
      for (int d = 0; d < 3; ++d)
        if (!l->u[d] || (d < g->ndim && !l->x[d]))
          return set_error(PIC_EINVAL, "lambda[%d] has a NULL array", s);
  }
  return PIC_OK;
}

// The adjoint step with ``partial`` (coef_partial_blocks * PIC_MAX_M
// doubles of device memory) for the coefficient reductions; allocates nothing.
// The fused 2D reverse applies: out-of-place outputs, the forward state and
// B^{n+1/2} given, a 2D grid and a one-coefficient Ampere stencil.
static bool adjoint_fused(const pic_grid* g, const pic_adjoint* adj) {
  const bool outs = adj->lEo[0] != nullptr;
  const bool next = adj->En[0] && adj->En[1] && adj->En[2] && adj->Bn[0] && adj->Bn[1] && adj->Bn[2];
  const bool half = next && adj->Bh[0] && adj->Bh[1] && adj->Bh[2];
  return outs && half && g->ndim == 2 && g->MB == 1 && adjoint_sweep2d_fits(g->mesh);
}

// Doubles of coefficient scratch the step needs.
static int64_t adjoint_partial_need(const pic_grid* g, const pic_adjoint* adj) {
  if (adjoint_fused(g, adj)) return adjoint_sweep2d_blocks(g->mesh) * 2 * PIC_MAX_M;
  return (int64_t)coef_partial_blocks(g->mesh) * PIC_MAX_M;
}

static int adjoint_body(pic_grid* g, const pic_adjoint* adj, const pic_particles* const* species,
                        pic_particles* const* lambda, int nspecies, int pusher, double* partial) {
  const Mesh& m = g->mesh;
  const double dt = g->dt;
  if (adjoint_fused(g, adj)) {
    void* En[3] = {g->E[0], g->E[1], g->E[2]};
    int rc = launch_adjoint_sweep2d(m, adj->lE, adj->lB, adj->lEo, adj->lBo, adj->En, adj->Bh, En, g->CE, g->ME,
                                    g->CB[0], dt, g->M, partial, adj->gCE, adj->gCB, g->stream);
    for (int s = 0; s < nspecies && !rc; ++s)
      rc = launch_adjoint_push(m, g->E, g->B, adj->lEo, adj->lBo, *species[s], *lambda[s], pusher, dt, g->stream);
    return rc;
  }
  void* none[3] = {nullptr, nullptr, nullptr};
  auto d = [](const void* p) { return (const double*)p; };
  void* const* lE = adj->lE;
  void* const* lB = adj->lB;
  // forward intermediates: E' = E^{n+1}, and B' = B^{n+1/2}, given by the
  // caller or recomputed as B^{n+1} + dt/2 curl_E E^{n+1} into the second
  // field set.  E^{n+1}, B^{n+1} come from the caller when given, else from a
  // forward sweep.
  const bool next = adj->En[0] && adj->En[1] && adj->En[2] && adj->Bn[0] && adj->Bn[1] && adj->Bn[2];
  const bool half = next && adj->Bh[0] && adj->Bh[1] && adj->Bh[2];
  void* hB[3] = {g->alt[3], g->alt[4], g->alt[5]};
  if (half)
    for (int c = 0; c < 3; ++c) {
      if ((uintptr_t)adj->Bh[c] & 15) return set_error(PIC_ESHAPE, "adjoint fields must be 16-byte aligned");
      for (int q = 0; q < 3; ++q)
        if (adj->Bh[c] == lE[q] || adj->Bh[c] == lB[q])
          return set_error(PIC_EINVAL, "the half-step field aliases a cotangent");
      hB[c] = const_cast<void*>(adj->Bh[c]);
    }
  void* const* aB = hB;
  void* nE[3] = {g->alt[0], g->alt[1], g->alt[2]};
  void* nB[3] = {g->alt[3], g->alt[4], g->alt[5]};
  int rc = PIC_OK;
  if (next) {
    for (int c = 0; c < 3; ++c) {
      nE[c] = const_cast<void*>(adj->En[c]);
      nB[c] = const_cast<void*>(adj->Bn[c]);
    }
  } else {
    rc = sweep_once(g, g->E, g->B, g->alt, g->alt + 3, 0);
  }
  void* const* aE = nE;
  if (!rc && !half) rc = launch_advance_b(g->prec, m, nE, nB, g->alt + 3, g->CE, g->ME, -0.5 * dt, g->stream);
  // third stage B'' = B' - dt/2 curl_E[C^E] E': dC^E from (lB, E')
  if (!rc) rc = launch_coef_grad(m, 0, d(lB[1]), d(aE[2]), d(lB[2]), d(aE[1]), 0.5 * dt / m.dx1, g->M, partial,
                                 adj->gCE, g->stream);
  if (!rc) rc = launch_advance_e(g->prec, m, lE, lB, none, g->CE, g->ME, -0.5 * dt, g->stream);
  // second stage E' = E + dt curl_B[C^B] B': dC^B from (lE', B')
  if (!rc) rc = launch_coef_grad(m, 1, d(lE[2]), d(aB[1]), d(lE[1]), d(aB[2]), dt / m.dx1, g->M, partial,
                                 adj->gCB, g->stream);
  if (!rc) rc = launch_advance_b(g->prec, m, lE, lB, lB, g->CB, g->MB, -dt, g->stream);
  // first stage B' = B - dt/2 curl_E[C^E] E: dC^E from (lB', E^n)
  if (!rc) rc = launch_coef_grad(m, 0, d(lB[1]), d(g->E[2]), d(lB[2]), d(g->E[1]), 0.5 * dt / m.dx1, g->M,
                                 partial, adj->gCE, g->stream);
  if (!rc) rc = launch_advance_e(g->prec, m, lE, lB, none, g->CE, g->ME, -0.5 * dt, g->stream);
  // particles: reverse of position update, push and gather at t^n
  for (int s = 0; s < nspecies && !rc; ++s)
    rc = launch_adjoint_push(m, g->E, g->B, lE, lB, *species[s], *lambda[s], pusher, dt, g->stream);
  if (!rc && adj->lEo[0]) {  // out of place requested on the in-place path: copy the result
    const size_t bytes = (size_t)g->n[0] * g->n[1] * g->n[2] * sizeof(double);
    for (int c = 0; c < 3 && !rc; ++c)
      if (hipMemcpyAsync(adj->lEo[c], lE[c], bytes, hipMemcpyDeviceToDevice, g->stream) != hipSuccess ||
          hipMemcpyAsync(adj->lBo[c], lB[c], bytes, hipMemcpyDeviceToDevice, g->stream) != hipSuccess)
        rc = set_error(PIC_EHIP, "adjoint output copy");
  }
  return rc;
}

int pic_adjoint_step(pic_grid* g, const pic_adjoint* adj, const pic_particles* const* species,
                     pic_particles* const* lambda, int nspecies, int pusher) {
  int rc = adjoint_args(g, adj, species, lambda, nspecies, pusher);
  if (rc) return rc;
  const int64_t need = adjoint_partial_need(g, adj);
  if (need > g->partial_cap) {
    (void)hipStreamSynchronize(g->stream);
    if (g->partial) (void)hipFree(g->partial);
    g->partial = nullptr;
    g->partial_cap = 0;
    if (hipMalloc((void**)&g->partial, (size_t)need * sizeof(double)) != hipSuccess)
      return set_error(PIC_ENOMEM, "cannot allocate the coefficient-gradient scratch");
    g->partial_cap = need;
  }
  return adjoint_body(g, adj, species, lambda, nspecies, pusher, g->partial);
}

int pic_adjoint_step_noalloc(pic_grid* g, const pic_adjoint* adj, const pic_particles* const* species,
                             pic_particles* const* lambda, int nspecies, int pusher) {
  int rc = adjoint_args(g, adj, species, lambda, nspecies, pusher);
  if (rc) return rc;
  const int64_t need = adjoint_partial_need(g, adj);
  if (need > kNoAllocDoubles)
    return set_error(PIC_EUNSUPPORTED,
                     "the allocation-free adjoint step needs %lld doubles of scratch for this mesh; it holds %lld "
                     "(use pic_adjoint_step)",
                     (long long)need, (long long)kNoAllocDoubles);
  if (!g->noalloc) return set_error(PIC_EHIP, "the adjoint scratch has no device address");
  return adjoint_body(g, adj, species, lambda, nspecies, pusher, g->noalloc);
}

int pic_set_shape(pic_grid* g, int order) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (order != 1 && order != 2) return set_error(PIC_EINVAL, "shape order must be 1 or 2");
  g->mesh.order = order;
  return PIC_OK;
}

int pic_set_sort_interval(pic_grid* g, int steps) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (steps < 1 || steps > 64) return set_error(PIC_EINVAL, "sort interval must be in 1..64");
  g->sort_every = steps;
  return PIC_OK;
}

int pic_sync(pic_grid* g) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  hipError_t e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "pending error");
  return PIC_OK;
}

int pic_check(pic_grid* g, const pic_particles* p) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (p) {
    int rc = check_particles(g, p);
    if (rc) return rc;
  }
  hipError_t e = hipMemsetAsync(g->d_flag, 0, sizeof(int), g->stream);
  if (e != hipSuccess) return hip_fail(e, "check: clear flag");
  int rc = launch_check(g->prec, g->mesh, g->E, g->B, p, g->d_flag, g->stream);
  if (rc) return rc;
  int flag = 0;
  e = hipMemcpyAsync(&flag, g->d_flag, sizeof(int), hipMemcpyDeviceToHost, g->stream);
  if (e != hipSuccess) return hip_fail(e, "check: read flag");
  e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) return hip_fail(e, "check: synchronize");
  int noconv = 0;
  e = hipMemcpyAsync(&noconv, g->d_noconv, sizeof(int), hipMemcpyDeviceToHost, g->stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->d_noconv, 0, sizeof(int), g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) return hip_fail(e, "check: read the convergence counter");
  if (flag & 1) return set_error(PIC_ENONFINITE, "non-finite field value");
  if (flag & 2) return set_error(PIC_ENONFINITE, "particle outside the box or non-finite momentum");
  if (noconv > 0)
    return set_error(PIC_ENOCONV,
                     "%d exact pushes since the last check ended their proper-time solve at the iteration cap (%d)",
                     noconv, g->mesh.exact_iters);
  return PIC_OK;
}

int pic_set_exact_iterations(pic_grid* g, int max_iter) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (max_iter < 1 || max_iter > 1000) return set_error(PIC_EINVAL, "iteration cap must be in 1..1000");
  g->mesh.exact_iters = max_iter;
  return PIC_OK;
}

int pic_set_deposit_mode(pic_grid* g, int mode) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (mode != PIC_DEPOSIT_ATOMIC && mode != PIC_DEPOSIT_DETERMINISTIC)
    return set_error(PIC_EINVAL, "bad deposit mode");
  g->deposit_mode = mode;
  return PIC_OK;
}

static int ensure_window_scratch(pic_grid* g, int64_t np) {
  const int64_t nb = window_blocks(np);
  if (nb > g->win_nb_cap) {
    (void)hipStreamSynchronize(g->stream);
    if (g->win_counts) (void)hipFree(g->win_counts);
    if (g->win_offs) (void)hipFree(g->win_offs);
    g->win_counts = nullptr;
    g->win_offs = nullptr;
    g->win_nb_cap = 0;
    if (hipMalloc((void**)&g->win_counts, (size_t)nb * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&g->win_offs, ((size_t)nb + 1) * sizeof(int64_t)) != hipSuccess)
      return set_error(PIC_ENOMEM, "cannot allocate the window compaction counters");
    g->win_nb_cap = nb;
  }
  if (np > g->win_cap) {
    (void)hipStreamSynchronize(g->stream);
    if (g->win_data) (void)hipFree(g->win_data);
    g->win_data = nullptr;
    g->win_cap = 0;
    if (hipMalloc((void**)&g->win_data, (size_t)np * 7 * sizeof(double)) != hipSuccess)
      return set_error(PIC_ENOMEM, "cannot allocate %lld particles of window scratch", (long long)np);
    g->win_cap = np;
  }
  return PIC_OK;
}

int pic_move_window(pic_grid* g, int64_t cells, pic_particles* const* species, int nspecies) {
  if (!g) return set_error(PIC_EINVAL, "grid is NULL");
  if (cells < 0 || cells >= g->n[0]) return set_error(PIC_EINVAL, "a window move needs 0 <= cells < n1");
  if (nspecies < 0 || (nspecies > 0 && !species)) return set_error(PIC_EINVAL, "bad species list");
  for (int s = 0; s < nspecies; ++s) {
    int rc = check_particles(g, species[s]);
    if (rc) return rc;
  }
  if (cells == 0) return PIC_OK;
  // scratch first: a failed allocation leaves the window unmoved
  int64_t npmax = 0;
  for (int s = 0; s < nspecies; ++s) npmax = std::max(npmax, species[s]->np);
  if (npmax > 0) {
    int rc = ensure_window_scratch(g, npmax);
    if (rc) return rc;
  }
  void* arrays[9];
  int na = 0;
  for (int c = 0; c < 3; ++c) arrays[na++] = g->E[c];
  for (int c = 0; c < 3; ++c) arrays[na++] = g->B[c];
  if (g->J[0] && g->J[1] && g->J[2])
    for (int c = 0; c < 3; ++c) arrays[na++] = g->J[c];
  const int64_t o = g->win_origin;
  int rc = launch_zero_columns(g->prec, g->mesh, arrays, na, o, cells, g->stream);
  if (rc) return rc;
  for (int s = 0; s < nspecies; ++s) {
    pic_particles* p = species[s];
    if (p->np == 0) continue;
    rc = launch_window_count(g->mesh, *p, o, cells, g->win_counts, g->win_offs, g->stream);
    if (rc) return rc;
    int64_t total = 0;
    hipError_t e = hipMemcpyAsync(&total, g->win_offs + window_blocks(p->np), sizeof(int64_t),
                                  hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "window survivor count");
    if (total == p->np) continue;
    pic_particles dst = *p;
    const int64_t cap = g->win_cap;
    for (int d = 0; d < 3; ++d) {
      dst.x[d] = g->win_data + d * cap;
      dst.u[d] = g->win_data + (3 + d) * cap;
    }
    dst.id = reinterpret_cast<int64_t*>(g->win_data + 6 * cap);
    rc = launch_window_scatter(g->mesh, *p, dst, o, cells, g->win_offs, g->stream);
    if (rc) return rc;
    const size_t bytes = (size_t)total * sizeof(double);
    for (int d = 0; d < 3 && e == hipSuccess; ++d) {
      if (p->x[d]) e = hipMemcpyAsync(p->x[d], dst.x[d], bytes, hipMemcpyDeviceToDevice, g->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(p->u[d], dst.u[d], bytes, hipMemcpyDeviceToDevice, g->stream);
    }
    if (e == hipSuccess && p->id) e = hipMemcpyAsync(p->id, dst.id, bytes, hipMemcpyDeviceToDevice, g->stream);
    if (e != hipSuccess) return hip_fail(e, "window compaction copy");
    p->np = total;
  }
  g->win_origin = (o + cells) % g->n[0];
  g->win_moved += cells;
  return PIC_OK;
}

int pic_window(const pic_grid* g, int64_t* origin, int64_t* moved) {
  if (!g || !origin || !moved) return set_error(PIC_EINVAL, "pic_window: NULL argument");
  *origin = g->win_origin;
  *moved = g->win_moved;
  return PIC_OK;
}

void pic_destroy(pic_grid* g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  for (int c = 0; c < 6; ++c)
    if (g->alt[c]) (void)hipFree(g->alt[c]);
  for (int d = 0; d < 3; ++d)
    if (g->xo[d]) (void)hipFree(g->xo[d]);
  for (SortState& st : g->sorts) free_sort(st);
  for (SortState& st : g->vsort_a) free_sort(st);
  for (SortState& st : g->vsort_b) free_sort(st);
  if (g->d_flag) (void)hipFree(g->d_flag);
  if (g->d_noconv) (void)hipFree(g->d_noconv);
  if (g->stage) (void)hipFree(g->stage);
  free_sort(g->dsort);
  if (g->partial) (void)hipFree(g->partial);
  if (g->corr_taps) (void)hipFree(g->corr_taps);
  if (g->Jc) (void)hipFree(g->Jc);
  if (g->win_counts) (void)hipFree(g->win_counts);
  if (g->win_offs) (void)hipFree(g->win_offs);
  if (g->win_data) (void)hipFree(g->win_data);
  delete g;
}

}  // extern "C"
