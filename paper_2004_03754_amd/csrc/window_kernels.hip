// Moving window along x1 (the single-particle runs of Sec. 4.1).
//
// Every kernel of the library is periodic along x1, so the window is a ring:
// moving it by s cells clears the s columns it leaves at the back, which are
// the columns that enter at the front, and moves the ring's origin.  Nothing
// else in the field arrays moves.  Particles keep their coordinates; those in
// the cleared columns leave the run by a stable compaction (count per block,
// one scan, scatter into scratch, copy back).
#include <hip/hip_runtime.h>

#include "yeepic_internal.h"

namespace yeepic {

namespace {

constexpr int kColBlock = 256;
constexpr int kWinBlock = 256;               // threads per compaction block
constexpr int kWinPer = 4;                   // particles per thread
constexpr int kWinChunk = kWinBlock * kWinPer;
constexpr int kScanBlock = 1024;

struct Columns {
  void* f[9];
};

// f[row][c] = 0 for c in [c0, c0 + s) mod n1, every row of every array
template <typename T>
__global__ void __launch_bounds__(kColBlock) zero_columns_kernel(Columns z, int64_t n1, int64_t rows, int64_t c0,
                                                                 int64_t s) {
  const int64_t i = (int64_t)blockIdx.x * kColBlock + threadIdx.x;
  if (i >= rows * s) return;
  const int64_t row = i / s;
  int64_t c = c0 + (i - row * s);
  if (c >= n1) c -= n1;
  static_cast<T*>(z.f[blockIdx.y])[row * n1 + c] = T(0);
}

// Graded damping layers at the two x1 ends of the window (the absorber of
// Cerjan, Kosloff, Kosloff and Reshef, 1985): in window cells [0, W) and
// [n1 - W, n1) every component is multiplied by exp(-sigma (d/W)^2), d the
// depth of its own staggered x1 position (window cell + 0 or 1/2) into the
// nearest strip.  Window cell s lives in array column (origin + s) mod n1.
struct Fields6 {
  void* f[6];
};

template <typename T>
__global__ void __launch_bounds__(kColBlock) damp_columns_kernel(Fields6 z, int64_t n1, int64_t rows, int64_t origin,
                                                                 int W, double sigma) {
  const int64_t ncol = 2 * (int64_t)W;
  const int64_t i = (int64_t)blockIdx.x * kColBlock + threadIdx.x;
  if (i >= rows * ncol) return;
  const int64_t row = i / ncol;
  const int64_t k = i - row * ncol;
  const int64_t s = k < W ? k : n1 - ncol + k;  // window cell
  int64_t c = origin + s;
  if (c >= n1) c -= n1;
  const int comp = blockIdx.y;                 // E1 E2 E3 B1 B2 B3
  const double off = (comp == 0 || comp == 4 || comp == 5) ? 0.5 : 0.0;
  const double pos = (double)s + off;
  double d = 0.0;
  if (pos < (double)W)
    d = (double)W - pos;
  else if (pos > (double)(n1 - W))
    d = pos - (double)(n1 - W);
  if (!(d > 0.0)) return;
  const double r = d / (double)W;
  T* f = static_cast<T*>(z.f[comp]) + row * n1 + c;
  *f = (T)((double)*f * exp(-sigma * (r * r)));
}

struct Leave {
  double inv_dx1;
  int64_t n1, origin, s;
};

// the particle's cell column lies among the s columns the window leaves
__device__ inline bool leaves(double x1, const Leave& w) {
  const double c = floor(x1 * w.inv_dx1);
  int64_t ci = c < 0.0 ? 0 : (c >= (double)w.n1 ? w.n1 - 1 : (int64_t)c);
  ci -= w.origin;
  if (ci < 0) ci += w.n1;
  return ci < w.s;
}

__global__ void __launch_bounds__(kWinBlock) window_count_kernel(const double* __restrict__ x1, int64_t np, Leave w,
                                                                 int* __restrict__ counts) {
  __shared__ int part[kWinBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kWinChunk;
  int keep = 0;
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) {
    const int64_t i = base + k * kWinBlock + threadIdx.x;
    const bool kept = i < np && !leaves(x1[i], w);
    keep += __popcll(__ballot(kept));
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = keep;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int q = 0; q < kWinBlock / 64; ++q) t += part[q];
    counts[blockIdx.x] = t;
  }
}

// one block: offs[b] = sum of counts[< b] (b <= nb), offs[nb] the total
__global__ void __launch_bounds__(kScanBlock) window_scan_kernel(const int* __restrict__ counts, int64_t nb,
                                                                 int64_t* __restrict__ offs) {
  __shared__ int64_t wsum[kScanBlock / 64];
  __shared__ int64_t carry_s;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < nb ? counts[i] : 0;
    int64_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int64_t before = carry_s;
    for (int q = 0; q < wv; ++q) before += wsum[q];
    if (i < nb) offs[i] = before + inc - v;
    __syncthreads();
    if (threadIdx.x == kScanBlock - 1) carry_s = before + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) offs[nb] = carry_s;
}

struct Soa {
  double* x[3];
  double* u[3];
  int64_t* id;
};

// survivors of block b go to dst[offs[b] + their rank in the block], in order
__global__ void __launch_bounds__(kWinBlock) window_scatter_kernel(Soa src, Soa dst, int64_t np, Leave w,
                                                                   const int64_t* __restrict__ offs) {
  __shared__ int wcnt[kWinPer][kWinBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kWinChunk;
  const unsigned long long below = (1ull << lane) - 1ull;
  bool kept[kWinPer];
  int rank[kWinPer];
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) {
    const int64_t i = base + k * kWinBlock + threadIdx.x;
    kept[k] = i < np && !leaves(src.x[0][i], w);
    const unsigned long long m = __ballot(kept[k]);
    rank[k] = __popcll(m & below);
    if (lane == 0) wcnt[k][wv] = __popcll(m);
  }
  __syncthreads();
  int64_t pre = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) {
    int before = 0;
    for (int q = 0; q < wv; ++q) before += wcnt[k][q];
    if (kept[k]) {
      const int64_t i = base + k * kWinBlock + threadIdx.x;
      const int64_t j = pre + before + rank[k];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (src.x[d]) dst.x[d][j] = src.x[d][i];
        dst.u[d][j] = src.u[d][i];
      }
      if (src.id) dst.id[j] = src.id[i];
    }
    for (int q = 0; q < kWinBlock / 64; ++q) pre += wcnt[k][q];
  }
}

int hip_status(const char* what) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

int launch_zero_columns(int prec, const Mesh& m, void* const* arrays, int narrays, int64_t c0, int64_t s,
                        void* stream) {
  if (narrays < 1 || narrays > 9 || s < 1 || s >= m.n1 || c0 < 0 || c0 >= m.n1)
    return set_error(PIC_EINVAL, "zero_columns: bad arguments");
  Columns z = {};
  for (int a = 0; a < narrays; ++a) z.f[a] = arrays[a];
  const int64_t rows = (int64_t)m.n2 * m.n3;
  const dim3 grid((unsigned)((rows * s + kColBlock - 1) / kColBlock), (unsigned)narrays);
  if (prec == PIC_FP64)
    hipLaunchKernelGGL(zero_columns_kernel<double>, grid, dim3(kColBlock), 0, (hipStream_t)stream, z,
                       (int64_t)m.n1, rows, c0, s);
  else
    hipLaunchKernelGGL(zero_columns_kernel<float>, grid, dim3(kColBlock), 0, (hipStream_t)stream, z,
                       (int64_t)m.n1, rows, c0, s);
  return hip_status("zero_columns_kernel");
}

int launch_damp_columns(int prec, const Mesh& m, void* const E[3], void* const B[3], int64_t origin, int W,
                        double sigma, void* stream) {
  if (W <= 0) return PIC_OK;
  Fields6 z;
  for (int c = 0; c < 3; ++c) {
    z.f[c] = E[c];
    z.f[3 + c] = B[c];
  }
  const int64_t rows = (int64_t)m.n2 * m.n3;
  const int64_t work = rows * 2 * W;
  const dim3 grid((unsigned)((work + kColBlock - 1) / kColBlock), 6);
  hipStream_t s = (hipStream_t)stream;
  if (prec == PIC_FP64)
    hipLaunchKernelGGL(damp_columns_kernel<double>, grid, dim3(kColBlock), 0, s, z, (int64_t)m.n1, rows, origin, W,
                       sigma);
  else
    hipLaunchKernelGGL(damp_columns_kernel<float>, grid, dim3(kColBlock), 0, s, z, (int64_t)m.n1, rows, origin, W,
                       sigma);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "absorber launch failed");
}

int64_t window_blocks(int64_t np) { return (np + kWinChunk - 1) / kWinChunk; }

int launch_window_count(const Mesh& m, const pic_particles& p, int64_t origin, int64_t s, int* counts,
                        int64_t* offs, void* stream) {
  const int64_t nb = window_blocks(p.np);
  const Leave w = {m.idx1, (int64_t)m.n1, origin, s};
  hipLaunchKernelGGL(window_count_kernel, dim3((unsigned)nb), dim3(kWinBlock), 0, (hipStream_t)stream, p.x[0],
                     p.np, w, counts);
  int rc = hip_status("window_count_kernel");
  if (rc) return rc;
  hipLaunchKernelGGL(window_scan_kernel, dim3(1), dim3(kScanBlock), 0, (hipStream_t)stream, counts, nb, offs);
  return hip_status("window_scan_kernel");
}

int launch_window_scatter(const Mesh& m, const pic_particles& src, const pic_particles& dst, int64_t origin,
                          int64_t s, const int64_t* offs, void* stream) {
  const int64_t nb = window_blocks(src.np);
  const Leave w = {m.idx1, (int64_t)m.n1, origin, s};
  Soa a = {}, b = {};
  for (int d = 0; d < 3; ++d) {
    a.x[d] = src.x[d];
    a.u[d] = src.u[d];
    b.x[d] = src.x[d] ? dst.x[d] : nullptr;
    b.u[d] = dst.u[d];
  }
  a.id = src.id;
  b.id = src.id ? dst.id : nullptr;
  hipLaunchKernelGGL(window_scatter_kernel, dim3((unsigned)nb), dim3(kWinBlock), 0, (hipStream_t)stream, a, b,
                     src.np, w, offs);
  return hip_status("window_scatter_kernel");
}

}  // namespace yeepic
