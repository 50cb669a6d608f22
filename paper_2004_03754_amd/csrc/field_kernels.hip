// Field kernels: Faraday half step, Ampere step, fused sweep (gfx950).
//
// Eq. (maxwell) with the App. B x1 operators
//   Faraday  d^E f_i = (1/dx1) sum_j C^E_j (f_{i+j}   - f_{i-j+1})
//   Ampere   d^B f_i = (1/dx1) sum_j C^B_j (f_{i+j-1} - f_{i-j})
// and Yee differences along x2, x3 (forward in Faraday, backward in Ampere).
// Arrays are [n3][n2][n1], x1 contiguous, periodic in every direction.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "yeepic_internal.h"

namespace yeepic {
namespace {

template <typename T, int W>
struct Taps {
  T a[W];
};

// ---------------------------------------------------------------------------
// Standalone steps.  A block of kSB threads owns kSB consecutive x1 cells of
// one (x2, x3) row; the two components under the wide x1 stencil are staged
// in LDS once (row segment plus W cells each side, coalesced), everything
// else is read directly.  In place is safe: a B update reads only E and its
// own B, and vice versa; the B step may also write a different array.
// ---------------------------------------------------------------------------
constexpr int kSB = 256;

template <typename T, int W>
__device__ __forceinline__ void stage_row(const T* __restrict__ f, T* __restrict__ s, size_t row, int i0, int n1) {
  for (int t = threadIdx.x; t < kSB + 2 * W; t += kSB) {
    int i = (i0 - W + t) % n1;
    i += (i < 0) ? n1 : 0;
    s[t] = f[row + i];
  }
}

// Bout <- Bin - h curl_E E (Bout may be Bin).  ``ce`` holds h C^E_j/dx1;
// hy = h/dx2, hz = h/dx3.
template <typename T, int W>
__global__ __launch_bounds__(kSB) void advance_b_kernel(const T* __restrict__ E1, const T* __restrict__ E2,
                                                        const T* __restrict__ E3, const T* Bi1, const T* Bi2,
                                                        const T* Bi3, T* Bo1, T* Bo2, T* Bo3, Mesh m,
                                                        Taps<T, W> ce, T hy, T hz) {
  __shared__ T s2[kSB + 2 * W], s3[kSB + 2 * W];
  const int i0 = blockIdx.x * kSB;
  const int i = i0 + (int)threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  const size_t row = ((size_t)k * m.n2 + j) * m.n1;
  stage_row<T, W>(E2, s2, row, i0, m.n1);
  stage_row<T, W>(E3, s3, row, i0, m.n1);
  __syncthreads();
  if (i >= m.n1) return;
  const int jp = (j + 1 == m.n2) ? 0 : j + 1;
  const int kp = (k + 1 == m.n3) ? 0 : k + 1;
  const size_t rowjp = ((size_t)k * m.n2 + jp) * m.n1;
  const size_t rowkp = ((size_t)kp * m.n2 + j) * m.n1;
  const size_t c = row + i;
  const int t = threadIdx.x + W;  // LDS slot of cell i
  T d1E3 = 0, d1E2 = 0;
#pragma unroll
  for (int q = 1; q <= W; ++q) {
    d1E3 += ce.a[q - 1] * (s3[t + q] - s3[t - q + 1]);
    d1E2 += ce.a[q - 1] * (s2[t + q] - s2[t - q + 1]);
  }
  const T e1 = E1[c], e2 = s2[t], e3 = s3[t];
  const T b1 = Bi1[c], b2 = Bi2[c], b3 = Bi3[c];
  Bo1[c] = b1 - (hy * (E3[rowjp + i] - e3) - hz * (E2[rowkp + i] - e2));
  Bo2[c] = b2 - (hz * (E1[rowkp + i] - e1) - d1E3);
  Bo3[c] = b3 - (d1E2 - hy * (E1[rowjp + i] - e1));
}

// E <- E + dt (curl_B B - J).  ``cb`` holds dt C^B_j/dx1; ty = dt/dx2,
// tz = dt/dx3; J may be null.
template <typename T, int W>
__global__ __launch_bounds__(kSB) void advance_e_kernel(T* __restrict__ E1, T* __restrict__ E2, T* __restrict__ E3,
                                                        const T* __restrict__ B1, const T* __restrict__ B2,
                                                        const T* __restrict__ B3, const T* __restrict__ J1,
                                                        const T* __restrict__ J2, const T* __restrict__ J3,
                                                        Mesh m, Taps<T, W> cb, T ty, T tz, T dt) {
  __shared__ T s2[kSB + 2 * W], s3[kSB + 2 * W];
  const int i0 = blockIdx.x * kSB;
  const int i = i0 + (int)threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  const size_t row = ((size_t)k * m.n2 + j) * m.n1;
  stage_row<T, W>(B2, s2, row, i0, m.n1);
  stage_row<T, W>(B3, s3, row, i0, m.n1);
  __syncthreads();
  if (i >= m.n1) return;
  const int jm = (j == 0) ? m.n2 - 1 : j - 1;
  const int km = (k == 0) ? m.n3 - 1 : k - 1;
  const size_t rowjm = ((size_t)k * m.n2 + jm) * m.n1;
  const size_t rowkm = ((size_t)km * m.n2 + j) * m.n1;
  const size_t c = row + i;
  const int t = threadIdx.x + W;
  T d1B3 = 0, d1B2 = 0;
#pragma unroll
  for (int q = 1; q <= W; ++q) {
    d1B3 += cb.a[q - 1] * (s3[t + q - 1] - s3[t - q]);
    d1B2 += cb.a[q - 1] * (s2[t + q - 1] - s2[t - q]);
  }
  const T b1 = B1[c], b2 = s2[t], b3 = s3[t];
  T c1 = ty * (b3 - B3[rowjm + i]) - tz * (b2 - B2[rowkm + i]);
  T c2 = tz * (b1 - B1[rowkm + i]) - d1B3;
  T c3 = d1B2 - ty * (b1 - B1[rowjm + i]);
  if (J1) {
    c1 -= dt * J1[c];
    c2 -= dt * J2[c];
    c3 -= dt * J3[c];
  }
  E1[c] += c1;
  E2[c] += c2;
  E3[c] += c3;
}

template <typename T, int W>
Taps<T, W> scaled_taps(const double* C, int M, double scale) {
  Taps<T, W> t;
  for (int q = 0; q < W; ++q) t.a[q] = (T)(q < M ? C[q] * scale : 0.0);
  return t;
}

dim3 cell_grid(const Mesh& m, int bx) { return dim3((m.n1 + bx - 1) / bx, m.n2, m.n3); }

template <typename T, int W>
int run_advance_b(const Mesh& m, void* const E[3], void* const B[3], void* const Bo[3], const double* CE, int ME,
                  double h, hipStream_t s) {
  const int bx = kSB;
  hipLaunchKernelGGL((advance_b_kernel<T, W>), cell_grid(m, bx), dim3(bx), 0, s, (const T*)E[0], (const T*)E[1],
                     (const T*)E[2], (const T*)B[0], (const T*)B[1], (const T*)B[2], (T*)Bo[0], (T*)Bo[1],
                     (T*)Bo[2], m, scaled_taps<T, W>(CE, ME, h / m.dx1),
                     (T)(h / m.dx2), (T)(m.ndim == 3 ? h / m.dx3 : 0.0));
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "advance_b launch failed");
}

template <typename T, int W>
int run_advance_e(const Mesh& m, void* const E[3], void* const B[3], void* const J[3], const double* CB, int MB,
                  double dt, hipStream_t s) {
  const int bx = kSB;
  hipLaunchKernelGGL((advance_e_kernel<T, W>), cell_grid(m, bx), dim3(bx), 0, s, (T*)E[0], (T*)E[1], (T*)E[2],
                     (const T*)B[0], (const T*)B[1], (const T*)B[2], (const T*)(J ? J[0] : nullptr),
                     (const T*)(J ? J[1] : nullptr), (const T*)(J ? J[2] : nullptr), m,
                     scaled_taps<T, W>(CB, MB, dt / m.dx1), (T)(dt / m.dx2),
                     (T)(m.ndim == 3 ? dt / m.dx3 : 0.0), (T)dt);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "advance_e launch failed");
}

template <typename T>
int dispatch_b(const Mesh& m, void* const E[3], void* const B[3], void* const Bo[3], const double* CE, int ME, double h,
               hipStream_t s) {
  switch (round_width(ME)) {
    case 1: return run_advance_b<T, 1>(m, E, B, Bo, CE, ME, h, s);
    case 2: return run_advance_b<T, 2>(m, E, B, Bo, CE, ME, h, s);
    case 4: return run_advance_b<T, 4>(m, E, B, Bo, CE, ME, h, s);
    case 8: return run_advance_b<T, 8>(m, E, B, Bo, CE, ME, h, s);
    default: return run_advance_b<T, 16>(m, E, B, Bo, CE, ME, h, s);
  }
}

template <typename T>
int dispatch_e(const Mesh& m, void* const E[3], void* const B[3], void* const J[3], const double* CB, int MB,
               double dt, hipStream_t s) {
  switch (round_width(MB)) {
    case 1: return run_advance_e<T, 1>(m, E, B, J, CB, MB, dt, s);
    case 2: return run_advance_e<T, 2>(m, E, B, J, CB, MB, dt, s);
    case 4: return run_advance_e<T, 4>(m, E, B, J, CB, MB, dt, s);
    case 8: return run_advance_e<T, 8>(m, E, B, J, CB, MB, dt, s);
    default: return run_advance_e<T, 16>(m, E, B, J, CB, MB, dt, s);
  }
}

// ---------------------------------------------------------------------------
// Fused sweep: B half step, E step, B half step in one pass.
//
// A workgroup owns a TX x TY tile of (x1, x2) columns and marches along x3
// over KZ planes.  Three plane-sized LDS buffer pairs hold, for the planes in
// flight, E^n (stage-1 input), B^{n+1/2} (stage-2 input) and E^{n+1}
// (stage-3 input); each is stored over the x1/x2 extent its consumer needs,
// so the wide Faraday stencil never leaves LDS.  Per plane kk:
//   stage 1: B^{n+1/2}(kk+1) = B^n - (dt/2) curl_E E^n       (LDS E^n kk+1, kk+2)
//   stage 2: E^{n+1}(kk+1)   = E^n + dt (curl_B B^{n+1/2} - J)  (LDS B^{n+1/2} kk, kk+1)
//   stage 3: B^{n+1}(kk)     = B^{n+1/2} - (dt/2) curl_E E^{n+1}  (LDS E^{n+1} kk, kk+1)
// The march starts two planes early to fill the pipeline.  Tile-relative
// x1 extents (left offset, width) of the three buffers:
//   E^n        HLE = 2ME+MB-2, PXE = TX+4ME+2MB-3, rows j-1 .. j+TY+1
//   B^{n+1/2}  HLB = ME+MB-1,  PXB = TX+2ME+2MB-2, rows j-1 .. j+TY
//   E^{n+1}    HLF = ME-1,     PXF = TX+2ME-1,     rows j   .. j+TY
// ---------------------------------------------------------------------------
template <typename T, int ME, int MB, int TX, int TY>
struct SweepGeom {
  // R consecutive x1 outputs per thread in the wide stages, read as 16-byte
  // LDS vectors; NC vectors cover one R-output window of the 2ME-tap stencil
  static constexpr int R = 16 / (int)sizeof(T);
  static constexpr int NC = (R + 2 * ME - 1 + R - 1) / R;
  static constexpr int rup(int v) { return (v + R - 1) / R * R; }
  static constexpr int mx(int a, int b) { return a > b ? a : b; }
  // left halos: HLE is a multiple of R (16-byte aligned global rows) and
  // HLB = HLE - ME + 1, so every stage-1 window starts on a vector boundary
  static constexpr int HLB = rup(ME + MB - 1 + ME - 1) - (ME - 1);
  static constexpr int HLE = HLB + ME - 1;
  static constexpr int HLF = ME - 1;
  static constexpr int PYE = TY + 3, PYB = TY + 2, PYF = TY + 1;
  static constexpr int PXB = rup(HLB + TX + ME + MB - 1);
  static constexpr int PXE = rup(mx(PXB - R + R * NC, HLE + TX + 2 * ME + MB - 1));
  static constexpr int PXF = rup(mx(TX - R + R * NC, TX + 2 * ME - 1));
  static constexpr int SE = PXE * PYE, SB = PXB * PYB, SF = PXF * PYF;  // one component, one plane
  static constexpr int GB = PXB / R, G3 = TX / R;                         // vector groups per row
  static constexpr int VE = PXE / R;                                      // vectors per E row
  static constexpr size_t lds_bytes = sizeof(T) * 2 * 3 * (size_t)(SE + SB + SF);
};

template <typename T, int ME, int MB>
struct SweepCoef {
  T ae[ME];  // (dt/2) C^E_q / dx1
  T ab[MB];  // dt C^B_q / dx1
  T hy, hz;  // (dt/2)/dx2, (dt/2)/dx3 (hz = 0 in 2D)
  T ty, tz;  // dt/dx2, dt/dx3
  T dt;
};

// 16-byte native vectors (clang ext_vector_type keeps arrays of them in
// registers, unlike the struct-based HIP vector types)
typedef double v2f64 __attribute__((ext_vector_type(2)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
template <typename T>
struct Vec16 {
  using type = typename std::conditional<sizeof(T) == 8, v2f64, v4f32>::type;
};

// load NC 16-byte vectors starting at an aligned LDS index
template <typename T, int NC, int R>
__device__ __forceinline__ void load_window(const T* __restrict__ src, T (&w)[NC * R]) {
  using V = typename Vec16<T>::type;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const V v = *reinterpret_cast<const V*>(src + c * R);
#pragma unroll
    for (int e = 0; e < R; ++e) w[c * R + e] = v[e];
  }
}

// R consecutive values starting OFF elements after an aligned LDS index,
// read as one or two aligned 16-byte vectors (lanes then touch consecutive
// 16-byte words: no bank conflicts)
template <typename T, int R, int OFF>
__device__ __forceinline__ void load_run(const T* __restrict__ aligned, T (&out)[R]) {
  using V = typename Vec16<T>::type;
  constexpr int q0 = OFF / R, rem = OFF % R;
  const V v0 = *reinterpret_cast<const V*>(aligned + q0 * R);
  if constexpr (rem == 0) {
#pragma unroll
    for (int e = 0; e < R; ++e) out[e] = v0[e];
  } else {
    const V v1 = *reinterpret_cast<const V*>(aligned + (q0 + 1) * R);
#pragma unroll
    for (int e = 0; e < R; ++e) out[e] = (e + rem < R) ? v0[e + rem] : v1[e + rem - R];
  }
}

template <typename T, int R>
__device__ __forceinline__ void store_vec(T* __restrict__ aligned, const T (&in)[R]) {
  using V = typename Vec16<T>::type;
  V v;
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = in[e];
  *reinterpret_cast<V*>(aligned) = v;
}

// Faraday-form tap sum for output u of a window whose index 0 is the
// output block start: sum_q a_q (w[u+ME-1+q] - w[u+ME-q])
template <typename T, int ME, int NW>
__device__ __forceinline__ T faraday_taps(const T (&w)[NW], const T (&a)[ME], int u) {
  T acc = 0;
#pragma unroll
  for (int q = 1; q <= ME; ++q) acc += a[q - 1] * (w[u + ME - 1 + q] - w[u + ME - q]);
  return acc;
}

template <typename T, int ME, int MB, int TX, int TY, int NT, bool HAS_J>
__global__ __launch_bounds__(NT) void sweep_kernel(const T* __restrict__ iE1, const T* __restrict__ iE2,
                                                   const T* __restrict__ iE3, const T* __restrict__ iB1,
                                                   const T* __restrict__ iB2, const T* __restrict__ iB3,
                                                   const T* __restrict__ J1, const T* __restrict__ J2,
                                                   const T* __restrict__ J3, T* __restrict__ oE1,
                                                   T* __restrict__ oE2, T* __restrict__ oE3, T* __restrict__ oB1,
                                                   T* __restrict__ oB2, T* __restrict__ oB3, Mesh m, int KZ,
                                                   int tiles_x, int tiles, SweepCoef<T, ME, MB> c) {
  using G = SweepGeom<T, ME, MB, TX, TY>;
  constexpr int R = G::R, NC = G::NC;
  // per-thread work slots of each phase (fixed for the whole march)
  constexpr int NLE = (3 * G::PYE * G::VE + NT - 1) / NT;
  constexpr int NG1 = G::PYB * G::GB;
  constexpr int NS1 = (NG1 + NT - 1) / NT;
  constexpr int NS2 = (G::SF + NT - 1) / NT;
  constexpr int NG3 = TY * G::G3;
  constexpr int NS3 = (NG3 + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  T* sE = lds;                 // [plane parity][component] x SE
  T* sB = sE + 2 * 3 * G::SE;  // [plane parity][component] x SB
  T* sF = sB + 2 * 3 * G::SB;  // [plane parity][component] x SF

  const int tid = threadIdx.x;
  // XCD-aware tile order: consecutive workgroup ids go round-robin to the 8
  // XCDs, so give each XCD a contiguous block of tiles (halo reuse in its L2)
  int tile = blockIdx.x;
  if (tiles % 8 == 0) tile = (tile % 8) * (tiles / 8) + tile / 8;
  const int i0 = (tile % tiles_x) * TX;
  const int j0 = (tile / tiles_x) * TY;
  const int k0 = blockIdx.y * KZ;
  const int kend = min(k0 + KZ, m.n3);
  const size_t plane_sz = (size_t)m.n1 * m.n2;
  auto gi = [&](int rel) {
    int i = (i0 + rel) % m.n1;
    return i < 0 ? i + m.n1 : i;
  };
  auto gj = [&](int rel) {
    int j = (j0 + rel) % m.n2;
    return j < 0 ? j + m.n2 : j;
  };
  auto poff = [&](int k) {
    k %= m.n3;
    return (size_t)(k < 0 ? k + m.n3 : k) * plane_sz;
  };

  // ---- slot tables (all modulo arithmetic happens here, once) ----
  using V = typename Vec16<T>::type;
  constexpr int NVE = 3 * G::PYE * G::VE;  // 16-byte vectors per E^n plane
  // slot s of this thread: component le_c[s] (-1: idle), vector offset
  // le_g[s] in the component's plane, LDS element index le_d[s]
  int le_c[NLE], le_g[NLE], le_d[NLE];
#pragma unroll
  for (int s = 0; s < NLE; ++s) {
    const int p = tid + s * NT;
    const int comp = p / (G::PYE * G::VE);
    const int q = p - comp * (G::PYE * G::VE);
    const int r = q / G::VE;
    const int x = (q - r * G::VE) * R;
    le_c[s] = p < NVE ? comp : -1;
    le_d[s] = comp * G::SE + r * G::PXE + x;
    le_g[s] = p < NVE ? (gj(r - 1) * m.n1 + gi(x - G::HLE)) / R : 0;
  }
  const V* vE1 = reinterpret_cast<const V*>(iE1);
  const V* vE2 = reinterpret_cast<const V*>(iE2);
  const V* vE3 = reinterpret_cast<const V*>(iE3);
  // stage 1: R-output groups over the B extent
  int s1_w[NS1], s1_b[NS1], s1_row[NS1], s1_col[NS1];
#pragma unroll
  for (int s = 0; s < NS1; ++s) {
    const int g = tid + s * NT;
    const int r = g / G::GB, x = (g - r * G::GB) * R;
    s1_w[s] = r * G::PXE + x;  // window start (aligned)
    s1_b[s] = r * G::PXB + x;
    s1_row[s] = g < NG1 ? gj(r - 1) * m.n1 : 0;
    s1_col[s] = g < NG1 ? gi(x - G::HLB) : 0;
  }
  int s2_cb[NS2], s2_ce[NS2], s2_g[NS2];
  bool s2_out[NS2];
#pragma unroll
  for (int s = 0; s < NS2; ++s) {
    const int p = tid + s * NT;
    const int r = p / G::PXF, x = p - (p / G::PXF) * G::PXF;
    s2_cb[s] = (r + 1) * G::PXB + x + (G::HLB - G::HLF);
    s2_ce[s] = (r + 1) * G::PXE + x + (G::HLE - G::HLF);
    s2_g[s] = p < G::SF ? gj(r) * m.n1 + gi(x - G::HLF) : 0;
    const int xr = x - G::HLF;
    s2_out[s] = p < G::SF && xr >= 0 && xr < TX && r < TY && i0 + xr < m.n1 && j0 + r < m.n2;
  }
  // stage 3: R-output groups over the output tile
  int s3_w[NS3], s3_b[NS3], s3_g[NS3], s3_n[NS3];
#pragma unroll
  for (int s = 0; s < NS3; ++s) {
    const int g = tid + s * NT;
    const int r = g / G::G3, x = (g - r * G::G3) * R;
    s3_w[s] = r * G::PXF + x;
    s3_b[s] = (r + 1) * G::PXB + x;  // aligned; the B position is HLB further
    const bool rowok = g < NG3 && j0 + r < m.n2;
    const int nx = m.n1 - (i0 + x);
    s3_n[s] = rowok ? (nx < 0 ? 0 : (nx > R ? R : nx)) : 0;  // valid outputs in the group
    s3_g[s] = s3_n[s] > 0 ? (j0 + r) * m.n1 + (i0 + x) : 0;
  }

  // ---- prologue: E^n planes k0-1, k0 into LDS; B^n and J of plane k0-1 ----
#define YP_LOAD_PLANE(k)                                                        \
  {                                                                             \
    const size_t voff = poff(k) / R; /* plane offsets are multiples of R */     \
    _Pragma("unroll") for (int s = 0; s < NLE; ++s) {                           \
      const V* src = le_c[s] == 0 ? vE1 : (le_c[s] == 1 ? vE2 : vE3);           \
      pfE[s] = src[voff + le_g[s]]; /* idle slots read offset 0 */            \
    }                                                                           \
  }
#define YP_STORE_PLANE(k)                                                       \
  {                                                                             \
    T* dst = sE + ((k) & 1) * 3 * G::SE;                                        \
    _Pragma("unroll") for (int s = 0; s < NLE; ++s) if (le_c[s] >= 0)           \
        *reinterpret_cast<V*>(dst + le_d[s]) = pfE[s];                          \
  }
  V pfE[NLE];
  YP_LOAD_PLANE(k0 - 1);
  YP_STORE_PLANE(k0 - 1);
  YP_LOAD_PLANE(k0);
  YP_STORE_PLANE(k0);
  T curB[NS1][R][3], nxtB[NS1][R][3];
  constexpr int NJ = HAS_J ? NS2 : 1;  // current prefetch only when there is a current
  T curJ[NJ][3], nxtJ[NJ][3];
  // Every thread issues every global load of the march (idle slots read the
  // plane's first cells, planes past the march wrap): with no load under a
  // branch, the compiler's wait counts stay exact (see sweep_yee_kernel).
  auto load_B = [&](int k, T (&dst)[NS1][R][3]) {
    const size_t off = poff(k);
#pragma unroll
    for (int s = 0; s < NS1; ++s) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        int col = s1_col[s] + u;
        col -= col >= m.n1 ? m.n1 : 0;
        const size_t g = off + s1_row[s] + col;
        dst[s][u][0] = iB1[g];
        dst[s][u][1] = iB2[g];
        dst[s][u][2] = iB3[g];
      }
    }
  };
  auto load_J = [&](int k, T (&dst)[NJ][3]) {
    const size_t off = poff(k);
#pragma unroll
    for (int s = 0; s < NJ; ++s) {
      dst[s][0] = dst[s][1] = dst[s][2] = 0;
      if (HAS_J) {
        dst[s][0] = J1[off + s2_g[s]];
        dst[s][1] = J2[off + s2_g[s]];
        dst[s][2] = J3[off + s2_g[s]];
      }
    }
  };
  load_B(k0 - 1, curB);
  load_J(k0 - 1, curJ);
  __syncthreads();

  for (int kk = k0 - 2; kk < kend; ++kk) {
    const int ka = kk + 1;  // plane of stages 1 and 2
    const bool more = kk + 1 < kend;
    // prefetch for the next plane: E^n(kk+3) -> LDS at the end of this
    // iteration; B^n, J of plane ka+1 for the next stages 1 and 2
    YP_LOAD_PLANE(kk + 3);
    load_B(ka + 1, nxtB);
    load_J(ka + 1, nxtJ);
    // ---- stage 1: B^{n+1/2}(ka) ----
    {
      const T* e1 = sE + (ka & 1) * 3 * G::SE;
      const T* e2 = e1 + G::SE;
      const T* e3 = e2 + G::SE;
      const T* n1 = sE + ((ka + 1) & 1) * 3 * G::SE;
      const T* n2 = n1 + G::SE;
      T* b1 = sB + (ka & 1) * 3 * G::SB;
      T* b2 = b1 + G::SB;
      T* b3 = b2 + G::SB;
#pragma unroll
      for (int s = 0; s < NS1; ++s) {
        if (tid + s * NT >= NG1) continue;
        // one component's window at a time keeps register pressure down
        T dE2[R], dE3[R], e2w[R], e3w[R];
        {
          T w[NC * R];
          load_window<T, NC, R>(e2 + s1_w[s], w);
#pragma unroll
          for (int u = 0; u < R; ++u) {
            dE2[u] = faraday_taps<T, ME>(w, c.ae, u);
            e2w[u] = w[u + ME - 1];
          }
        }
        {
          T w[NC * R];
          load_window<T, NC, R>(e3 + s1_w[s], w);
#pragma unroll
          for (int u = 0; u < R; ++u) {
            dE3[u] = faraday_taps<T, ME>(w, c.ae, u);
            e3w[u] = w[u + ME - 1];
          }
        }
        // the B positions' own E values (index window start + ME - 1)
        T e1c[R], e1n[R], e3n[R], n1c[R], n2c[R];
        load_run<T, R, ME - 1>(e1 + s1_w[s], e1c);
        load_run<T, R, ME - 1>(e1 + s1_w[s] + G::PXE, e1n);
        load_run<T, R, ME - 1>(e3 + s1_w[s] + G::PXE, e3n);
        load_run<T, R, ME - 1>(n1 + s1_w[s], n1c);
        load_run<T, R, ME - 1>(n2 + s1_w[s], n2c);
        T o1[R], o2[R], o3[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
          o1[u] = curB[s][u][0] - (c.hy * (e3n[u] - e3w[u]) - c.hz * (n2c[u] - e2w[u]));
          o2[u] = curB[s][u][1] - (c.hz * (n1c[u] - e1c[u]) - dE3[u]);
          o3[u] = curB[s][u][2] - (dE2[u] - c.hy * (e1n[u] - e1c[u]));
        }
        store_vec<T, R>(b1 + s1_b[s], o1);
        store_vec<T, R>(b2 + s1_b[s], o2);
        store_vec<T, R>(b3 + s1_b[s], o3);
      }
    }
    __syncthreads();
    // ---- stage 2: E^{n+1}(ka) ----
    {
      const T* b1 = sB + (ka & 1) * 3 * G::SB;
      const T* b2 = b1 + G::SB;
      const T* b3 = b2 + G::SB;
      const T* p1 = sB + ((ka - 1) & 1) * 3 * G::SB;
      const T* p2 = p1 + G::SB;
      const T* e1 = sE + (ka & 1) * 3 * G::SE;
      const T* e2 = e1 + G::SE;
      const T* e3 = e2 + G::SE;
      T* f1 = sF + (ka & 1) * 3 * G::SF;
      T* f2 = f1 + G::SF;
      T* f3 = f2 + G::SF;
      const bool out_plane = ka >= k0 && ka < kend;
      const size_t off = poff(ka);
#pragma unroll
      for (int s = 0; s < NS2; ++s) {
        const int p = tid + s * NT;
        if (p >= G::SF) continue;
        const int cb = s2_cb[s], ce = s2_ce[s];
        T dB3 = 0, dB2 = 0;
#pragma unroll
        for (int q = 1; q <= MB; ++q) {
          dB3 += c.ab[q - 1] * (b3[cb + q - 1] - b3[cb - q]);
          dB2 += c.ab[q - 1] * (b2[cb + q - 1] - b2[cb - q]);
        }
        const T b1c = b1[cb], b2c = b2[cb], b3c = b3[cb];
        T c1 = c.ty * (b3c - b3[cb - G::PXB]) - c.tz * (b2c - p2[cb]);
        T c2 = c.tz * (b1c - p1[cb]) - dB3;
        T c3 = dB2 - c.ty * (b1c - b1[cb - G::PXB]);
        if constexpr (HAS_J) {
          c1 -= c.dt * curJ[s][0];
          c2 -= c.dt * curJ[s][1];
          c3 -= c.dt * curJ[s][2];
        }
        const T v1 = e1[ce] + c1, v2 = e2[ce] + c2, v3 = e3[ce] + c3;
        f1[p] = v1;
        f2[p] = v2;
        f3[p] = v3;
        if (out_plane && s2_out[s]) {
          const size_t g = off + s2_g[s];
          oE1[g] = v1;
          oE2[g] = v2;
          oE3[g] = v3;
        }
      }
    }
    __syncthreads();
    // ---- stage 3: B^{n+1}(kk) on the output tile ----
    if (kk >= k0) {
      const T* f1 = sF + (kk & 1) * 3 * G::SF;
      const T* f2 = f1 + G::SF;
      const T* f3 = f2 + G::SF;
      const T* g1 = sF + ((kk + 1) & 1) * 3 * G::SF;
      const T* g2 = g1 + G::SF;
      const T* b1 = sB + (kk & 1) * 3 * G::SB;
      const T* b2 = b1 + G::SB;
      const T* b3 = b2 + G::SB;
      const size_t off = poff(kk);
#pragma unroll
      for (int s = 0; s < NS3; ++s) {
        if (s3_n[s] == 0) continue;
        T dF2[R], dF3[R], f2w[R], f3w[R];
        {
          T w[NC * R];
          load_window<T, NC, R>(f2 + s3_w[s], w);
#pragma unroll
          for (int u = 0; u < R; ++u) {
            dF2[u] = faraday_taps<T, ME>(w, c.ae, u);
            f2w[u] = w[u + ME - 1];
          }
        }
        {
          T w[NC * R];
          load_window<T, NC, R>(f3 + s3_w[s], w);
#pragma unroll
          for (int u = 0; u < R; ++u) {
            dF3[u] = faraday_taps<T, ME>(w, c.ae, u);
            f3w[u] = w[u + ME - 1];
          }
        }
        T f1c[R], f1n[R], f3n[R], g1c[R], g2c[R], hb1[R], hb2[R], hb3[R];
        load_run<T, R, ME - 1>(f1 + s3_w[s], f1c);
        load_run<T, R, ME - 1>(f1 + s3_w[s] + G::PXF, f1n);
        load_run<T, R, ME - 1>(f3 + s3_w[s] + G::PXF, f3n);
        load_run<T, R, ME - 1>(g1 + s3_w[s], g1c);
        load_run<T, R, ME - 1>(g2 + s3_w[s], g2c);
        load_run<T, R, G::HLB>(b1 + s3_b[s], hb1);
        load_run<T, R, G::HLB>(b2 + s3_b[s], hb2);
        load_run<T, R, G::HLB>(b3 + s3_b[s], hb3);
        T o1[R], o2[R], o3[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
          o1[u] = hb1[u] - (c.hy * (f3n[u] - f3w[u]) - c.hz * (g2c[u] - f2w[u]));
          o2[u] = hb2[u] - (c.hz * (g1c[u] - f1c[u]) - dF3[u]);
          o3[u] = hb3[u] - (dF2[u] - c.hy * (f1n[u] - f1c[u]));
        }
        const size_t g = off + s3_g[s];
        if (s3_n[s] == R) {
          store_vec<T, R>(oB1 + g, o1);
          store_vec<T, R>(oB2 + g, o2);
          store_vec<T, R>(oB3 + g, o3);
        } else {
#pragma unroll
          for (int u = 0; u < R; ++u)
            if (u < s3_n[s]) {
              oB1[g + u] = o1[u];
              oB2[g + u] = o2[u];
              oB3[g + u] = o3[u];
            }
        }
      }
    }
    if (more) {
      YP_STORE_PLANE(kk + 3);
#pragma unroll
      for (int s = 0; s < NS1; ++s)
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
          for (int q = 0; q < 3; ++q) curB[s][u][q] = nxtB[s][u][q];
#pragma unroll
      for (int s = 0; s < NJ; ++s)
#pragma unroll
        for (int q = 0; q < 3; ++q) curJ[s][q] = nxtJ[s][q];
    }
    __syncthreads();
  }
#undef YP_LOAD_PLANE
#undef YP_STORE_PLANE
}

// ---------------------------------------------------------------------------
// Fused sweep for the Yee Ampere operator (C^B = e1, which the App. B design
// gives at dt = dx1/2): the same three stages as sweep_kernel, in a layout
// that holds TY = 8 rows of cells per tile.
//
// Only one plane of each stage's input is kept in LDS.  What a stage needs
// from a neighbouring x3 plane it needs at its own positions, and the thread
// that owns those positions holds it in registers:
//   * stage 1 at plane ka needs E1, E2 of plane ka+1: loaded from memory one
//     plane ahead by the same thread;
//   * stage 2 at ka needs B^{n+1/2}(ka-1), and stage 3 at ka-1 needs it as
//     well: the thread re-reads its own B^{n+1/2} from LDS after each plane;
//   * stage 3 at ka-1 reads E^{n+1}(ka-1) across the tile and E^{n+1}(ka) at
//     its own positions: E^{n+1} is double-buffered.
// A task is RW = 4 consecutive x1 outputs of one row, so the 2ME-tap
// Faraday windows are read once per four outputs.  The same thread owns the
// same task in every stage.  FP64 tasks are laid out 8 groups x 2 rows per 16
// lanes, with row pitches of 2 mod 4 elements: the 16-byte LDS reads of 16
// lanes then fall on 16 distinct bank quads.
// Per plane ka (stage 3 on plane ka-1):
//   E(ka+1) -> registers | stage 1: B^{n+1/2}(ka) -> LDS | B^n(ka+1), E1/E2(ka+2)
//   own -> registers | barrier | stage 2: E^{n+1}(ka) -> LDS, memory | stage 3:
//   B^{n+1}(ka-1) -> memory | barrier | E(ka+1) -> LDS | barrier.
// Extents (columns from the tile's first column, rows from its first row):
//   B^{n+1/2}: columns [-HB, TX+HB), rows -1..TY
//   E^{n+1}:   columns [-HB, TX+HB), rows  0..TY
//   E1:        columns [-HB, TX+HB), rows -1..TY+1
//   E2:        columns [-2HB, TX+2HB), rows -1..TY
//   E3:        columns [-2HB, TX+2HB), rows -1..TY+1
// ---------------------------------------------------------------------------
template <typename T, int ME, int TX, int TY_>
struct YeeGeom {
  static constexpr int R = 16 / (int)sizeof(T);  // elements per 16-byte vector
  static constexpr int RW = 4;                    // outputs per task
  static constexpr int TY = TY_;
  static constexpr int VW = RW / R;               // vectors per task row segment
  static constexpr int HB = ME <= 4 ? 4 : ME;     // B and E^{n+1} halo (>= ME, multiple of 4)
  static constexpr int WB = TX + 2 * HB, WE = TX + 4 * HB;
  static constexpr int NWIN = (RW + HB + ME + R - 1) / R * R;  // Faraday window elements
  static constexpr int NWV = NWIN / R;
  static constexpr int NGX = WB / RW;  // task groups per row
  static constexpr int GT0 = HB / RW, NGT = TX / RW;
  static constexpr int PYE = TY + 3, PYB = TY + 2, PYF = TY + 1;
  static constexpr int PAD = sizeof(T) == 8 ? 2 : 0;
  static constexpr int PE = WE + PAD, PB = WB + PAD;
  static constexpr int SE3 = PYE * PE, SE1 = PYE * PB, SE2 = (PYE - 1) * PE;
  static constexpr int SB = PYB * PB, SF = PYF * PB;
  static constexpr int O_E1 = SE3, O_E2 = O_E1 + SE1, O_B = O_E2 + SE2, O_F = O_B + 3 * SB;
  static constexpr int NLDS = O_F + 6 * SF;
  static constexpr size_t lds_bytes = sizeof(T) * (size_t)NLDS;
  static constexpr int CG = sizeof(T) == 8 ? 8 : 16, CR = 16 / CG;  // task groups x rows per 16 lanes
  static constexpr int NCX = (NGX + CG - 1) / CG;
  // task slots: the NT3 tile positions, the halo groups of the tile rows, then
  // rows TY .. PYB-1 (see yee_task)
  static constexpr int NT3 = TY * NGT, NH = 2 * GT0 * TY;
  static constexpr int NTASK = NT3 + NH + (PYB - TY + CR - 1) / CR * NCX * 16;
  // E plane loader: 16-byte vectors of E3 (PYE x WE), E1 (PYE x WB), E2 ((PYE-1) x WE)
  static constexpr int L3 = PYE * (WE / R), L1 = PYE * (WB / R), L2 = (PYE - 1) * (WE / R);
  static constexpr int NLV = L3 + L1 + L2;
};

// Task position (row tr, group tg) of task slot t.  Slots [0, NT3) hold the
// tile positions (rows 0..TY-1, groups GT0..GT0+NGT-1) in chunks of CG groups
// x CR rows per 16 lanes, so that they fill whole waves, one per SIMD at 256
// slots; slots [NT3, NT3+NH) the 2 GT0 halo groups of each tile row, row by
// row; then rows TY..PYB-1 in CG x CR chunks.  A slot past the last position
// gets tr = PYB (no task).  16 consecutive lanes read 16-byte LDS vectors at
// distinct bank quads in each part (row pitches of 2 mod 4 elements at FP64).
template <class G>
__device__ __forceinline__ void yee_task(int t, int& tr, int& tg) {
  const int l16 = t & 15, gl = l16 % G::CG, rl = l16 / G::CG;
  static_assert(G::NGT % G::CG == 0 && G::NT3 % 16 == 0 && G::NH % 16 == 0, "task layout");
  if (t < G::NT3) {
    constexpr int cpr = G::NGT / G::CG;  // chunks per band of CR rows
    const int c = t >> 4;
    tr = (c / cpr) * G::CR + rl;
    tg = G::GT0 + (c % cpr) * G::CG + gl;
    return;
  }
  t -= G::NT3;
  if (t < G::NH) {
    const int h = t % (2 * G::GT0);
    tr = t / (2 * G::GT0);
    tg = h < G::GT0 ? h : G::NGT + h;
    return;
  }
  const int c = (t - G::NH) >> 4;
  tr = G::TY + (c / G::NCX) * G::CR + rl;
  tg = (c % G::NCX) * G::CG + gl;
  if (tg >= G::NGX || tr >= G::PYB) tr = G::PYB;
}

// RW aligned consecutive elements as 16-byte vectors (LDS or global memory)
template <typename T, int RW>
__device__ __forceinline__ void ld_run(const T* __restrict__ p, T (&o)[RW]) {
  using V = typename Vec16<T>::type;
  constexpr int R = 16 / (int)sizeof(T);
#pragma unroll
  for (int v = 0; v < RW / R; ++v) {
    const V a = *reinterpret_cast<const V*>(p + v * R);
#pragma unroll
    for (int e = 0; e < R; ++e) o[v * R + e] = a[e];
  }
}
template <typename T, int RW>
__device__ __forceinline__ void st_run(T* __restrict__ p, const T (&o)[RW]) {
  using V = typename Vec16<T>::type;
  constexpr int R = 16 / (int)sizeof(T);
#pragma unroll
  for (int v = 0; v < RW / R; ++v) {
    V a;
#pragma unroll
    for (int e = 0; e < R; ++e) a[e] = o[v * R + e];
    *reinterpret_cast<V*>(p + v * R) = a;
  }
}

// non-temporal variant for the sweep's outputs (written once, never re-read)
template <typename T, int RW>
__device__ __forceinline__ void st_run_nt(T* __restrict__ p, const T (&o)[RW]) {
  using V = typename Vec16<T>::type;
  constexpr int R = 16 / (int)sizeof(T);
#pragma unroll
  for (int v = 0; v < RW / R; ++v) {
    V a;
#pragma unroll
    for (int e = 0; e < R; ++e) a[e] = o[v * R + e];
    __builtin_nontemporal_store(a, reinterpret_cast<V*>(p + v * R));
  }
}

// Faraday taps of output u for a window whose index 0 is HB columns left of
// the task's first output: sum_q a_q (w[u+HB+q] - w[u+HB-q+1])
template <typename T, int ME, int HB, int NW>
__device__ __forceinline__ T faraday_w(const T (&w)[NW], const T (&a)[ME], int u) {
  T acc = 0;
#pragma unroll
  for (int q = 1; q <= ME; ++q) acc += a[q - 1] * (w[u + HB + q] - w[u + HB - q + 1]);
  return acc;
}

template <typename T, int ME, int TX, int TY, int NT, int WPE, bool HAS_J, bool FLAT>
__global__ __launch_bounds__(NT, WPE) void sweep_yee_kernel(const T* __restrict__ iE1, const T* __restrict__ iE2,
                                                       const T* __restrict__ iE3, const T* __restrict__ iB1,
                                                       const T* __restrict__ iB2, const T* __restrict__ iB3,
                                                       const T* __restrict__ J1, const T* __restrict__ J2,
                                                       const T* __restrict__ J3, T* __restrict__ oE1,
                                                       T* __restrict__ oE2, T* __restrict__ oE3,
                                                       T* __restrict__ oB1, T* __restrict__ oB2,
                                                       T* __restrict__ oB3, T* __restrict__ oH1,
                                                       T* __restrict__ oH2, T* __restrict__ oH3, Mesh m,
                                                       int tiles_x, int tiles, int KZ, SweepCoef<T, ME, 1> c) {
  using G = YeeGeom<T, ME, TX, TY>;
  using V = typename Vec16<T>::type;
  constexpr int R = G::R, RW = G::RW, HB = G::HB;
  // loader slots per component (each slot loads one component)
  constexpr int N3S = (G::L3 + NT - 1) / NT, N1S = (G::L1 + NT - 1) / NT, N2S = (G::L2 + NT - 1) / NT;
  static_assert(G::NTASK <= NT, "tasks exceed the workgroup");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* const lds = reinterpret_cast<T*>(lds_raw);
  T* const sE3 = lds;
  T* const sE1 = lds + G::O_E1;
  T* const sE2 = lds + G::O_E2;
  T* const sB = lds + G::O_B;  // [component][PYB][PB]
  T* const sF = lds + G::O_F;  // [plane parity][component][PYF][PB]

  const int tid = threadIdx.x;
  // XCD-aware tile order (consecutive workgroups go round-robin to the 8 XCDs)
  int tile = blockIdx.x;
  if (tiles % 8 == 0) tile = (tile % 8) * (tiles / 8) + tile / 8;
  const int i0 = (tile % tiles_x) * TX, j0 = (tile / tiles_x) * TY;
  const size_t plane_sz = (size_t)m.n1 * m.n2;
  auto gi = [&](int rel) {
    int i = (i0 + rel) % m.n1;
    return i < 0 ? i + m.n1 : i;
  };
  auto gj = [&](int rel) {
    int j = (j0 + rel) % m.n2;
    return j < 0 ? j + m.n2 : j;
  };
  auto poff = [&](int k) {
    k %= m.n3;
    return (size_t)(k < 0 ? k + m.n3 : k) * plane_sz;
  };

  // this thread's task: group tg (columns x .. x+RW-1), row tr
  int tr, tg;
  yee_task<G>(tid, tr, tg);
  const int x = -HB + RW * tg;
  const bool t1 = tr < G::PYB;        // B^{n+1/2} row tr-1
  const bool t2 = tr < G::PYF;        // E^{n+1} row tr
  const bool t3 = tid < G::NT3;       // tile output (B1, B2 of stage 3)
  // stage 3's B3 at tile position tid - NT3 is computed by this thread: the
  // two waves of each SIMD share the tile's stage 3
  static_assert(2 * G::NT3 <= NT, "stage-3 split needs two slots per tile position");
  const bool w3 = tid >= G::NT3 && tid < 2 * G::NT3;
  int tr3, tg3;
  yee_task<G>(w3 ? tid - G::NT3 : 0, tr3, tg3);
  const int x3 = -HB + RW * tg3, wcol3 = RW * tg3;
  // in-plane offsets of the task's first element (a plane holds < 2^31 cells)
  const int g1 = t1 ? gj(tr - 1) * m.n1 + gi(x) : 0;
  const int g2 = t2 ? gj(tr) * m.n1 + gi(x) : 0;
  const bool out = t3 && j0 + tr < m.n2 && i0 + x < m.n1;
  const bool out3 = w3 && j0 + tr3 < m.n2 && i0 + x3 < m.n1;
  const int g3 = out3 ? gj(tr3) * m.n1 + gi(x3) : 0;
  // stage-1 tasks on the tile also write B^{n+1/2} (when oH1 is given)
  const bool out_h = oH1 && t1 && tr >= 1 && tr <= TY && tg >= G::GT0 && tg < G::GT0 + G::NGT &&
                     j0 + tr - 1 < m.n2 && i0 + x < m.n1;
  const int wcol = RW * tg;  // LDS column of the task's window / B-extent position

  // E plane loader: slot s of component q covers vector tid + s NT of that
  // component's region; only the wrapped global offset is kept
  int ga3[N3S], ga1[N1S], ga2[N2S];
  auto slot_g = [&](int v, int wv, int halo) {
    const int row = v / wv, col = (v - row * wv) * R;
    return gj(row - 1) * m.n1 + gi(col - halo);
  };
#pragma unroll
  for (int s = 0; s < N3S; ++s) ga3[s] = tid + s * NT < G::L3 ? slot_g(tid + s * NT, G::WE / R, 2 * HB) : 0;
#pragma unroll
  for (int s = 0; s < N1S; ++s) ga1[s] = tid + s * NT < G::L1 ? slot_g(tid + s * NT, G::WB / R, HB) : 0;
#pragma unroll
  for (int s = 0; s < N2S; ++s) ga2[s] = tid + s * NT < G::L2 ? slot_g(tid + s * NT, G::WE / R, 2 * HB) : 0;
  // Every thread issues every global load of the march, whether or not it
  // uses the value (idle slots and tasks read the plane's first vector), and
  // past the last plane as well.  The compiler's wait counts take the fewest
  // memory operations any path issues after a load; with no load under a
  // branch, stage 1 waits only for the loads of the plane before, not for the
  // E-plane prefetch issued at the top of the iteration.
  V pe3[N3S], pe1[N1S], pe2[N2S];
  auto load_E = [&](size_t o) {  // o: offset of the plane
#pragma unroll
    for (int s = 0; s < N3S; ++s) pe3[s] = *reinterpret_cast<const V*>(iE3 + o + ga3[s]);
#pragma unroll
    for (int s = 0; s < N1S; ++s) pe1[s] = *reinterpret_cast<const V*>(iE1 + o + ga1[s]);
#pragma unroll
    for (int s = 0; s < N2S; ++s) pe2[s] = *reinterpret_cast<const V*>(iE2 + o + ga2[s]);
  };
  auto lds_at = [&](int v, int wv, int pitch) {
    const int row = v / wv;
    return row * pitch + (v - row * wv) * R;
  };
  auto store_E = [&]() {
#pragma unroll
    for (int s = 0; s < N3S; ++s) {
      const int v = tid + s * NT;
      if (v < G::L3) *reinterpret_cast<V*>(sE3 + lds_at(v, G::WE / R, G::PE)) = pe3[s];
    }
#pragma unroll
    for (int s = 0; s < N1S; ++s) {
      const int v = tid + s * NT;
      if (v < G::L1) *reinterpret_cast<V*>(sE1 + lds_at(v, G::WB / R, G::PB)) = pe1[s];
    }
#pragma unroll
    for (int s = 0; s < N2S; ++s) {
      const int v = tid + s * NT;
      if (v < G::L2) *reinterpret_cast<V*>(sE2 + lds_at(v, G::WE / R, G::PE)) = pe2[s];
    }
  };

  T bn[3][RW], nn[2][RW], cb[3][RW], jv[HAS_J ? 3 : 1][RW];
  // B^n(k), E1/E2(k+1) at the stage-1 positions.  A stack of 2D planes
  // (FLAT) has no x3 derivative, so the next plane's E1/E2 are not read.
  auto load_own = [&](size_t pk, size_t pk1) {
    const size_t o = pk + g1, on = pk1 + g1;
    ld_run<T, RW>(iB1 + o, bn[0]);
    ld_run<T, RW>(iB2 + o, bn[1]);
    ld_run<T, RW>(iB3 + o, bn[2]);
    if constexpr (FLAT) {
#pragma unroll
      for (int u = 0; u < RW; ++u) nn[0][u] = nn[1][u] = 0;
      (void)on;
    } else {
      ld_run<T, RW>(iE1 + on, nn[0]);
      ld_run<T, RW>(iE2 + on, nn[1]);
    }
  };
  auto load_J = [&](size_t pk) {
    if constexpr (HAS_J) {
      const size_t o = pk + g2;
      ld_run<T, RW>(J1 + o, jv[0]);
      ld_run<T, RW>(J2 + o, jv[1]);
      ld_run<T, RW>(J3 + o, jv[2]);
    }
  };

  // ---- prologue: E(k0-1) in LDS; B^n(k0-1), E1/E2(k0) own, J(k0-1) ----
  // (the march covers planes k0 .. kend-1: one x3 chunk of KZ planes)
  const int k0 = blockIdx.y * KZ, kend = min(m.n3, k0 + KZ);
  // offsets of planes ka-1 .. ka+2: at FP64 carried from plane to plane (a
  // quarter of the loop's scalar instructions), at FP32 recomputed (carried
  // offsets push the 128-VGPR FP32 build into spilling)
  constexpr bool carry = sizeof(T) == 8;
  const size_t wrap = (size_t)m.n3 * plane_sz;
  size_t cm1 = poff(k0 - 2), c0 = poff(k0 - 1), c1 = poff(k0), c2 = poff(k0 + 1);
  load_E(c0);
  store_E();
  load_own(c0, c1);
  load_J(c0);
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int u = 0; u < RW; ++u) cb[q][u] = 0;
  __syncthreads();

  for (int ka = k0 - 1; ka <= kend; ++ka) {
    const bool more = ka < kend;
    auto pl = [&](int d) -> size_t {  // offset of plane ka+d, d = -1 .. 2
      if constexpr (carry) return d < 0 ? cm1 : d == 0 ? c0 : d == 1 ? c1 : c2;
      else return poff(ka + d);
    };
    load_E(pl(1));
    // ---- stage 1: B^{n+1/2}(ka) on the B extent ----
    if (t1) {
      T* bo = sB + tr * G::PB + wcol;
      T e1c[RW], e2w[RW];
      ld_run<T, RW>(sE1 + tr * G::PB + wcol, e1c);
      {  // B3 from the x1 derivative of E2 and the x2 difference of E1
        T w[G::NWIN], e1n[RW], o3[RW];
        load_window<T, G::NWV, R>(sE2 + tr * G::PE + wcol, w);
        ld_run<T, RW>(sE1 + (tr + 1) * G::PB + wcol, e1n);
#pragma unroll
        for (int u = 0; u < RW; ++u) {
          e2w[u] = w[u + HB];
          o3[u] = bn[2][u] - (faraday_w<T, ME, HB>(w, c.ae, u) - c.hy * (e1n[u] - e1c[u]));
        }
        st_run<T, RW>(bo + 2 * G::SB, o3);
        if (out_h && ka >= k0 && ka < kend) st_run<T, RW>(oH3 + pl(0) + g1, o3);
      }
      {  // B2 and B1
        T w[G::NWIN], e3n[RW], o1[RW], o2[RW];
        load_window<T, G::NWV, R>(sE3 + tr * G::PE + wcol, w);
        ld_run<T, RW>(sE3 + (tr + 1) * G::PE + wcol + HB, e3n);
#pragma unroll
        for (int u = 0; u < RW; ++u) {
          o2[u] = bn[1][u] - (c.hz * (nn[0][u] - e1c[u]) - faraday_w<T, ME, HB>(w, c.ae, u));
          o1[u] = bn[0][u] - (c.hy * (e3n[u] - w[u + HB]) - c.hz * (nn[1][u] - e2w[u]));
        }
        st_run<T, RW>(bo, o1);
        st_run<T, RW>(bo + G::SB, o2);
        if (out_h && ka >= k0 && ka < kend) {
          const size_t o = pl(0) + g1;
          st_run<T, RW>(oH1 + o, o1);
          st_run<T, RW>(oH2 + o, o2);
        }
      }
    }
    load_own(pl(1), pl(2));
    __syncthreads();
    // ---- stage 2: E^{n+1}(ka) on the E^{n+1} extent ----
    T g1c[RW], g2c[RW];
    if (t2) {
      const T* b = sB + (tr + 1) * G::PB + wcol;
      T b1c[RW], b2c[RW], b3c[RW], b1s[RW], b3s[RW];
      ld_run<T, RW>(b, b1c);
      ld_run<T, RW>(b + G::SB, b2c);
      ld_run<T, RW>(b + 2 * G::SB, b3c);
      ld_run<T, RW>(b - G::PB, b1s);
      ld_run<T, RW>(b + 2 * G::SB - G::PB, b3s);
      // x1 neighbour of the first output (the extent's first column, whose
      // E^{n+1} is never read, takes its own value)
      const int lm = wcol > 0 ? -1 : 0;
      const T b2l = b[G::SB + lm], b3l = b[2 * G::SB + lm];
      T e1o[RW], e2o[RW], e3o[RW];
      ld_run<T, RW>(sE1 + (tr + 1) * G::PB + wcol, e1o);
      ld_run<T, RW>(sE2 + (tr + 1) * G::PE + wcol + HB, e2o);
      ld_run<T, RW>(sE3 + (tr + 1) * G::PE + wcol + HB, e3o);
      T f3[RW];
#pragma unroll
      for (int u = 0; u < RW; ++u) {
        const T b3p = u == 0 ? b3l : b3c[u - 1];
        const T b2p = u == 0 ? b2l : b2c[u - 1];
        T c1 = c.ty * (b3c[u] - b3s[u]) - c.tz * (b2c[u] - cb[1][u]);
        T c2 = c.tz * (b1c[u] - cb[0][u]) - c.ab[0] * (b3c[u] - b3p);
        T c3 = c.ab[0] * (b2c[u] - b2p) - c.ty * (b1c[u] - b1s[u]);
        if constexpr (HAS_J) {
          c1 -= c.dt * jv[0][u];
          c2 -= c.dt * jv[1][u];
          c3 -= c.dt * jv[2][u];
        }
        g1c[u] = e1o[u] + c1;
        g2c[u] = e2o[u] + c2;
        f3[u] = e3o[u] + c3;
      }
      T* f = sF + (ka & 1) * 3 * G::SF + tr * G::PB + wcol;
      st_run<T, RW>(f, g1c);
      st_run<T, RW>(f + G::SF, g2c);
      st_run<T, RW>(f + 2 * G::SF, f3);
      if (out && ka >= k0 && ka < kend) {
        const size_t o = pl(0) + g2;
        st_run_nt<T, RW>(oE1 + o, g1c);
        st_run_nt<T, RW>(oE2 + o, g2c);
        st_run_nt<T, RW>(oE3 + o, f3);
      }
    }
    load_J(pl(1));
    // ---- stage 3: B^{n+1}(ka-1) on the tile ----
    if (t3 && ka - 1 >= k0) {  // B2 and B1 at the thread's own tile position
      const T* f = sF + ((ka - 1) & 1) * 3 * G::SF + tr * G::PB;
      T w[G::NWIN], f1c[RW], f2c[RW], f3n[RW], o1[RW], o2[RW];
      ld_run<T, RW>(f + wcol, f1c);
      ld_run<T, RW>(f + G::SF + wcol, f2c);
      load_window<T, G::NWV, R>(f + 2 * G::SF + wcol - HB, w);
      ld_run<T, RW>(f + 2 * G::SF + G::PB + wcol, f3n);
#pragma unroll
      for (int u = 0; u < RW; ++u) {
        o2[u] = cb[1][u] - (c.hz * (g1c[u] - f1c[u]) - faraday_w<T, ME, HB>(w, c.ae, u));
        o1[u] = cb[0][u] - (c.hy * (f3n[u] - w[u + HB]) - c.hz * (g2c[u] - f2c[u]));
      }
      if (out) {
        const size_t o = pl(-1) + g2;
        st_run_nt<T, RW>(oB1 + o, o1);
        st_run_nt<T, RW>(oB2 + o, o2);
      }
    }
    if (w3 && ka - 1 >= k0) {  // B3 from the x1 derivative of E2 and the x2 difference of E1
      const T* f = sF + ((ka - 1) & 1) * 3 * G::SF + tr3 * G::PB;
      T w[G::NWIN], f1c[RW], f1n[RW], o3[RW];
      ld_run<T, RW>(f + wcol3, f1c);
      load_window<T, G::NWV, R>(f + G::SF + wcol3 - HB, w);
      ld_run<T, RW>(f + G::PB + wcol3, f1n);
#pragma unroll
      for (int u = 0; u < RW; ++u)
        o3[u] = cb[2][u] - (faraday_w<T, ME, HB>(w, c.ae, u) - c.hy * (f1n[u] - f1c[u]));
      if (out3) st_run_nt<T, RW>(oB3 + pl(-1) + g3, o3);
    }
    // B^{n+1/2}(ka) for stage 2 at ka+1 (components 1, 2 at the task's
    // position) and stage 3 at ka (component 3 at the B3 position)
    if (t2) {
      const T* b = sB + (tr + 1) * G::PB + wcol;
      ld_run<T, RW>(b, cb[0]);
      ld_run<T, RW>(b + G::SB, cb[1]);
    }
    if (w3) ld_run<T, RW>(sB + 2 * G::SB + (tr3 + 1) * G::PB + wcol3, cb[2]);
    __syncthreads();
    if (more) store_E();
    __syncthreads();
    if constexpr (carry) {
      cm1 = c0;
      c0 = c1;
      c1 = c2;
      c2 += plane_sz;
      if (c2 >= wrap) c2 -= wrap;
    }
  }
}

// ---------------------------------------------------------------------------
// x1 current correction (Sec. 3.3, Eq. correction): the Ampere-law x1 current
// is the deposited one times [k]_Yee/[k]_B1 per x1 mode, applied here as the
// periodic convolution out_i = sum_{|m| <= KW} h_|m| J1_{i-m} along each x1
// row (the host computes the taps from that ratio).  A wave owns 512
// consecutive outputs of one row, 8 per lane.  The row window
// [s0 - KW, s0 + 512 + KW) is staged in LDS with one pad word after every 8
// values, so that lanes 8 values apart read different banks; the taps are
// uniform (scalar) loads.  Accumulation in FP64 for either precision.
// ---------------------------------------------------------------------------
template <typename T, int KW>
__global__ __launch_bounds__(256) void correct_j1_kernel(const T* __restrict__ J1, T* __restrict__ out,
                                                         const double* __restrict__ h, int n1, int64_t units,
                                                         int nseg) {
  constexpr int SEG = 512, RWc = 8, WIN = SEG + 2 * KW, WINP = WIN + WIN / 8 + 1;
  __shared__ double win[4][WINP];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t unit = (int64_t)blockIdx.x * 4 + wave;
  const bool live = unit < units;
  const int64_t row = live ? unit / nseg : 0;
  const int s0 = live ? (int)(unit - row * nseg) * SEG : 0;
  const T* src = J1 + row * (int64_t)n1;
  double* w = win[wave];
  if (n1 >= WIN) {  // the window wraps at most once
    for (int t = lane; t < WIN; t += 64) {
      int i = s0 - KW + t;
      i += i < 0 ? n1 : (i >= n1 ? -n1 : 0);
      w[t + (t >> 3)] = live ? (double)src[i] : 0.0;
    }
  } else {
    for (int t = lane; t < WIN; t += 64) {
      int i = (s0 - KW + t) % n1;
      if (i < 0) i += n1;
      w[t + (t >> 3)] = live ? (double)src[i] : 0.0;
    }
  }
  __syncthreads();  // the only barrier: every thread reaches it
  if (!live) return;
  // output s0 + 8 lane + u takes the window value at index 8 lane + t with tap
  // m = u + KW - t (its source lies m cells to the left)
  const double* wl = w + 9 * lane;
  double acc[RWc] = {};
#pragma unroll
  for (int t = 0; t < RWc + 2 * KW; ++t) {
    const double v = wl[t + (t >> 3)];
#pragma unroll
    for (int u = 0; u < RWc; ++u) {
      constexpr int lo = -KW;
      const int mm = u + KW - t;
      if (mm >= lo && mm <= KW) acc[u] += h[mm < 0 ? -mm : mm] * v;
    }
  }
  T* dst = out + row * (int64_t)n1;
#pragma unroll
  for (int u = 0; u < RWc; ++u) {
    const int i = s0 + RWc * lane + u;
    if (i < n1) dst[i] = (T)acc[u];
  }
}

template <typename T, int KW>
int run_correct_j1(const Mesh& m, const void* J1, void* out, const double* taps, hipStream_t s) {
  const int nseg = (m.n1 + 511) / 512;
  const int64_t units = (int64_t)m.n2 * m.n3 * nseg;
  const int64_t blocks = (units + 3) / 4;
  if (blocks > 0x7fffffff) return set_error(PIC_ESHAPE, "current correction: too many rows");
  hipLaunchKernelGGL((correct_j1_kernel<T, KW>), dim3((unsigned)blocks), dim3(256), 0, s, (const T*)J1, (T*)out,
                     taps, m.n1, units, nseg);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "current correction launch failed");
}

template <typename T>
int dispatch_correct_j1(const Mesh& m, const void* J1, void* out, const double* taps, int kw, hipStream_t s) {
  switch (kw) {
    case 8: return run_correct_j1<T, 8>(m, J1, out, taps, s);
    case 16: return run_correct_j1<T, 16>(m, J1, out, taps, s);
    case 24: return run_correct_j1<T, 24>(m, J1, out, taps, s);
    case 32: return run_correct_j1<T, 32>(m, J1, out, taps, s);
    case 40: return run_correct_j1<T, 40>(m, J1, out, taps, s);
    case 48: return run_correct_j1<T, 48>(m, J1, out, taps, s);
    case 64: return run_correct_j1<T, 64>(m, J1, out, taps, s);
    default: return set_error(PIC_EINVAL, "current correction: tap width %d", kw);
  }
}

// compute units of the current device (queried once per device)
int device_cus() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    cached[dev] = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0 ? n : 256;
  }
  return cached[dev];
}

template <typename T, int ME, int TX, int TY, int NT, int WPE>
int launch_sweep_yee(const Mesh& m, void* const Ein[3], void* const Bin[3], void* const J[3], void* const Eout[3],
                     void* const Bout[3], void* const Bh[3], const SweepCoef<T, ME, 1>& c, int tiles_x, int tiles,
                     int wgs_per_cu, hipStream_t s) {
  using G = YeeGeom<T, ME, TX, TY>;
  const bool hasJ = J && J[0];
  const bool flat = m.ndim == 2;
  auto kern = hasJ ? (flat ? sweep_yee_kernel<T, ME, TX, TY, NT, WPE, true, true>
                           : sweep_yee_kernel<T, ME, TX, TY, NT, WPE, true, false>)
                   : (flat ? sweep_yee_kernel<T, ME, TX, TY, NT, WPE, false, true>
                           : sweep_yee_kernel<T, ME, TX, TY, NT, WPE, false, false>);
  static_assert(G::lds_bytes <= 160 * 1024, "sweep tile exceeds LDS");
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::lds_bytes) !=
      hipSuccess)
    return set_error(PIC_EHIP, "sweep: cannot reserve %zu bytes of LDS", G::lds_bytes);
  // too few tiles to fill the chip: split the x3 march into chunks (each one
  // re-reads the two planes before it)
  int nz = 1;
  const int want = wgs_per_cu * device_cus();
  if (tiles < want) nz = min(m.n3, (want + tiles - 1) / tiles);
  const int KZ = (m.n3 + nz - 1) / nz;
  nz = (m.n3 + KZ - 1) / KZ;
  hipLaunchKernelGGL(kern, dim3(tiles, nz), dim3(NT), G::lds_bytes, s, (const T*)Ein[0], (const T*)Ein[1],
                     (const T*)Ein[2], (const T*)Bin[0], (const T*)Bin[1], (const T*)Bin[2],
                     (const T*)(hasJ ? J[0] : nullptr), (const T*)(hasJ ? J[1] : nullptr),
                     (const T*)(hasJ ? J[2] : nullptr), (T*)Eout[0], (T*)Eout[1], (T*)Eout[2], (T*)Bout[0],
                     (T*)Bout[1], (T*)Bout[2], (T*)(Bh ? Bh[0] : nullptr), (T*)(Bh ? Bh[1] : nullptr),
                     (T*)(Bh ? Bh[2] : nullptr), m, tiles_x, tiles, KZ, c);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "sweep launch failed");
}

template <typename T, int ME, int TX, int TY, int NT>
int run_sweep_yee(const Mesh& m, void* const Ein[3], void* const Bin[3], void* const J[3], void* const Eout[3],
                  void* const Bout[3], void* const Bh[3], const double* CE, int MEr, const double* CB, double dt,
                  hipStream_t s) {
  SweepCoef<T, ME, 1> c;
  for (int q = 0; q < ME; ++q) c.ae[q] = (T)(q < MEr ? CE[q] * (dt / 2) / m.dx1 : 0.0);
  c.ab[0] = (T)(CB[0] * dt / m.dx1);
  c.hy = (T)((dt / 2) / m.dx2);
  c.hz = (T)(m.ndim == 3 ? (dt / 2) / m.dx3 : 0.0);
  c.ty = (T)(dt / m.dx2);
  c.tz = (T)(m.ndim == 3 ? dt / m.dx3 : 0.0);
  c.dt = (T)dt;
  const int tiles_x = (m.n1 + TX - 1) / TX;
  const int tiles = tiles_x * ((m.n2 + TY - 1) / TY);
  // FP32 tiles fit two workgroups per CU (LDS and 128 VGPRs); that pays
  // where the mesh has fewer than two tiles per CU (the x3 march is then
  // split to fill the slots) and there is no current to read.  With at least
  // two tiles per CU, or with J (whose 128-VGPR build spills 13 registers),
  // one workgroup per CU (144 VGPRs, no spills) streams faster.  FP64 takes
  // one workgroup per CU.
  if constexpr (sizeof(T) == 4) {
    if (tiles >= 2 * device_cus() || (J && J[0]))
      return launch_sweep_yee<T, ME, TX, TY, NT, 2>(m, Ein, Bin, J, Eout, Bout, Bh, c, tiles_x, tiles, 1, s);
    return launch_sweep_yee<T, ME, TX, TY, NT, 4>(m, Ein, Bin, J, Eout, Bout, Bh, c, tiles_x, tiles, 2, s);
  }
  return launch_sweep_yee<T, ME, TX, TY, NT, 2>(m, Ein, Bin, J, Eout, Bout, Bh, c, tiles_x, tiles, 1, s);
}

template <typename T, int ME, int MB, int TX, int TY, int NT>
int run_sweep(const Mesh& m, void* const Ein[3], void* const Bin[3], void* const J[3], void* const Eout[3],
              void* const Bout[3], const double* CE, int MEr, const double* CB, int MBr, double dt, hipStream_t s) {
  using G = SweepGeom<T, ME, MB, TX, TY>;
  SweepCoef<T, ME, MB> c;
  for (int q = 0; q < ME; ++q) c.ae[q] = (T)(q < MEr ? CE[q] * (dt / 2) / m.dx1 : 0.0);
  for (int q = 0; q < MB; ++q) c.ab[q] = (T)(q < MBr ? CB[q] * dt / m.dx1 : 0.0);
  c.hy = (T)((dt / 2) / m.dx2);
  c.hz = (T)(m.ndim == 3 ? (dt / 2) / m.dx3 : 0.0);
  c.ty = (T)(dt / m.dx2);
  c.tz = (T)(m.ndim == 3 ? dt / m.dx3 : 0.0);
  c.dt = (T)dt;
  const int tiles_x = (m.n1 + TX - 1) / TX;
  const int tiles_y = (m.n2 + TY - 1) / TY;
  // too few tiles to fill the chip: split the x3 march into chunks, as the
  // Yee-Ampere sweep does (each chunk re-reads the planes its pipeline needs)
  const int tiles = tiles_x * tiles_y;
  const int wgs_per_cu = G::lds_bytes * 2 <= 160 * 1024 ? 2 : 1;
  int nz = 1;
  const int want = wgs_per_cu * device_cus();
  if (tiles < want) nz = min(m.n3, (want + tiles - 1) / tiles);
  const int KZ = (m.n3 + nz - 1) / nz;
  const bool hasJ = J && J[0];
  auto kern = hasJ ? sweep_kernel<T, ME, MB, TX, TY, NT, true> : sweep_kernel<T, ME, MB, TX, TY, NT, false>;
  static_assert(G::lds_bytes <= 160 * 1024, "sweep tile exceeds LDS");
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::lds_bytes) !=
      hipSuccess)
    return set_error(PIC_EHIP, "sweep: cannot reserve %zu bytes of LDS", G::lds_bytes);
  hipLaunchKernelGGL(kern, dim3(tiles_x * tiles_y, (m.n3 + KZ - 1) / KZ), dim3(NT), G::lds_bytes, s,
                     (const T*)Ein[0], (const T*)Ein[1], (const T*)Ein[2], (const T*)Bin[0], (const T*)Bin[1],
                     (const T*)Bin[2], (const T*)(hasJ ? J[0] : nullptr), (const T*)(hasJ ? J[1] : nullptr),
                     (const T*)(hasJ ? J[2] : nullptr), (T*)Eout[0], (T*)Eout[1], (T*)Eout[2], (T*)Bout[0],
                     (T*)Bout[1], (T*)Bout[2], m, KZ, tiles_x, tiles_x * tiles_y, c);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "sweep launch failed");
}

template <typename T, int TXn, int TY, int NT>
int dispatch_sweep(const Mesh& m, void* const Ein[3], void* const Bin[3], void* const J[3], void* const Eout[3],
                   void* const Bout[3], void* const Bh[3], const double* CE, int ME, const double* CB, int MB,
                   double dt, hipStream_t s) {
  const int we = round_width(ME), wb = round_width(MB);
  const int w = we > wb ? we : wb;
  // Ampere stencil either Yee (width 1) or padded to the Faraday width
  if (wb == 1) {
    constexpr int YT = 8;  // rows per tile of the Yee-Ampere sweep
    switch (we) {
      case 1: return run_sweep_yee<T, 1, 128, YT, NT>(m, Ein, Bin, J, Eout, Bout, Bh, CE, ME, CB, dt, s);
      case 2: return run_sweep_yee<T, 2, 128, YT, NT>(m, Ein, Bin, J, Eout, Bout, Bh, CE, ME, CB, dt, s);
      case 4: return run_sweep_yee<T, 4, 128, YT, NT>(m, Ein, Bin, J, Eout, Bout, Bh, CE, ME, CB, dt, s);
      case 8: return run_sweep_yee<T, 8, 128, YT, NT>(m, Ein, Bin, J, Eout, Bout, Bh, CE, ME, CB, dt, s);
      default: return run_sweep_yee<T, 16, 128, YT, NT>(m, Ein, Bin, J, Eout, Bout, Bh, CE, ME, CB, dt, s);
    }
  }
  // general Ampere stencil: B^{n+1/2} (when asked for) from its own half step
  if (Bh && Bh[0]) {
    const int rc = dispatch_b<T>(m, Ein, Bin, Bh, CE, ME, dt / 2, s);
    if (rc) return rc;
  }
  switch (w) {
    case 2: return run_sweep<T, 2, 2, TXn, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
    case 4: return run_sweep<T, 4, 4, TXn, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
    case 8: return run_sweep<T, 8, 8, TXn, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
    default: return run_sweep<T, 16, 16, TXn, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
  }
}

}  // namespace

int round_width(int m) {
  for (int w : kWidths)
    if (m <= w) return w;
  return kWidths[4];
}

int launch_advance_b(int prec, const Mesh& m, void* const E[3], void* const B[3], void* const Bout[3],
                     const double* CE, int ME, double h, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return prec == PIC_FP64 ? dispatch_b<double>(m, E, B, Bout, CE, ME, h, s)
                          : dispatch_b<float>(m, E, B, Bout, CE, ME, h, s);
}

int launch_sweep(int prec, const Mesh& m, void* const Ein[3], void* const Bin[3], void* const J[3],
                 void* const Eout[3], void* const Bout[3], void* const Bh[3], const double* CE, int ME,
                 const double* CB, int MB, double dt, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (prec == PIC_FP64)
    return dispatch_sweep<double, 64, 4, 512>(m, Ein, Bin, J, Eout, Bout, Bh, CE, ME, CB, MB, dt, s);
  return dispatch_sweep<float, 128, 8, 512>(m, Ein, Bin, J, Eout, Bout, Bh, CE, ME, CB, MB, dt, s);
}

int launch_correct_j1(int prec, const Mesh& m, const void* J1, void* out, const double* taps, int kw,
                      void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return prec == PIC_FP64 ? dispatch_correct_j1<double>(m, J1, out, taps, kw, s)
                          : dispatch_correct_j1<float>(m, J1, out, taps, kw, s);
}

int launch_advance_e(int prec, const Mesh& m, void* const E[3], void* const B[3], void* const J[3],
                     const double* CB, int MB, double dt, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return prec == PIC_FP64 ? dispatch_e<double>(m, E, B, J, CB, MB, dt, s)
                          : dispatch_e<float>(m, E, B, J, CB, MB, dt, s);
}

}  // namespace yeepic
