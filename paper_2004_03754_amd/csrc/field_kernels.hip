// Field kernels: Faraday half step, Ampere step, fused sweep (gfx950).
//
// Eq. (maxwell) with the App. B x1 operators
//   Faraday  d^E f_i = (1/dx1) sum_j C^E_j (f_{i+j}   - f_{i-j+1})
//   Ampere   d^B f_i = (1/dx1) sum_j C^B_j (f_{i+j-1} - f_{i-j})
// and Yee differences along x2, x3 (forward in Faraday, backward in Ampere).
// Arrays are [n3][n2][n1], x1 contiguous, periodic in every direction.
#include <hip/hip_runtime.h>

#include "yeepic_internal.h"

namespace yeepic {
namespace {

template <typename T, int W>
struct Taps {
  T a[W];
};

__device__ __forceinline__ int wrap1(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

// ---------------------------------------------------------------------------
// Standalone steps: one thread per cell, neighbours read through the caches.
// In place is safe: a B update reads only E and its own B, and vice versa.
// ---------------------------------------------------------------------------

// B <- B - h curl_E E.  ``ce`` holds h C^E_j/dx1; hy = h/dx2, hz = h/dx3.
template <typename T, int W>
__global__ __launch_bounds__(256) void advance_b_kernel(const T* __restrict__ E1, const T* __restrict__ E2,
                                                        const T* __restrict__ E3, T* __restrict__ B1,
                                                        T* __restrict__ B2, T* __restrict__ B3, Mesh m,
                                                        Taps<T, W> ce, T hy, T hz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (i >= m.n1) return;
  const int jp = (j + 1 == m.n2) ? 0 : j + 1;
  const int kp = (k + 1 == m.n3) ? 0 : k + 1;
  const size_t row = ((size_t)k * m.n2 + j) * m.n1;
  const size_t rowjp = ((size_t)k * m.n2 + jp) * m.n1;
  const size_t rowkp = ((size_t)kp * m.n2 + j) * m.n1;
  const size_t c = row + i;
  T d1E3 = 0, d1E2 = 0;
#pragma unroll
  for (int q = 1; q <= W; ++q) {
    const int ip = wrap1(i + q, m.n1);
    const int im = wrap1(i - q + 1, m.n1);
    d1E3 += ce.a[q - 1] * (E3[row + ip] - E3[row + im]);
    d1E2 += ce.a[q - 1] * (E2[row + ip] - E2[row + im]);
  }
  const T e1 = E1[c], e2 = E2[c], e3 = E3[c];
  B1[c] -= hy * (E3[rowjp + i] - e3) - hz * (E2[rowkp + i] - e2);
  B2[c] -= hz * (E1[rowkp + i] - e1) - d1E3;
  B3[c] -= d1E2 - hy * (E1[rowjp + i] - e1);
}

// E <- E + dt (curl_B B - J).  ``cb`` holds dt C^B_j/dx1; ty = dt/dx2,
// tz = dt/dx3; J may be null.
template <typename T, int W>
__global__ __launch_bounds__(256) void advance_e_kernel(T* __restrict__ E1, T* __restrict__ E2, T* __restrict__ E3,
                                                        const T* __restrict__ B1, const T* __restrict__ B2,
                                                        const T* __restrict__ B3, const T* __restrict__ J1,
                                                        const T* __restrict__ J2, const T* __restrict__ J3,
                                                        Mesh m, Taps<T, W> cb, T ty, T tz, T dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (i >= m.n1) return;
  const int jm = (j == 0) ? m.n2 - 1 : j - 1;
  const int km = (k == 0) ? m.n3 - 1 : k - 1;
  const size_t row = ((size_t)k * m.n2 + j) * m.n1;
  const size_t rowjm = ((size_t)k * m.n2 + jm) * m.n1;
  const size_t rowkm = ((size_t)km * m.n2 + j) * m.n1;
  const size_t c = row + i;
  T d1B3 = 0, d1B2 = 0;
#pragma unroll
  for (int q = 1; q <= W; ++q) {
    const int ip = wrap1(i + q - 1, m.n1);
    const int im = wrap1(i - q, m.n1);
    d1B3 += cb.a[q - 1] * (B3[row + ip] - B3[row + im]);
    d1B2 += cb.a[q - 1] * (B2[row + ip] - B2[row + im]);
  }
  const T b1 = B1[c], b2 = B2[c], b3 = B3[c];
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
int run_advance_b(const Mesh& m, void* const E[3], void* const B[3], const double* CE, int ME, double h,
                  hipStream_t s) {
  const int bx = m.n1 >= 256 ? 256 : m.n1;
  hipLaunchKernelGGL((advance_b_kernel<T, W>), cell_grid(m, bx), dim3(bx), 0, s, (const T*)E[0], (const T*)E[1],
                     (const T*)E[2], (T*)B[0], (T*)B[1], (T*)B[2], m, scaled_taps<T, W>(CE, ME, h / m.dx1),
                     (T)(h / m.dx2), (T)(m.ndim == 3 ? h / m.dx3 : 0.0));
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "advance_b launch failed");
}

template <typename T, int W>
int run_advance_e(const Mesh& m, void* const E[3], void* const B[3], void* const J[3], const double* CB, int MB,
                  double dt, hipStream_t s) {
  const int bx = m.n1 >= 256 ? 256 : m.n1;
  hipLaunchKernelGGL((advance_e_kernel<T, W>), cell_grid(m, bx), dim3(bx), 0, s, (T*)E[0], (T*)E[1], (T*)E[2],
                     (const T*)B[0], (const T*)B[1], (const T*)B[2], (const T*)(J ? J[0] : nullptr),
                     (const T*)(J ? J[1] : nullptr), (const T*)(J ? J[2] : nullptr), m,
                     scaled_taps<T, W>(CB, MB, dt / m.dx1), (T)(dt / m.dx2),
                     (T)(m.ndim == 3 ? dt / m.dx3 : 0.0), (T)dt);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "advance_e launch failed");
}

template <typename T>
int dispatch_b(const Mesh& m, void* const E[3], void* const B[3], const double* CE, int ME, double h, hipStream_t s) {
  switch (round_width(ME)) {
    case 1: return run_advance_b<T, 1>(m, E, B, CE, ME, h, s);
    case 2: return run_advance_b<T, 2>(m, E, B, CE, ME, h, s);
    case 4: return run_advance_b<T, 4>(m, E, B, CE, ME, h, s);
    case 8: return run_advance_b<T, 8>(m, E, B, CE, ME, h, s);
    default: return run_advance_b<T, 16>(m, E, B, CE, ME, h, s);
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
  static constexpr int HLE = 2 * ME + MB - 2, PXE = TX + 4 * ME + 2 * MB - 3, PYE = TY + 3;
  static constexpr int HLB = ME + MB - 1, PXB = TX + 2 * ME + 2 * MB - 2, PYB = TY + 2;
  static constexpr int HLF = ME - 1, PXF = TX + 2 * ME - 1, PYF = TY + 1;
  static constexpr int SE = PXE * PYE, SB = PXB * PYB, SF = PXF * PYF;  // one component, one plane
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

template <typename T, int ME, int MB, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void sweep_kernel(const T* __restrict__ iE1, const T* __restrict__ iE2,
                                                   const T* __restrict__ iE3, const T* __restrict__ iB1,
                                                   const T* __restrict__ iB2, const T* __restrict__ iB3,
                                                   const T* __restrict__ J1, const T* __restrict__ J2,
                                                   const T* __restrict__ J3, T* __restrict__ oE1,
                                                   T* __restrict__ oE2, T* __restrict__ oE3, T* __restrict__ oB1,
                                                   T* __restrict__ oB2, T* __restrict__ oB3, Mesh m, int KZ,
                                                   int tiles_x, SweepCoef<T, ME, MB> c) {
  using G = SweepGeom<T, ME, MB, TX, TY>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  // [buffer][component] planes
  T* sE = lds;                       // 2 x 3 x SE
  T* sB = sE + 2 * 3 * G::SE;        // 2 x 3 x SB
  T* sF = sB + 2 * 3 * G::SB;        // 2 x 3 x SF
  auto pE = [&](int plane, int comp) { return sE + ((plane & 1) * 3 + comp) * G::SE; };
  auto pB = [&](int plane, int comp) { return sB + ((plane & 1) * 3 + comp) * G::SB; };
  auto pF = [&](int plane, int comp) { return sF + ((plane & 1) * 3 + comp) * G::SF; };

  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int i0 = (tile % tiles_x) * TX;
  const int j0 = (tile / tiles_x) * TY;
  const int k0 = blockIdx.y * KZ;
  const int kend = min(k0 + KZ, m.n3);
  const size_t plane_sz = (size_t)m.n1 * m.n2;
  const T* inE[3] = {iE1, iE2, iE3};

  auto gi = [&](int rel) {  // tile-relative x1 -> global, periodic
    int i = (i0 + rel) % m.n1;
    return i < 0 ? i + m.n1 : i;
  };
  auto gj = [&](int rel) {
    int j = (j0 + rel) % m.n2;
    return j < 0 ? j + m.n2 : j;
  };
  auto gk = [&](int k) {
    k %= m.n3;
    return k < 0 ? k + m.n3 : k;
  };

  auto load_E = [&](int plane) {
    const size_t base = (size_t)gk(plane) * plane_sz;
    for (int p = tid; p < 3 * G::SE; p += NT) {
      const int comp = p / G::SE;
      const int q = p - comp * G::SE;
      const int r = q / G::PXE;
      const int x = q - r * G::PXE;
      pE(plane, comp)[q] = inE[comp][base + (size_t)gj(r - 1) * m.n1 + gi(x - G::HLE)];
    }
  };

  load_E(k0 - 1);
  load_E(k0);
  __syncthreads();

  for (int kk = k0 - 2; kk < kend; ++kk) {
    const int ka = kk + 1;  // plane of stages 1 and 2
    // ---- stage 1: B^{n+1/2}(ka) over the B buffer extent ----
    {
      const T* e1 = pE(ka, 0);
      const T* e2 = pE(ka, 1);
      const T* e3 = pE(ka, 2);
      const T* n1 = pE(ka + 1, 0);
      const T* n2 = pE(ka + 1, 1);
      T* b1 = pB(ka, 0);
      T* b2 = pB(ka, 1);
      T* b3 = pB(ka, 2);
      const size_t base = (size_t)gk(ka) * plane_sz;
      for (int p = tid; p < G::SB; p += NT) {
        const int r = p / G::PXB;
        const int x = p - r * G::PXB;
        const int xe = x + (G::HLE - G::HLB);
        const int ce = r * G::PXE + xe;  // E row r <-> B row r (both start at j-1)
        T dE3 = 0, dE2 = 0;
#pragma unroll
        for (int q = 1; q <= ME; ++q) {
          dE3 += c.ae[q - 1] * (e3[ce + q] - e3[ce - q + 1]);
          dE2 += c.ae[q - 1] * (e2[ce + q] - e2[ce - q + 1]);
        }
        const size_t g = base + (size_t)gj(r - 1) * m.n1 + gi(x - G::HLB);
        const T e1c = e1[ce], e2c = e2[ce], e3c = e3[ce];
        b1[p] = iB1[g] - (c.hy * (e3[ce + G::PXE] - e3c) - c.hz * (n2[ce] - e2c));
        b2[p] = iB2[g] - (c.hz * (n1[ce] - e1c) - dE3);
        b3[p] = iB3[g] - (dE2 - c.hy * (e1[ce + G::PXE] - e1c));
      }
    }
    __syncthreads();
    // ---- stage 2: E^{n+1}(ka) over the F buffer extent ----
    {
      const T* b1 = pB(ka, 0);
      const T* b2 = pB(ka, 1);
      const T* b3 = pB(ka, 2);
      const T* p1 = pB(ka - 1, 0);
      const T* p2 = pB(ka - 1, 1);
      const T* e1 = pE(ka, 0);
      const T* e2 = pE(ka, 1);
      const T* e3 = pE(ka, 2);
      T* f1 = pF(ka, 0);
      T* f2 = pF(ka, 1);
      T* f3 = pF(ka, 2);
      const bool out_plane = ka >= k0 && ka < kend;
      const int kg = gk(ka);
      const size_t base = (size_t)kg * plane_sz;
      for (int p = tid; p < G::SF; p += NT) {
        const int r = p / G::PXF;
        const int x = p - r * G::PXF;
        const int cb = (r + 1) * G::PXB + x + MB;             // B row of j is r+1
        const int ce = (r + 1) * G::PXE + x + (ME + MB - 1);  // E row of j is r+1
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
        const int ig = gi(x - G::HLF), jg = gj(r);
        const size_t g = base + (size_t)jg * m.n1 + ig;
        if (J1) {
          c1 -= c.dt * J1[g];
          c2 -= c.dt * J2[g];
          c3 -= c.dt * J3[g];
        }
        const T v1 = e1[ce] + c1, v2 = e2[ce] + c2, v3 = e3[ce] + c3;
        f1[p] = v1;
        f2[p] = v2;
        f3[p] = v3;
        const int xr = x - G::HLF;
        if (out_plane && xr >= 0 && xr < TX && r < TY && i0 + xr < m.n1 && j0 + r < m.n2) {
          oE1[g] = v1;
          oE2[g] = v2;
          oE3[g] = v3;
        }
      }
    }
    __syncthreads();
    // ---- stage 3: B^{n+1}(kk) on the output tile; refill E^n ----
    if (kk >= k0) {
      const T* f1 = pF(kk, 0);
      const T* f2 = pF(kk, 1);
      const T* f3 = pF(kk, 2);
      const T* g1 = pF(kk + 1, 0);
      const T* g2 = pF(kk + 1, 1);
      const T* b1 = pB(kk, 0);
      const T* b2 = pB(kk, 1);
      const T* b3 = pB(kk, 2);
      const size_t base = (size_t)gk(kk) * plane_sz;
      for (int p = tid; p < TX * TY; p += NT) {
        const int r = p / TX;
        const int x = p - r * TX;
        if (i0 + x >= m.n1 || j0 + r >= m.n2) continue;
        const int cf = r * G::PXF + x + G::HLF;
        const int cb = (r + 1) * G::PXB + x + G::HLB;
        T dF3 = 0, dF2 = 0;
#pragma unroll
        for (int q = 1; q <= ME; ++q) {
          dF3 += c.ae[q - 1] * (f3[cf + q] - f3[cf - q + 1]);
          dF2 += c.ae[q - 1] * (f2[cf + q] - f2[cf - q + 1]);
        }
        const T f1c = f1[cf], f2c = f2[cf], f3c = f3[cf];
        const size_t g = base + (size_t)(j0 + r) * m.n1 + (i0 + x);
        oB1[g] = b1[cb] - (c.hy * (f3[cf + G::PXF] - f3c) - c.hz * (g2[cf] - f2c));
        oB2[g] = b2[cb] - (c.hz * (g1[cf] - f1c) - dF3);
        oB3[g] = b3[cb] - (dF2 - c.hy * (f1[cf + G::PXF] - f1c));
      }
    }
    if (kk + 1 < kend) load_E(kk + 3);
    __syncthreads();
  }
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
  const int KZ = m.n3;
  auto kern = sweep_kernel<T, ME, MB, TX, TY, NT>;
  static_assert(G::lds_bytes <= 160 * 1024, "sweep tile exceeds LDS");
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::lds_bytes) !=
      hipSuccess)
    return set_error(PIC_EHIP, "sweep: cannot reserve %zu bytes of LDS", G::lds_bytes);
  const bool hasJ = J && J[0];
  hipLaunchKernelGGL(kern, dim3(tiles_x * tiles_y, (m.n3 + KZ - 1) / KZ), dim3(NT), G::lds_bytes, s,
                     (const T*)Ein[0], (const T*)Ein[1], (const T*)Ein[2], (const T*)Bin[0], (const T*)Bin[1],
                     (const T*)Bin[2], (const T*)(hasJ ? J[0] : nullptr), (const T*)(hasJ ? J[1] : nullptr),
                     (const T*)(hasJ ? J[2] : nullptr), (T*)Eout[0], (T*)Eout[1], (T*)Eout[2], (T*)Bout[0],
                     (T*)Bout[1], (T*)Bout[2], m, KZ, tiles_x, c);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "sweep launch failed");
}

template <typename T, int TXw, int TXn>
int dispatch_sweep(const Mesh& m, void* const Ein[3], void* const Bin[3], void* const J[3], void* const Eout[3],
                   void* const Bout[3], const double* CE, int ME, const double* CB, int MB, double dt,
                   hipStream_t s) {
  const int we = round_width(ME), wb = round_width(MB);
  const int w = we > wb ? we : wb;
  constexpr int TY = 4, NT = 512;
  // Ampere stencil either Yee (width 1) or padded to the Faraday width
  if (wb == 1) {
    switch (we) {
      case 1: return run_sweep<T, 1, 1, TXw, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
      case 2: return run_sweep<T, 2, 1, TXw, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
      case 4: return run_sweep<T, 4, 1, TXw, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
      case 8: return run_sweep<T, 8, 1, TXw, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
      default: return run_sweep<T, 16, 1, TXw, TY, NT>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
    }
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

int launch_advance_b(int prec, const Mesh& m, void* const E[3], void* const B[3], const double* CE, int ME,
                     double h, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return prec == PIC_FP64 ? dispatch_b<double>(m, E, B, CE, ME, h, s) : dispatch_b<float>(m, E, B, CE, ME, h, s);
}

int launch_sweep(int prec, const Mesh& m, void* const Ein[3], void* const Bin[3], void* const J[3],
                 void* const Eout[3], void* const Bout[3], const double* CE, int ME, const double* CB, int MB,
                 double dt, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (prec == PIC_FP64) return dispatch_sweep<double, 128, 64>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
  return dispatch_sweep<float, 128, 128>(m, Ein, Bin, J, Eout, Bout, CE, ME, CB, MB, dt, s);
}

int launch_advance_e(int prec, const Mesh& m, void* const E[3], void* const B[3], void* const J[3],
                     const double* CB, int MB, double dt, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return prec == PIC_FP64 ? dispatch_e<double>(m, E, B, J, CB, MB, dt, s)
                          : dispatch_e<float>(m, E, B, J, CB, MB, dt, s);
}

}  // namespace yeepic
