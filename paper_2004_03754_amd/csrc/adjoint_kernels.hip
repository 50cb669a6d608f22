// Adjoint (reverse-mode) kernels of one vacuum step (gfx950, FP64).
//
// Field step.  With the App. B operators, the transpose of the Faraday x1
// operator with coefficients C is minus the Ampere operator with the same C,
// and the transpose of a Yee forward difference is minus the backward one.
// Hence curl_E[C]^T = curl_B[C] and curl_B[C]^T = curl_E[C], and the reverse
// of  B' = B - dt/2 curl_E[C^E] E,  E' = E + dt curl_B[C^B] B',
//     B'' = B' - dt/2 curl_E[C^E] E'  is, on cotangents (lE, lB),
//   lE += -dt/2 curl_B[C^E] lB ;  lB += dt curl_E[C^B] lE ;
//   lE += -dt/2 curl_B[C^E] lB,
// three single-stage launches of the forward kernels with the coefficient
// roles swapped (api.hip).  This file holds the rest:
//
// * dL/dC_j.  C_j enters the x1 derivative through the differences
//   f_{i+j} - f_{i-j+1} (Faraday) or f_{i+j-1} - f_{i-j} (Ampere), so each
//   stage contributes a sum over cells of (cotangent of the stage output) x
//   (difference of the stage input): coef_partial + coef_finalize, a
//   deterministic two-pass reduction (per-block partial sums, then one block
//   per coefficient).
// * the particle adjoint: reverse of gather (App. A), the Boris or exact push
//   (Sec. 1) and the position update (Sec. 4.1).  The gather's reverse scatters the
//   cotangent of each interpolated field value into the field cotangent with
//   the same linear-shape weights, and adds the weights' x derivative to the
//   position cotangent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "particle_common.h"

namespace yeepic {
namespace {

using namespace pdev;

constexpr int kLags = PIC_MAX_M;  // every coefficient of the vector gets a gradient
constexpr int kCT = 256;           // threads of a coefficient-reduction block
constexpr int kCRW = 4;            // consecutive x1 cells per thread
constexpr int kRow = kCT * kCRW;   // cells of x1 per block
constexpr int kRows = 8;           // x1 rows each block accumulates before reducing

// Partial sums  acc_j = sum_i la_i D_j(fa)_i - lb_i D_j(fb)_i,  j = 1..kLags,
// over kRow cells of each of kRows consecutive x1 rows;  D_j f_i = f_{i+j} -
// f_{i-j+1} (FORM 0, Faraday) or f_{i+j-1} - f_{i-j} (FORM 1, Ampere).  Block
// b covers rows (b / nbx) * kRows .. + kRows (clipped to nrows) and cells
// [(b % nbx) kRow, + kRow) of each.  Each row segment of fa and fb is staged
// in LDS; a thread reads the 2 kLags + kCRW values around its kCRW cells once
// per array (16-byte reads), keeps its kLags sums in registers over the rows,
// and the block reduces them once.
template <int FORM>
__global__ __launch_bounds__(kCT) void coef_partial_kernel(const double* __restrict__ la,
                                                           const double* __restrict__ fa,
                                                           const double* __restrict__ lb,
                                                           const double* __restrict__ fb, int n1, int nbx,
                                                           int nrows, double* __restrict__ partial) {
  constexpr int NW = kCRW + 2 * kLags;  // window of one thread (index k: cell ib - kLags + k)
  __shared__ __align__(16) double sa[kRow + 2 * kLags];
  __shared__ __align__(16) double sb[kRow + 2 * kLags];
  __shared__ double red[kCT / 64][kLags];
  const int r0 = (blockIdx.x / nbx) * kRows;
  const int r1 = min(r0 + kRows, nrows);
  const int i0 = (blockIdx.x % nbx) * kRow;
  const int t = threadIdx.x;
  const int ib = i0 + kCRW * t;  // first cell of this thread
  double acc[kLags];
#pragma unroll
  for (int j = 0; j < kLags; ++j) acc[j] = 0.0;
  for (int rr = r0; rr < r1; ++rr) {
    const size_t row = (size_t)rr * n1;
    __syncthreads();  // the previous row's reads are done
    for (int q = t; q < kRow + 2 * kLags; q += kCT) {
      int ii = (i0 - kLags + q) % n1;
      ii += (ii < 0) ? n1 : 0;
      sa[q] = fa[row + ii];
      sb[q] = fb[row + ii];
    }
    __syncthreads();
    double a[kCRW], b[kCRW];
#pragma unroll
    for (int u = 0; u < kCRW; ++u) {
      a[u] = (ib + u < n1) ? la[row + ib + u] : 0.0;
      b[u] = (ib + u < n1) ? lb[row + ib + u] : 0.0;
    }
#pragma unroll
    for (int arr = 0; arr < 2; ++arr) {
      double w[NW];
      {
        typedef double v2 __attribute__((ext_vector_type(2)));
        const v2* src = reinterpret_cast<const v2*>((arr == 0 ? sa : sb) + kCRW * t);
#pragma unroll
        for (int k = 0; k < NW / 2; ++k) {
          const v2 v = src[k];
          w[2 * k] = v[0];
          w[2 * k + 1] = v[1];
        }
      }
#pragma unroll
      for (int u = 0; u < kCRW; ++u) {
        const double x = arr == 0 ? a[u] : -b[u];
#pragma unroll
        for (int j = 1; j <= kLags; ++j) {
          const int hi = FORM == 0 ? kLags + u + j : kLags + u + j - 1;
          const int lo = FORM == 0 ? kLags + u - j + 1 : kLags + u - j;
          acc[j - 1] += x * (w[hi] - w[lo]);
        }
      }
    }
  }
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int j = 0; j < kLags; ++j) {
    double v = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][j] = v;
  }
  __syncthreads();
  if (t < kLags) {
    double s = 0;
#pragma unroll
    for (int w = 0; w < kCT / 64; ++w) s += red[w][t];
    partial[(size_t)blockIdx.x * kLags + t] = s;
  }
}

// g[j] += scale * sum_b partial[b][j] for j < M; one block per coefficient.
__global__ __launch_bounds__(256) void coef_finalize_kernel(const double* __restrict__ partial, int nblocks,
                                                            double scale, double* __restrict__ g) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[(size_t)b * kLags + j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) g[j] += scale * (((red[0] + red[1]) + red[2]) + red[3]);
}

// ---------------------------------------------------------------------------
// Fused reverse of one 2D vacuum sweep for a Yee-width Ampere stencil
// (C^B = c e1: the proposed solver at dt = dx1/2), the stacked-plane batch of
// the differentiated workload.  With h = dt/2 and the cotangents (lE, lB) of
// (E^{n+1}, B^{n+1}):
//   lE1 = lE - h curl_B[C^E] lB        (reverse of the second B half step)
//   lB1 = lB + dt curl_E[C^B] lE1      (reverse of the E step)
//   lE0 = lE1 - h curl_B[C^E] lB1      (reverse of the first B half step)
// plus the three stages' lag products for dL/dC^E and dL/dC^B, in one pass.
// The mesh is cut into tiles of TX x TY cells of one plane.  For a tile, lB
// is staged with the halo the three stages need (2W - 1 .. 2W cells along
// x1, two rows below and one above) and lE with half of it; both are updated
// in LDS stage by stage, lE0 and lB1 are written out of place (neighbouring
// tiles read the inputs' halos), and the rows of E^{n+1}, B^{n+1/2} and E^n
// the products need are staged beside them.  The stencil arithmetic is that
// of advance_e_kernel / advance_b_kernel and the products those of
// coef_partial_kernel; only the order of the sums differs.
//
// The tiles take all of a CU's LDS, so one workgroup runs per CU; to keep
// HBM busy, the launch is persistent: a fixed grid of kAdjBlocks workgroups
// walks runs of consecutive tiles along x2 (work items), and a workgroup
// issues the loads of its next tile into registers before it computes the
// current one.  The lag products stay in registers over all of a
// workgroup's tiles and are reduced once, so the partial sums (and their
// order) depend on the mesh only.
// ---------------------------------------------------------------------------
constexpr int kAW = kLags;  // x1 reach of the wide (Faraday C^E) stencil
constexpr int kATX = 128, kATY = 8;
constexpr int kAPOS = kATX * kATY / 4;  // four-cell positions of a tile
constexpr int kANT = 2 * kAPOS;         // two threads per position: two waves per SIMD
constexpr int kARB = kATY + 3, kAXB = kATX + 4 * kAW;  // lB tile: rows j0-2 .., cols i0-2W ..
constexpr int kARE = kATY + 2, kAXE = kATX + 2 * kAW;  // lE tile: rows j0-1 .., cols i0-W ..
constexpr int kAXF = kATX + 2 * kAW;                   // forward-field rows: cols i0-W ..
constexpr size_t kALdsB = (size_t)3 * kARB * kAXB, kALdsE = (size_t)3 * kARE * kAXE;
constexpr size_t kALdsF = (size_t)6 * kATY * kAXF;
constexpr size_t kALds = (kALdsB + kALdsE + kALdsF) * sizeof(double);
constexpr int kAdjBlocks = 256;  // persistent workgroups: one per CU of an MI355X

struct Coef16 {
  double c[kAW];
};

struct AdjPlane {
  const double* li[6];   // lE1 lE2 lE3 lB1 lB2 lB3 at t^{n+1} (read)
  double* lo[6];         // the same at t^n (written)
  const double* fw[6];   // E^{n+1}_2, E^{n+1}_3, B^{n+1/2}_2, B^{n+1/2}_3, E^n_2, E^n_3
};

// Work items: item w is strip w % strips (x1 cells strip*TX ..), chunk
// (w / strips) % ysplit of the strip's nty tile rows (tpb tiles from
// chunk*tpb, clipped to nty; never empty), plane w / (strips * ysplit).
struct AdjWork {
  int strips, ysplit, tpb, nty, nwork;
};

struct AdjTile {
  int item, y, yend, i0, k;
};

__device__ __forceinline__ AdjTile adj_item(const AdjWork& W, int w) {
  AdjTile c;
  c.item = w;
  const int strip = w % W.strips, rest = w / W.strips;
  c.y = (rest % W.ysplit) * W.tpb;
  c.yend = min(W.nty, c.y + W.tpb);
  c.i0 = strip * kATX;
  c.k = rest / W.ysplit;
  return c;
}

// Periodic wrap of a tile row or column index that lies within [-n, 2n):
// tiles start inside the mesh and their halos reach at most one period out
// when n1 >= kAXB and n2 >= kATY + 3 (checked by the launcher, which falls
// back to the full remainder otherwise).
template <bool kNear>
__device__ __forceinline__ int wrap_index(int i, int n) {
  if (kNear) {
    i += i < 0 ? n : 0;
    return i - (i >= n ? n : 0);
  }
  i %= n;
  return i + (i < 0 ? n : 0);
}

// Loads a rows x cols window of one plane of ``src`` (rows from j, cols
// from i, periodic) into v[]: element q = t + it * kANT of the window, row
// q / cols, col q % cols.  All loads of a call are issued before any is used.
template <bool kNear, int kRows, int kCols>
__device__ __forceinline__ void load_window(const double* __restrict__ src, const Mesh& m, int k, int j, int i,
                                            int t, double* v) {
  constexpr int kN = (kRows * kCols + kANT - 1) / kANT;
  const double* __restrict__ plane = src + (size_t)k * m.n2 * m.n1;  // uniform; in-plane offsets fit 32 bits
#pragma unroll
  for (int it = 0; it < kN; ++it) {
    const int q = t + it * kANT;
    if (kRows * kCols % kANT == 0 || q < kRows * kCols) {
      const int r = q / kCols, x = q % kCols;
      const int jj = wrap_index<kNear>(j + r, m.n2), ii = wrap_index<kNear>(i + x, m.n1);
      v[it] = plane[(unsigned)(jj * m.n1 + ii)];
    }
  }
}

// Lag products of four cells with one staged forward row: for j = 1..W,
//   acc[j-1] += sum_u x[u] D_j f,  D_j f = f_{i+j} - f_{i-j+1} (Faraday,
//   FORM 0) or f_{i+j-1} - f_{i-j} (Ampere, FORM 1), cell i = first + u,
// w0 the row from W cells left of the first cell (2W + 4 values).
template <int FORM>
__device__ __forceinline__ void lag_products(const double* __restrict__ w0, const double x[4], double acc[kAW]) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  double w[2 * kAW + 4];
  const v2* src = reinterpret_cast<const v2*>(w0);
#pragma unroll
  for (int k = 0; k < kAW + 2; ++k) {
    const v2 v = src[k];
    w[2 * k] = v[0];
    w[2 * k + 1] = v[1];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
#pragma unroll
    for (int j = 1; j <= kAW; ++j)
      acc[j - 1] += FORM == 0 ? x[u] * (w[kAW + u + j] - w[kAW + u - j + 1])
                              : x[u] * (w[kAW + u + j - 1] - w[kAW + u - j]);
  }
}

template <int kRows, int kCols>
__device__ __forceinline__ void store_window(double* dst, int t, const double* v) {
  constexpr int kN = (kRows * kCols + kANT - 1) / kANT;
#pragma unroll
  for (int it = 0; it < kN; ++it) {
    const int q = t + it * kANT;
    if (kRows * kCols % kANT == 0 || q < kRows * kCols) dst[q] = v[it];
  }
}

// The wide x1 stage on four consecutive cells of one LDS row: for u < 4,
//   out[u] = sum_q a_q (w[W + u + q - 1] - w[W + u - q]),
// w the 2W + 3 values of the source row starting W cells left of the first.
__device__ __forceinline__ void wide4(const double* __restrict__ w0, const Coef16& a, double out[4]) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  double w[2 * kAW + 4];
  const v2* src = reinterpret_cast<const v2*>(w0);
#pragma unroll
  for (int k = 0; k < kAW + 2; ++k) {
    const v2 v = src[k];
    w[2 * k] = v[0];
    w[2 * k + 1] = v[1];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    double s = 0.0;
#pragma unroll
    for (int q = 1; q <= kAW; ++q) s += a.c[q - 1] * (w[kAW + u + q - 1] - w[kAW + u - q]);
    out[u] = s;
  }
}

// Sum over a workgroup's threads of acc[0..W) through LDS: each thread
// stores its values (column t of the [W][kRS] table ``tab``), kTS threads
// sum each row's values in strided groups, and thread t < W returns the sum
// of row t (others return 0).  Callers have synchronised before the table is
// written; it is free again on return.
constexpr int kTS = kANT / kAW;  // threads summing one row (a half-wave reads one row: no bank conflicts)
constexpr int kRS = kANT + 16;   // padded row
static_assert(kTS * kAW == kANT && kANT % kTS == 0 && (kANT / kTS) % 2 == 0, "threads per accumulator row");
static_assert((size_t)kAW * kRS <= kALdsB + kALdsE, "the tile-sum table fits over the cotangent tiles");
__device__ __forceinline__ double tile_sum(const double acc[kAW], double* tab, double* grp, int t) {
#pragma unroll
  for (int j = 0; j < kAW; ++j) tab[j * kRS + t] = acc[j];
  __syncthreads();
  {
    const int row = t / kTS, part = t % kTS;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 0; i < kANT / kTS; i += 2) {
      s0 += tab[row * kRS + i * kTS + part];
      s1 += tab[row * kRS + (i + 1) * kTS + part];
    }
    grp[row * kTS + part] = s0 + s1;
  }
  __syncthreads();
  double s = 0.0;
  if (t < kAW) {
#pragma unroll
    for (int w = 0; w < kTS; ++w) s += grp[t * kTS + w];
  }
  return s;
}

template <bool kNear>
__global__ __launch_bounds__(kANT) void adjoint_sweep2d_kernel(AdjPlane P, Mesh m, AdjWork W, Coef16 a, double ty,
                                                               double b1, double hy, double* __restrict__ partial) {
  extern __shared__ __align__(16) double lds[];
  double* sB = lds;                      // [3][kARB][kAXB]
  double* sE = lds + kALdsB;             // [3][kARE][kAXE]
  double* sF = lds + kALdsB + kALdsE;    // [6][kATY][kAXF]: rows j0 .., cols i0-W ..
  const int t = threadIdx.x;
  auto B = [&](int c, int r, int x) -> double& { return sB[((size_t)c * kARB + r) * kAXB + x]; };
  auto Ev = [&](int c, int r, int x) -> double& { return sE[((size_t)c * kARE + r) * kAXE + x]; };
  // a tile's loads into registers: the cotangents lB (rows j0-2 .., cols
  // i0-2W ..) and lE (rows j0-1 .., cols i0-W ..), issued a tile ahead, and
  // the forward rows of the lag products (rows j0 .., cols i0-W ..), issued
  // at the start of the tile and stored once the three stages are done
  constexpr int kPB = (kARB * kAXB + kANT - 1) / kANT, kPE = (kARE * kAXE + kANT - 1) / kANT;
  constexpr int kPF = (kATY * kAXF + kANT - 1) / kANT;
  double vB[3][kPB], vE[3][kPE], vF[6][kPF];
  auto load_tile = [&](const AdjTile& c) {
    const int j0 = c.y * kATY;
#pragma unroll
    for (int q = 0; q < 3; ++q) load_window<kNear, kARB, kAXB>(P.li[3 + q], m, c.k, j0 - 2, c.i0 - 2 * kAW, t, vB[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) load_window<kNear, kARE, kAXE>(P.li[q], m, c.k, j0 - 1, c.i0 - kAW, t, vE[q]);
  };
  auto load_rows = [&](const AdjTile& c) {
#pragma unroll
    for (int q = 0; q < 6; ++q) load_window<kNear, kATY, kAXF>(P.fw[q], m, c.k, c.y * kATY, c.i0 - kAW, t, vF[q]);
  };
  double* tab = sB;  // [W][kRS] tile-sum table, over the cotangent tiles once their products are taken
  __shared__ double grp[kAW * kTS];
  double totE = 0.0, totB = 0.0;  // thread t < W: the workgroup's sums of lag t + 1
  // this thread's four-cell position (row tr, group g) and half of the work
  // at that position
  const int pos = t % kAPOS, half = t / kAPOS;
  const int tr = pos / (kATX / 4), g = pos % (kATX / 4);
  AdjTile cur = adj_item(W, blockIdx.x);  // gridDim.x <= nwork
  load_tile(cur);
  for (;;) {
#pragma unroll
    for (int q = 0; q < 3; ++q) store_window<kARB, kAXB>(sB + (size_t)q * kARB * kAXB, t, vB[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) store_window<kARE, kAXE>(sE + (size_t)q * kARE * kAXE, t, vE[q]);
    __syncthreads();
    load_rows(cur);
    // the next tile of this workgroup: the next along x2 in the item, else
    // the first of its next item; its loads fly while this one is computed
    AdjTile nxt = cur;
    if (++nxt.y >= nxt.yend) nxt = adj_item(W, cur.item + gridDim.x);
    const bool more = nxt.item < W.nwork;
    if (more) load_tile(nxt);
    const int i0 = cur.i0, j0 = cur.y * kATY, k = cur.k;
    const int gi = i0 + 4 * g, gj = j0 + tr;
    bool own[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) own[u] = gi + u < m.n1 && gj < m.n2;
    // the input lB at the interior cells (products with E'2 and E'3, taken
    // by the first half)
    double lb2[4], lb3[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      lb2[u] = own[u] ? B(1, tr + 2, 2 * kAW + 4 * g + u) : 0.0;
      lb3[u] = own[u] ? B(2, tr + 2, 2 * kAW + 4 * g + u) : 0.0;
    }
    // lE1 = lE - h curl_B[C^E] lB on the whole lE tile, four cells at a
    // time: item q < kNE updates lE_1 and lE_2 (wide stencil of lB_3), item
    // q >= kNE lE_3 (wide stencil of lB_2) of the same four cells
    constexpr int kNE = kARE * (kAXE / 4);
    for (int q = t; q < 2 * kNE; q += kANT) {
      const int q1 = q < kNE ? q : q - kNE;
      const int re = q1 / (kAXE / 4), ce = 4 * (q1 % (kAXE / 4));
      const int rb = re + 1, cb = ce + kAW;
      double d[4];
      wide4(&B(q < kNE ? 2 : 1, rb, ce), a, d);
      if (q < kNE) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          Ev(0, re, ce + u) += ty * (B(2, rb, cb + u) - B(2, rb - 1, cb + u));
          Ev(1, re, ce + u) -= d[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) Ev(2, re, ce + u) += d[u] - ty * (B(0, rb, cb + u) - B(0, rb - 1, cb + u));
      }
    }
    __syncthreads();
    // lB1 = lB + dt curl_E[c e1] lE1 on rows j0-1 .. j0+TY-1, cols i0-W .. i0+TX+W-2
    constexpr int kNB = kATX + 2 * kAW - 1;
    for (int q = t; q < (kATY + 1) * kNB; q += kANT) {
      const int rb = 1 + q / kNB, cb = kAW + q % kNB;
      const int re = rb - 1, ce = cb - kAW;
      B(0, rb, cb) -= hy * (Ev(2, re + 1, ce) - Ev(2, re, ce));
      B(1, rb, cb) += b1 * (Ev(2, re, ce + 1) - Ev(2, re, ce));
      B(2, rb, cb) -= b1 * (Ev(1, re, ce + 1) - Ev(1, re, ce)) - hy * (Ev(0, re + 1, ce) - Ev(0, re, ce));
    }
    __syncthreads();
    // lE0 = lE1 - h curl_B[C^E] lB1 on the interior; write lE0 and lB1.  The
    // first half takes lE0_1, lE0_2 (wide stencil of lB1_3), lB1_1, lB1_3;
    // the second lE0_3 (wide stencil of lB1_2) and lB1_2.
    const int re = tr + 1, ce = kAW + 4 * g, rb = re + 1, cb = ce + kAW;
    {
      double d[4];
      wide4(&B(half == 0 ? 2 : 1, rb, ce), a, d);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!own[u]) continue;
        const size_t o = ((size_t)k * m.n2 + gj) * m.n1 + gi + u;
        if (half == 0) {
          P.lo[0][o] = Ev(0, re, ce + u) + ty * (B(2, rb, cb + u) - B(2, rb - 1, cb + u));
          P.lo[1][o] = Ev(1, re, ce + u) - d[u];
          P.lo[3][o] = B(0, rb, cb + u);
          P.lo[5][o] = B(2, rb, cb + u);
        } else {
          P.lo[2][o] = Ev(2, re, ce + u) + d[u] - ty * (B(0, rb, cb + u) - B(0, rb - 1, cb + u));
          P.lo[4][o] = B(1, rb, cb + u);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) store_window<kATY, kAXF>(sF + (size_t)q * kATY * kAXF, t, vF[q]);
    __syncthreads();
    // lag products of the interior cells, one form at a time: Faraday
    // (dL/dC^E) from E'2, E'3 with the input lB (first half) and E^n2, E^n3
    // with lB1 (second half, from sB); Ampere (dL/dC^B) from B'2 (first
    // half) and B'3 (second half) with lE1 (from sE, read before the
    // Faraday table covers it).  Window of 4 cells at i: staged cols
    // 4g .. 4g + 35 = x1 i - W .. i + W + 3 of row tr.
    auto frow = [&](int arr) { return &sF[((size_t)arr * kATY + tr) * kAXF + 4 * g]; };
    double xa[4];  // lE1_3 (first half) or -lE1_2 (second half) at the interior cells
#pragma unroll
    for (int u = 0; u < 4; ++u) xa[u] = own[u] ? (half == 0 ? Ev(2, re, ce + u) : -Ev(1, re, ce + u)) : 0.0;
    {
      double acc[kAW], x0[4], x1[4];
#pragma unroll
      for (int j = 0; j < kAW; ++j) acc[j] = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x0[u] = half == 0 ? -lb3[u] : (own[u] ? -B(2, rb, cb + u) : 0.0);  // with E'2 / E^n2
        x1[u] = half == 0 ? lb2[u] : (own[u] ? B(1, rb, cb + u) : 0.0);    // with E'3 / E^n3
      }
      lag_products<0>(frow(half == 0 ? 0 : 4), x0, acc);
      lag_products<0>(frow(half == 0 ? 1 : 5), x1, acc);
      __syncthreads();  // sB and sE are free: they hold the table
      totE += tile_sum(acc, tab, grp, t);
    }
    {
      double acc[kAW];
#pragma unroll
      for (int j = 0; j < kAW; ++j) acc[j] = 0.0;
      lag_products<1>(frow(half == 0 ? 2 : 3), xa, acc);
      totB += tile_sum(acc, tab, grp, t);
    }
    if (!more) break;
    cur = nxt;
  }
  if (t < kAW) {
    partial[(size_t)blockIdx.x * 2 * kAW + t] = totE;
    partial[(size_t)blockIdx.x * 2 * kAW + kAW + t] = totB;
  }
}

// gE[j] += sE * sum_b partial[b][j], gB[j] += sB * sum_b partial[b][W + j]
__global__ __launch_bounds__(256) void coef_finalize2_kernel(const double* __restrict__ partial, int64_t nblocks,
                                                             int M, double sE, double sBv, double* __restrict__ gE,
                                                             double* __restrict__ gB) {
  __shared__ double red[4];
  const int j = blockIdx.x % M, which = blockIdx.x / M;
  const int col = which * kAW + j;
  double s = 0;
  for (int64_t b = threadIdx.x; b < nblocks; b += 256) s += partial[b * 2 * kAW + col];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double v = ((red[0] + red[1]) + red[2]) + red[3];
    if (which == 0)
      gE[j] += sE * v;
    else
      gB[j] += sBv * v;
  }
}

// Reverse of boris(): u is the input momentum, lun the cotangent of the
// output momentum; returns the cotangents of u, E and B.
__device__ __forceinline__ void boris_vjp(const double u[3], const double E[3], const double B[3], double qm,
                                          double dt, const double lun[3], double lu[3], double lE[3],
                                          double lB[3]) {
  const double eps = 0.5 * qm * dt;
  const double um[3] = {u[0] + eps * E[0], u[1] + eps * E[1], u[2] + eps * E[2]};
  const double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  const double eg = eps / g;
  const double t[3] = {eg * B[0], eg * B[1], eg * B[2]};
  const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  const double f = 2.0 / (1.0 + tt);
  const double s[3] = {f * t[0], f * t[1], f * t[2]};
  const double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                        um[2] + (um[0] * t[1] - um[1] * t[0])};
  // u' = um + up x s + eps E
  double lum[3] = {lun[0], lun[1], lun[2]};
  const double lup[3] = {s[1] * lun[2] - s[2] * lun[1], s[2] * lun[0] - s[0] * lun[2],
                         s[0] * lun[1] - s[1] * lun[0]};  // s x lun
  const double ls[3] = {lun[1] * up[2] - lun[2] * up[1], lun[2] * up[0] - lun[0] * up[2],
                        lun[0] * up[1] - lun[1] * up[0]};  // lun x up
  // s = f t, f = 2/(1 + t.t)
  const double st = t[0] * ls[0] + t[1] * ls[1] + t[2] * ls[2];
  double lt[3];
  for (int d = 0; d < 3; ++d) lt[d] = f * ls[d] - f * f * st * t[d];
  // up = um + um x t
  lum[0] += lup[0] + (t[1] * lup[2] - t[2] * lup[1]);
  lum[1] += lup[1] + (t[2] * lup[0] - t[0] * lup[2]);
  lum[2] += lup[2] + (t[0] * lup[1] - t[1] * lup[0]);
  lt[0] += lup[1] * um[2] - lup[2] * um[1];
  lt[1] += lup[2] * um[0] - lup[0] * um[2];
  lt[2] += lup[0] * um[1] - lup[1] * um[0];
  // t = (eps/g) B,  g = sqrt(1 + um.um)
  const double bl = B[0] * lt[0] + B[1] * lt[1] + B[2] * lt[2];
  const double lg = -(eg / g) * bl;
  for (int d = 0; d < 3; ++d) {
    lB[d] = eg * lt[d];
    lum[d] += (lg / g) * um[d];
  }
  // um = u + eps E, and the last half kick
  for (int d = 0; d < 3; ++d) {
    lu[d] = lum[d];
    lE[d] = eps * (lum[d] + lun[d]);
  }
}

// ---------------------------------------------------------------------------
// Reverse of the exact push, by forward-mode differentiation one input
// direction at a time (9 directions: u, E, B).  A dual number carries a value
// and one directional derivative; the exponential's coefficients are
// re-evaluated in dual arithmetic along the same branches as the forward.
// The root tau* of t(tau) = dt depends on the inputs implicitly:
// d tau*/d theta = -(d t/d theta at fixed tau)/gamma(tau*).
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual dsqrt(Dual a) {
  const double r = sqrt(a.v);
  return {r, r > 0 ? a.d / (2 * r) : 0.0};
}
__device__ __forceinline__ Dual dsinh(Dual a) { return {sinh(a.v), cosh(a.v) * a.d}; }
__device__ __forceinline__ Dual dsin(Dual a) { return {sin(a.v), cos(a.v) * a.d}; }

struct ExpCoefD {
  Dual a0, a1, a2, a3, A1, A3;
};

// exp_coef in dual arithmetic (same branches, chosen by the values)
__device__ __forceinline__ ExpCoefD exp_coef_dual(Dual k2, Dual w2, Dual tau) {
  const Dual t2 = tau * tau;
  const Dual X = k2 * t2, Y = w2 * t2;
  ExpCoefD e;
  if (X.v <= 1.0 && Y.v <= 1.0) {
    const Dual Z = -Y;
    Dual h = {1.0, 0.0}, zk = {1.0, 0.0};
    Dual G[7];
    for (int m = 0; m < 7; ++m) G[m] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 14; ++k) {
      G[2] = G[2] + kInvFact.v[2 * k + 2] * h;
      G[3] = G[3] + kInvFact.v[2 * k + 3] * h;
      G[4] = G[4] + kInvFact.v[2 * k + 4] * h;
      G[5] = G[5] + kInvFact.v[2 * k + 5] * h;
      G[6] = G[6] + kInvFact.v[2 * k + 6] * h;
      zk = zk * Z;
      h = X * h + zk;
    }
    const Dual XY = X * Y;
    e.a0 = XY * G[4] + 1.0;
    e.a1 = tau * (XY * G[5] + 1.0);
    e.a2 = t2 * G[2];
    e.a3 = t2 * tau * G[3];
    e.A1 = t2 * (XY * G[6] + 0.5);
    e.A3 = t2 * t2 * G[4];
    return e;
  }
  Dual sh, ch1, sn, cs1;
  if (sqrt(k2.v) * fabs(tau.v) < 1e-4) {
    sh = tau * (X * (1.0 / 6.0) * (X * (1.0 / 20.0) + 1.0) + 1.0);
    ch1 = 0.5 * t2 * (X * (1.0 / 12.0) * (X * (1.0 / 30.0) + 1.0) + 1.0);
  } else {
    const Dual kap = dsqrt(k2);
    sh = dsinh(kap * tau) / kap;
    const Dual s = dsinh(0.5 * (kap * tau)) / kap;
    ch1 = 2.0 * (s * s);
  }
  if (sqrt(w2.v) * fabs(tau.v) < 1e-4) {
    sn = tau * (-(Y * (1.0 / 6.0) * (-(Y * (1.0 / 20.0)) + 1.0)) + 1.0);
    cs1 = 0.5 * t2 * (-(Y * (1.0 / 12.0) * (-(Y * (1.0 / 30.0)) + 1.0)) + 1.0);
  } else {
    const Dual om = dsqrt(w2);
    sn = dsin(om * tau) / om;
    const Dual s = dsin(0.5 * (om * tau)) / om;
    cs1 = 2.0 * (s * s);
  }
  const Dual inv = Dual{1.0, 0.0} / (k2 + w2);
  const Dual chx = k2 * ch1 + 1.0, cy = -(w2 * cs1) + 1.0;
  e.a0 = (w2 * chx + k2 * cy) * inv;
  e.a1 = (w2 * sh + k2 * sn) * inv;
  e.a2 = (k2 * ch1 + w2 * cs1) * inv;
  e.a3 = (sh - sn) * inv;
  e.A1 = (w2 * ch1 + k2 * cs1) * inv;
  e.A3 = (ch1 - cs1) * inv;
  return e;
}

__device__ __forceinline__ void apply_F_dual(const Dual E[3], const Dual B[3], double qm, const Dual v[4], Dual o[4]) {
  o[0] = qm * (E[0] * v[1] + E[1] * v[2] + E[2] * v[3]);
  o[1] = qm * (E[0] * v[0] + B[2] * v[2] - B[1] * v[3]);
  o[2] = qm * (E[1] * v[0] - B[2] * v[1] + B[0] * v[3]);
  o[3] = qm * (E[2] * v[0] + B[1] * v[1] - B[0] * v[2]);
}

// Reverse of analytic(): u is the input momentum, lun the cotangent of the
// output momentum; returns the cotangents of u, E and B.
__device__ void analytic_vjp(const double u[3], const double E[3], const double B[3], double qm, double dt,
                             const double lun[3], double lu[3], double lE[3], double lB[3], int max_iter) {
  ExactState st;
  bool conv;  // the forward recompute of the same push counts a failed solve
  const double tau_s = analytic_solve(u, E, B, qm, dt, st, max_iter, conv);
  for (int dir = 0; dir < 9; ++dir) {
    Dual ud[3], Ed[3], Bd[3];
    for (int c = 0; c < 3; ++c) {
      ud[c] = {u[c], dir == c ? 1.0 : 0.0};
      Ed[c] = {E[c], dir == 3 + c ? 1.0 : 0.0};
      Bd[c] = {B[c], dir == 6 + c ? 1.0 : 0.0};
    }
    const Dual E2 = Ed[0] * Ed[0] + Ed[1] * Ed[1] + Ed[2] * Ed[2];
    const Dual B2 = Bd[0] * Bd[0] + Bd[1] * Bd[1] + Bd[2] * Bd[2];
    const Dual EB = Ed[0] * Bd[0] + Ed[1] * Bd[1] + Ed[2] * Bd[2];
    const double q2 = qm * qm;
    const Dual P = 0.5 * (E2 - B2);
    // Q = sqrt(P^2 + EB^2) is homogeneous of degree 2 in the fields: its
    // derivative vanishes where it does
    const Dual Q = dsqrt(P * P + EB * EB);
    Dual k2, w2;
    if (P.v >= 0) {
      k2 = q2 * (P + Q);
      w2 = (P + Q).v > 0 ? q2 * ((EB * EB) / (P + Q)) : Dual{0.0, 0.0};
    } else {
      w2 = q2 * (Q - P);
      k2 = q2 * ((EB * EB) / (Q - P));
    }
    Dual U0[4], V1[4], V2[4], V3[4];
    U0[0] = dsqrt(ud[0] * ud[0] + ud[1] * ud[1] + ud[2] * ud[2] + 1.0);
    for (int c = 0; c < 3; ++c) U0[c + 1] = ud[c];
    apply_F_dual(Ed, Bd, qm, U0, V1);
    apply_F_dual(Ed, Bd, qm, V1, V2);
    apply_F_dual(Ed, Bd, qm, V2, V3);
    // lab time and gamma at the root with tau held fixed, then the root's
    // implicit derivative
    const ExpCoefD e0 = exp_coef_dual(k2, w2, Dual{tau_s, 0.0});
    const Dual t = e0.a1 * U0[0] + e0.A1 * V1[0] + e0.a3 * V2[0] + e0.A3 * V3[0];
    const Dual g = e0.a0 * U0[0] + e0.a1 * V1[0] + e0.a2 * V2[0] + e0.a3 * V3[0];
    const Dual tau = {tau_s, -t.d / g.v};
    const ExpCoefD e = exp_coef_dual(k2, w2, tau);
    double acc = 0;
    for (int c = 0; c < 3; ++c) {
      const Dual o = e.a0 * U0[c + 1] + e.a1 * V1[c + 1] + e.a2 * V2[c + 1] + e.a3 * V3[c + 1];
      acc += o.d * lun[c];
    }
    if (dir < 3)
      lu[dir] = acc;
    else if (dir < 6)
      lE[dir - 3] = acc;
    else
      lB[dir - 6] = acc;
  }
}

// Reverse of one 3D linear-shape interpolation: scatter lv W into lf at the
// eight nodes and add lv dv/dx to lx.
__device__ __forceinline__ void interp3_vjp(const double* __restrict__ f, double* lf, const Axis& a,
                                            const Axis& b, const Axis& c, const Mesh& m, double lv,
                                            double lx[3]) {
  if (lv == 0.0) return;
  const size_t pl = (size_t)m.n1 * m.n2;
  const size_t r00 = (size_t)c.i0 * pl + (size_t)b.i0 * m.n1;
  const size_t r01 = (size_t)c.i0 * pl + (size_t)b.i1 * m.n1;
  const size_t r10 = (size_t)c.i1 * pl + (size_t)b.i0 * m.n1;
  const size_t r11 = (size_t)c.i1 * pl + (size_t)b.i1 * m.n1;
  const double f000 = f[r00 + a.i0], f001 = f[r00 + a.i1];
  const double f010 = f[r01 + a.i0], f011 = f[r01 + a.i1];
  const double f100 = f[r10 + a.i0], f101 = f[r10 + a.i1];
  const double f110 = f[r11 + a.i0], f111 = f[r11 + a.i1];
  lx[0] += lv * m.idx1 *
           (c.w0 * (b.w0 * (f001 - f000) + b.w1 * (f011 - f010)) + c.w1 * (b.w0 * (f101 - f100) + b.w1 * (f111 - f110)));
  lx[1] += lv * m.idx2 *
           (c.w0 * (a.w0 * (f010 - f000) + a.w1 * (f011 - f001)) + c.w1 * (a.w0 * (f110 - f100) + a.w1 * (f111 - f101)));
  lx[2] += lv * m.idx3 *
           (b.w0 * (a.w0 * (f100 - f000) + a.w1 * (f101 - f001)) + b.w1 * (a.w0 * (f110 - f010) + a.w1 * (f111 - f011)));
  atomic_add(&lf[r00 + a.i0], lv * c.w0 * b.w0 * a.w0);
  atomic_add(&lf[r00 + a.i1], lv * c.w0 * b.w0 * a.w1);
  atomic_add(&lf[r01 + a.i0], lv * c.w0 * b.w1 * a.w0);
  atomic_add(&lf[r01 + a.i1], lv * c.w0 * b.w1 * a.w1);
  atomic_add(&lf[r10 + a.i0], lv * c.w1 * b.w0 * a.w0);
  atomic_add(&lf[r10 + a.i1], lv * c.w1 * b.w0 * a.w1);
  atomic_add(&lf[r11 + a.i0], lv * c.w1 * b.w1 * a.w0);
  atomic_add(&lf[r11 + a.i1], lv * c.w1 * b.w1 * a.w1);
}

// 2D form: four nodes in the particle's plane (``f`` and ``lf`` already
// point at it).
__device__ __forceinline__ void interp2_vjp(const double* __restrict__ f, double* lf, const Axis& a,
                                            const Axis& b, const Mesh& m, double lv, double lx[3]) {
  if (lv == 0.0) return;
  const size_t r0 = (size_t)b.i0 * m.n1, r1 = (size_t)b.i1 * m.n1;
  const double f00 = f[r0 + a.i0], f01 = f[r0 + a.i1], f10 = f[r1 + a.i0], f11 = f[r1 + a.i1];
  lx[0] += lv * m.idx1 * (b.w0 * (f01 - f00) + b.w1 * (f11 - f10));
  lx[1] += lv * m.idx2 * (a.w0 * (f10 - f00) + a.w1 * (f11 - f01));
  atomic_add(&lf[r0 + a.i0], lv * b.w0 * a.w0);
  atomic_add(&lf[r0 + a.i1], lv * b.w0 * a.w1);
  atomic_add(&lf[r1 + a.i0], lv * b.w1 * a.w0);
  atomic_add(&lf[r1 + a.i1], lv * b.w1 * a.w1);
}

struct AdjFields {
  const double* f[6];  // forward E1 E2 E3 B1 B2 B3 at t^n
  double* l[6];        // their cotangents (accumulated)
};

// One thread per particle: reverse of gather + Boris + position update.
// In: x^n, u^{n-1/2}, lx = dL/dx^{n+1}, lu = dL/du^{n+1/2}.
// Out: lx = dL/dx^n, lu = dL/du^{n-1/2}; field cotangents accumulated.
template <int NDIM, int PUSH>
__global__ __launch_bounds__(256) void adjoint_push_kernel(AdjFields F, Mesh m, const double* __restrict__ x1,
                                                            const double* __restrict__ x2,
                                                            const double* __restrict__ x3,
                                                            const double* __restrict__ u1,
                                                            const double* __restrict__ u2,
                                                            const double* __restrict__ u3, double* __restrict__ lx1,
                                                            double* __restrict__ lx2, double* __restrict__ lx3,
                                                            double* __restrict__ lu1, double* __restrict__ lu2,
                                                            double* __restrict__ lu3, int64_t np, double qm,
                                                            double dt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const bool stacked = NDIM == 2 && m.n3 > 1;
  const double x[3] = {x1[p], x2[p], (NDIM == 3 || stacked) ? x3[p] : 0.0};
  const double u[3] = {u1[p], u2[p], u3[p]};
  double E[3], B[3];
  gather6<double, NDIM>(F.f[0], F.f[1], F.f[2], F.f[3], F.f[4], F.f[5], m, x, E, B);
  // forward push (recomputed) for the position update's Jacobian
  double un[3] = {u[0], u[1], u[2]};
  if (PUSH == PIC_PUSH_BORIS)
    boris(un, E, B, qm, dt);
  else
    analytic(un, E, B, qm, dt, m);
  const double gn = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
  double lx[3] = {lx1[p], lx2[p], NDIM == 3 ? lx3[p] : 0.0};
  // x_d' = x_d + dt u'_d/gamma' for d < NDIM (the wrap is a constant shift)
  double ux = 0;
  for (int d = 0; d < NDIM; ++d) ux += un[d] * lx[d];
  const double ig = dt / gn, ig3 = ig / (gn * gn);
  double lun[3] = {lu1[p], lu2[p], lu3[p]};
  for (int d = 0; d < 3; ++d) lun[d] += (d < NDIM ? ig * lx[d] : 0.0) - ig3 * un[d] * ux;
  double lu[3], lE[3], lB[3];
  if (PUSH == PIC_PUSH_BORIS)
    boris_vjp(u, E, B, qm, dt, lun, lu, lE, lB);
  else
    analytic_vjp(u, E, B, qm, dt, lun, lu, lE, lB, m.exact_iters);
  // reverse of the gather
  const Axis a0 = axis(x[0], m.idx1, 0.0, m.n1), ah = axis(x[0], m.idx1, 0.5, m.n1);
  const Axis b0 = axis(x[1], m.idx2, 0.0, m.n2), bh = axis(x[1], m.idx2, 0.5, m.n2);
  if (NDIM == 3) {
    const Axis c0 = axis(x[2], m.idx3, 0.0, m.n3), ch = axis(x[2], m.idx3, 0.5, m.n3);
    interp3_vjp(F.f[0], F.l[0], ah, b0, c0, m, lE[0], lx);
    interp3_vjp(F.f[1], F.l[1], a0, bh, c0, m, lE[1], lx);
    interp3_vjp(F.f[2], F.l[2], a0, b0, ch, m, lE[2], lx);
    interp3_vjp(F.f[3], F.l[3], a0, bh, ch, m, lB[0], lx);
    interp3_vjp(F.f[4], F.l[4], ah, b0, ch, m, lB[1], lx);
    interp3_vjp(F.f[5], F.l[5], ah, bh, c0, m, lB[2], lx);
    lx3[p] = lx[2];
  } else {
    const size_t off = plane_offset(m, x[2]);
    interp2_vjp(F.f[0] + off, F.l[0] + off, ah, b0, m, lE[0], lx);
    interp2_vjp(F.f[1] + off, F.l[1] + off, a0, bh, m, lE[1], lx);
    interp2_vjp(F.f[2] + off, F.l[2] + off, a0, b0, m, lE[2], lx);
    interp2_vjp(F.f[3] + off, F.l[3] + off, a0, bh, m, lB[0], lx);
    interp2_vjp(F.f[4] + off, F.l[4] + off, ah, b0, m, lB[1], lx);
    interp2_vjp(F.f[5] + off, F.l[5] + off, ah, bh, m, lB[2], lx);
  }
  lx1[p] = lx[0];
  lx2[p] = lx[1];
  lu1[p] = lu[0];
  lu2[p] = lu[1];
  lu3[p] = lu[2];
}

}  // namespace

int coef_partial_blocks(const Mesh& m) {
  const int nbx = (m.n1 + kRow - 1) / kRow;
  const int nrows = m.n2 * m.n3;
  return nbx * ((nrows + kRows - 1) / kRows);
}

int launch_coef_grad(const Mesh& m, int form, const double* la, const double* fa, const double* lb,
                     const double* fb, double scale, int M, double* partial, double* g, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int nbx = (m.n1 + kRow - 1) / kRow;
  const int nblocks = coef_partial_blocks(m);
  const int nrows = m.n2 * m.n3;
  if (form == 0)
    hipLaunchKernelGGL(coef_partial_kernel<0>, dim3(nblocks), dim3(kCT), 0, s, la, fa, lb, fb, m.n1, nbx, nrows,
                       partial);
  else
    hipLaunchKernelGGL(coef_partial_kernel<1>, dim3(nblocks), dim3(kCT), 0, s, la, fa, lb, fb, m.n1, nbx, nrows,
                       partial);
  hipLaunchKernelGGL(coef_finalize_kernel, dim3(M), dim3(256), 0, s, (const double*)partial, nblocks, scale, g);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "coefficient-gradient launch failed");
}

// Work items for the fused reverse: enough chunks along x2 that every
// persistent workgroup has at least one item, each chunk never empty.
static AdjWork adj_work(const Mesh& m) {
  AdjWork W;
  W.strips = (m.n1 + kATX - 1) / kATX;
  W.nty = (m.n2 + kATY - 1) / kATY;
  const int64_t pairs = (int64_t)W.strips * m.n3;
  const int64_t want = (kAdjBlocks + pairs - 1) / pairs;
  const int ys = (int)std::min<int64_t>(W.nty, std::max<int64_t>(1, want));
  W.tpb = (W.nty + ys - 1) / ys;
  W.ysplit = (W.nty + W.tpb - 1) / W.tpb;
  const int64_t total = pairs * W.ysplit;
  W.nwork = total > INT32_MAX - kAdjBlocks ? -1 : (int)total;  // -1: too many items for int indices
  return W;
}

bool adjoint_sweep2d_fits(const Mesh& m) {
  return (int64_t)m.n1 * m.n2 <= INT32_MAX && adj_work(m).nwork > 0;
}

int64_t adjoint_sweep2d_blocks(const Mesh& m) {
  const AdjWork W = adj_work(m);
  return W.nwork < 0 ? kAdjBlocks : std::min<int64_t>(W.nwork, kAdjBlocks);
}

int launch_adjoint_sweep2d(const Mesh& m, void* const lE[3], void* const lB[3], void* const lEo[3],
                           void* const lBo[3], const void* const Enext[3], const void* const Bhalf[3],
                           void* const En[3], const double* CE, int ME, double cb1, double dt, int M,
                           double* partial, double* gCE, double* gCB, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  AdjPlane P;
  for (int c = 0; c < 3; ++c) {
    P.li[c] = (const double*)lE[c];
    P.li[3 + c] = (const double*)lB[c];
    P.lo[c] = (double*)lEo[c];
    P.lo[3 + c] = (double*)lBo[c];
  }
  P.fw[0] = (const double*)Enext[1];
  P.fw[1] = (const double*)Enext[2];
  P.fw[2] = (const double*)Bhalf[1];
  P.fw[3] = (const double*)Bhalf[2];
  P.fw[4] = (const double*)En[1];
  P.fw[5] = (const double*)En[2];
  Coef16 a;
  const double h = -0.5 * dt;
  for (int q = 0; q < kAW; ++q) a.c[q] = (q < ME ? CE[q] : 0.0) * h / m.dx1;
  if (!adjoint_sweep2d_fits(m)) return set_error(PIC_EUNSUPPORTED, "adjoint sweep: mesh too large for the fused path");
  const AdjWork W = adj_work(m);
  const int64_t nb = adjoint_sweep2d_blocks(m);
  const bool near = m.n1 >= kAXB && m.n2 >= kATY + 3;
  const void* kern = near ? (const void*)adjoint_sweep2d_kernel<true> : (const void*)adjoint_sweep2d_kernel<false>;
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kALds) != hipSuccess)
    return set_error(PIC_EHIP, "adjoint sweep: cannot reserve %zu bytes of LDS", kALds);
  const double ty = h / m.dx2, bx = cb1 * (-dt) / m.dx1, hy = -dt / m.dx2;
  if (near)
    hipLaunchKernelGGL(adjoint_sweep2d_kernel<true>, dim3((unsigned)nb), dim3(kANT), kALds, s, P, m, W, a, ty, bx, hy,
                       partial);
  else
    hipLaunchKernelGGL(adjoint_sweep2d_kernel<false>, dim3((unsigned)nb), dim3(kANT), kALds, s, P, m, W, a, ty, bx,
                       hy, partial);
  hipLaunchKernelGGL(coef_finalize2_kernel, dim3(2 * M), dim3(256), 0, s, (const double*)partial, nb, M,
                     0.5 * dt / m.dx1, dt / m.dx1, gCE, gCB);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "adjoint sweep launch failed");
}

int launch_adjoint_push(const Mesh& m, void* const E[3], void* const B[3], void* const lE[3], void* const lB[3],
                        const pic_particles& p, const pic_particles& lam, int pusher, double dt, void* stream) {
  if (p.np == 0) return PIC_OK;
  hipStream_t s = (hipStream_t)stream;
  AdjFields F;
  for (int c = 0; c < 3; ++c) {
    F.f[c] = (const double*)E[c];
    F.f[3 + c] = (const double*)B[c];
    F.l[c] = (double*)lE[c];
    F.l[3 + c] = (double*)lB[c];
  }
  const dim3 grid((unsigned)((p.np + 255) / 256)), block(256);
  const double qm = p.q / p.m;
#define YP_ADJ(ND, PU)                                                                                        \
  hipLaunchKernelGGL((adjoint_push_kernel<ND, PU>), grid, block, 0, s, F, m, p.x[0], p.x[1], p.x[2], p.u[0], p.u[1], \
                     p.u[2], lam.x[0], lam.x[1], lam.x[2], lam.u[0], lam.u[1], lam.u[2], p.np, qm, dt)
  if (m.ndim == 3) {
    if (pusher == PIC_PUSH_BORIS) YP_ADJ(3, PIC_PUSH_BORIS); else YP_ADJ(3, PIC_PUSH_ANALYTIC);
  } else {
    if (pusher == PIC_PUSH_BORIS) YP_ADJ(2, PIC_PUSH_BORIS); else YP_ADJ(2, PIC_PUSH_ANALYTIC);
  }
#undef YP_ADJ
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "adjoint push launch failed");
}

}  // namespace yeepic
