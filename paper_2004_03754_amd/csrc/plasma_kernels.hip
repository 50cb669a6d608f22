// Plasma step kernels (gfx950): particles sorted by spatial tile so that the
// charge-conserving current (Sec. 3.3) is accumulated in LDS per tile.
//
//   tile_count   tile key of every particle, counts per tile (wave-aggregated)
//   tile_scan    exclusive scan of the counts (one workgroup)
//   tile_scatter counting-sort scatter of x, u (and ids) into scratch
//   tile_rank    the same sort as a permutation only: perm[sorted] = source
//   tile_push    per tile: gather + push + position update of its particles,
//                Esirkepov current into an LDS tile, one atomic flush per node
//   tile_deposit the same current for given old and new positions
//   reduce_stage deterministic mode: the tiles' currents are stored, not
//                added, and summed per node in a fixed order
//
// A tile is tx x ty x tz cells.  Particles stay sorted for S steps; since
// |v| < c a particle drifts at most ceil((S-1) dt/dx_d) cells (the margin m_d)
// out of its tile, so the LDS current tile spans t_d + 2 m_d + 3 nodes per
// direction.  A particle found outside that span (only possible for invalid
// input) deposits through global atomics instead.
#include <hip/hip_runtime.h>

#include <cmath>

#include "particle_common.h"

namespace yeepic {
namespace {

using namespace pdev;

__device__ __forceinline__ int cell_of(double x, double idx, int n) {
  double f = floor(x * idx);
  f = fmin(fmax(f, 0.0), (double)(n - 1));
  return (int)f;
}

// Sort key of a position: its tile, then within the tile its x3 cell plane
// and pair of x2 cell rows.  A tile's particles are thus grouped so that the
// 64 particles of a wave mostly share one plane and two rows (16 cells, 4
// particles per cell at 8 per cell): the gather's loads of a wave then touch
// about 3 field rows per plane instead of the tile's 64, and the L1, shared
// by the waves of three tiles, keeps far more of them.  (Finer bins crowd a
// wave's current atomics onto fewer nodes.)
__device__ __forceinline__ int tile_key_at(double x1, double x2, double x3, const Mesh& m, const TileGeom& tg) {
  // divisions by the tile size as one multiply-high each (exact for cell
  // indices below 2^29 at tile sizes up to 8)
  const int cx = (int)__umulhi((unsigned)cell_of(x1, m.idx1, m.n1), tg.mt[0]);
  const int y = cell_of(x2, m.idx2, m.n2);
  const int cy = (int)__umulhi((unsigned)y, tg.mt[1]);
  const int z = cell_of(x3, m.idx3, m.n3);
  const int cz = (int)__umulhi((unsigned)z, tg.mt[2]);
  const int pairs = (tg.t[1] + 1) / 2;
  return ((cz * tg.nt[1] + cy) * tg.nt[0] + cx) * tg.sub + (z - cz * tg.t[2]) * pairs + (y - cy * tg.t[1]) / 2;
}

__device__ __forceinline__ int tile_key(const double* const* x, int64_t p, const Mesh& m, const TileGeom& tg) {
  return tile_key_at(x[0][p], x[1][p], x[2][p], m, tg);
}

// lanes with equal consecutive keys form runs; returns the run leader lane
// of this lane and the run length (for leaders)
__device__ __forceinline__ void key_runs(int key, int& leader_lane, int& runlen) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1);
  const bool leader = lane == 0 || prev != key;
  const unsigned long long lead = __ballot(leader);
  const unsigned long long upto = lead & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
  leader_lane = 63 - __clzll(upto);
  const unsigned long long above = lane == 63 ? 0ull : (lead >> (lane + 1));
  const int next = above ? lane + __ffsll((long long)above) : 64;
  runlen = next - lane;
}

__global__ __launch_bounds__(256) void tile_count_kernel(const double* __restrict__ x1, const double* __restrict__ x2,
                                                         const double* __restrict__ x3, int64_t np, Mesh m,
                                                         TileGeom tg, int* __restrict__ keys,
                                                         int* __restrict__ counts) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double* x[3] = {x1, x2, x3};
  int key = -1;
  if (p < np) {
    key = tile_key(x, p, m, tg);
    keys[p] = key;
  }
  int leader_lane, runlen;
  key_runs(key, leader_lane, runlen);
  if (leader_lane == (int)(threadIdx.x & 63) && key >= 0) atomicAdd(&counts[key], runlen);
}

// Exclusive scan of n tile counts in two passes over segments of kScanSeg
// counts (one workgroup of 1024 threads, four consecutive counts per thread):
// the segment sums, then each segment's scan plus the sum of the segments
// before it.  The second pass also clears the scatter cursors and writes
// offsets[n] = total.
constexpr int kScanSeg = 4096;

__device__ __forceinline__ int load_count(const int* __restrict__ c, int i, int n) { return i < n ? c[i] : 0; }

__global__ __launch_bounds__(1024) void tile_segsum_kernel(const int* __restrict__ counts, int n,
                                                           int* __restrict__ segsum) {
  __shared__ int wsum[16];
  const int t = threadIdx.x, base = blockIdx.x * kScanSeg + 4 * t;
  int v = load_count(counts, base, n) + load_count(counts, base + 1, n) + load_count(counts, base + 2, n) +
          load_count(counts, base + 3, n);
  for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d);
  if ((t & 63) == 0) wsum[t >> 6] = v;
  __syncthreads();
  if (t == 0) {
    int s = 0;
    for (int w = 0; w < 16; ++w) s += wsum[w];
    segsum[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(1024) void tile_segscan_kernel(const int* __restrict__ counts, int n,
                                                            const int* __restrict__ segsum, int nseg,
                                                            int* __restrict__ offsets, int* __restrict__ cursors) {
  __shared__ int wpre[16];
  __shared__ int segbase;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (w == 0) {  // sum of the preceding segments
    int s = 0;
    for (int i = lane; i < (int)blockIdx.x; i += 64) s += segsum[i];
    for (int d = 32; d > 0; d >>= 1) s += __shfl_down(s, d);
    if (lane == 0) segbase = s;
  }
  const int base = blockIdx.x * kScanSeg + 4 * t;
  const int c0 = load_count(counts, base, n), c1 = load_count(counts, base + 1, n),
            c2 = load_count(counts, base + 2, n), c3 = load_count(counts, base + 3, n);
  const int mine = c0 + c1 + c2 + c3;
  int inc = mine;  // inclusive scan across the wave
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(inc, d);
    if (lane >= d) inc += y;
  }
  if (lane == 63) wpre[w] = inc;
  __syncthreads();
  int before = segbase;
  for (int v = 0; v < w; ++v) before += wpre[v];
  int run = before + inc - mine;
  const int cs[4] = {c0, c1, c2, c3};
  for (int e = 0; e < 4; ++e)
    if (base + e < n) {
      offsets[base + e] = run;
      cursors[base + e] = 0;
      run += cs[e];
    }
  if (blockIdx.x == nseg - 1 && t == 1023) {
    int total = segbase;
    for (int v = 0; v < 16; ++v) total += wpre[v];
    offsets[n] = total;
  }
}

__global__ __launch_bounds__(256) void tile_scatter_kernel(const double* __restrict__ x1, const double* __restrict__ x2,
                                                           const double* __restrict__ x3, const double* __restrict__ u1,
                                                           const double* __restrict__ u2, const double* __restrict__ u3,
                                                           const int64_t* __restrict__ id, const int* __restrict__ keys,
                                                           const int* __restrict__ offsets, int* __restrict__ cursors,
                                                           int64_t np, double* __restrict__ sx1, double* __restrict__ sx2,
                                                           double* __restrict__ sx3, double* __restrict__ su1,
                                                           double* __restrict__ su2, double* __restrict__ su3,
                                                           int64_t* __restrict__ sid) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < np;
  const int key = live ? keys[p] : -1;
  // the particle's state is read before the cursor atomic, so that its
  // loads overlap the atomic's round trip
  double v[6] = {0, 0, 0, 0, 0, 0};
  int64_t pid = 0;
  if (live) {
    v[0] = __builtin_nontemporal_load(x1 + p);
    v[1] = __builtin_nontemporal_load(x2 + p);
    v[2] = __builtin_nontemporal_load(x3 + p);
    v[3] = __builtin_nontemporal_load(u1 + p);
    v[4] = __builtin_nontemporal_load(u2 + p);
    v[5] = __builtin_nontemporal_load(u3 + p);
    if (id) pid = __builtin_nontemporal_load(id + p);
  }
  int leader_lane, runlen;
  key_runs(key, leader_lane, runlen);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (leader_lane == lane && key >= 0) base = atomicAdd(&cursors[key], runlen);
  base = __shfl(base, leader_lane);
  if (!live) return;
  const int64_t q = (int64_t)offsets[key] + base + (lane - leader_lane);
  __builtin_nontemporal_store(v[0], sx1 + q);
  __builtin_nontemporal_store(v[1], sx2 + q);
  __builtin_nontemporal_store(v[2], sx3 + q);
  __builtin_nontemporal_store(v[3], su1 + q);
  __builtin_nontemporal_store(v[4], su2 + q);
  __builtin_nontemporal_store(v[5], su3 + q);
  if (id) __builtin_nontemporal_store(pid, sid + q);
}

// The counting sort's placement without moving the particles: perm[q] = p
// for the sorted position q of particle p (the same cursor runs as
// tile_scatter).  The push that follows reads each particle through perm and
// writes it at its sorted position into the other particle buffer, so a sort
// costs no pass over the particle data of its own.
// Each wave ranks four runs of 64 consecutive particles (one per group of its
// 256-particle chunk), so that the four key -> offset -> cursor round trips
// overlap.
constexpr int kRankGroups = 4;

__global__ __launch_bounds__(256) void tile_rank_kernel(const int* __restrict__ keys, const int* __restrict__ offsets,
                                                        int* __restrict__ cursors, int64_t np,
                                                        int* __restrict__ perm) {
  const int lane = threadIdx.x & 63;
  const int64_t p0 = ((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63)) * kRankGroups + lane;
  int key[kRankGroups], off[kRankGroups], lead[kRankGroups], base[kRankGroups];
#pragma unroll
  for (int r = 0; r < kRankGroups; ++r) {
    const int64_t p = p0 + 64 * r;
    key[r] = p < np ? keys[p] : -1;
  }
#pragma unroll
  for (int r = 0; r < kRankGroups; ++r) {
    int runlen;
    key_runs(key[r], lead[r], runlen);
    off[r] = key[r] >= 0 ? offsets[key[r]] : 0;
    base[r] = 0;
    if (lead[r] == lane && key[r] >= 0) base[r] = atomicAdd(&cursors[key[r]], runlen);
  }
#pragma unroll
  for (int r = 0; r < kRankGroups; ++r) {
    const int b = __shfl(base[r], lead[r]);
    const int64_t p = p0 + 64 * r;
    if (p < np) perm[(int64_t)off[r] + b + (lane - lead[r])] = (int)p;
  }
}

// ---------------------------------------------------------------------------
// The tile current: 64-bit fixed point in LDS.  Integer LDS adds are an order
// of magnitude faster than float ones on this part, and integer sums do not
// depend on the order of the adds.
//
// Scale.  Every Esirkepov contribution is at most c = max_d |q w| dx_d/dt in
// magnitude: it is -q w (dx_d/dt) times a running sum of shape differences
// (a difference of two partial sums of shape values, so at most 1 in
// magnitude) times a transverse weight in [0, 1].  A node of a tile receives
// at most one contribution per component from each of the tile's ``count``
// particles, so with the quantum q_t = 2^(e - 61), e = floor(log2(count c)),
// no node sum can exceed 2^62 in magnitude: the accumulator cannot overflow
// for any particle load or move, and each contribution is rounded to q_t.
//
// FP32 grids take e = max(floor(log2(count c)), floor(log2 c) + 11), so that
// every scaled contribution is below 2^51 in magnitude and converts to an
// integer with one add of 1.5 2^52 (round to nearest even, as llrint, whose
// 64-bit form takes six instructions); the quantum is then at most 2^-49 c,
// far below FP32 resolution.
//
// FP64 grids keep two words per node: hi = round(v/q_t) and the rounding
// residual in units of q_t 2^-L, lo = round((v/q_t - hi) 2^L), L = 63 -
// bitlength(count) (again no overflow).  The node value (hi + lo 2^-L) q_t is
// then the sum of the FP64 contributions to within 2^-L q_t per contribution:
// the tile current equals the exact sum of its contributions rounded about
// once, whatever the order of the adds.
// ---------------------------------------------------------------------------
struct TileScale {
  double s, us;    // 1/q_t and q_t
  double sl, usl;  // 2^L and q_t 2^-L (two-word accumulation)
};

// cmax: the largest |c_d| = |q w| dx_d/dt.
template <bool TWO>
__device__ __forceinline__ TileScale tile_scale(int count, double cmax) {
  const double cq = (double)count * cmax;
  int e = cq > 0.0 ? ilogb(cq) : 0;
  if (!TWO && cmax > 0.0) e = max(e, ilogb(cmax) + 11);
  const int L = 63 - (32 - __clz(count > 0 ? count : 1));
  TileScale t;
  t.s = ldexp(1.0, 61 - e);
  t.us = ldexp(1.0, e - 61);
  t.sl = ldexp(1.0, L);
  t.usl = ldexp(1.0, e - 61 - L);
  return t;
}

// v: a contribution (FP64 grids), or the contribution already in units of
// the quantum (FP32 grids, |v| < 2^51).
template <bool TWO>
__device__ __forceinline__ void acc_add(unsigned long long* hi, unsigned long long* lo, double v, const TileScale& ts) {
  if (TWO) {
    // the product rounds first (v is itself rounded), so y - h below is
    // exact, whether or not the compiler fuses it with the scaling
    const double y = v * ts.s;  // exact: a power-of-two scaling, |y| < 2^62
    const long long h = llrint(y);
    atomicAdd(hi, (unsigned long long)h);
    atomicAdd(lo, (unsigned long long)llrint((y - (double)h) * ts.sl));
  } else {
    const double y = v;
    const double t = y + 6755399441055744.0;  // 1.5 2^52: the integer round(y) lands in the low bits
    atomicAdd(hi, (unsigned long long)(__double_as_longlong(t) - 0x4338000000000000LL));
  }
}

template <bool TWO>
__device__ __forceinline__ double acc_value(unsigned long long hi, unsigned long long lo, const TileScale& ts) {
  double v = (double)(long long)hi * ts.us;
  if (TWO) v += (double)(long long)lo * ts.usl;
  return v;
}

// Geometry of one tile's LDS current: origin m + 1 nodes below the tile.
struct TileWin {
  int lo[3];
  int r0, r1, R;
};

__device__ __forceinline__ TileWin tile_window(int tile, const TileGeom& tg) {
  TileWin w;
  const int tx = tile % tg.nt[0], ty = (tile / tg.nt[0]) % tg.nt[1], tz = tile / (tg.nt[0] * tg.nt[1]);
  w.lo[0] = tx * tg.t[0];
  w.lo[1] = ty * tg.t[1];
  w.lo[2] = tz * tg.t[2];
  w.r0 = tg.r[0];
  w.r1 = tg.r[1];
  w.R = tg.r[0] * tg.r[1] * tg.r[2];
  return w;
}

// Esirkepov current of one particle moving from xo to xn (Sec. 3.3): into
// the tile's LDS accumulator when its stencil lies inside the tile window,
// else (only for input moving faster than c) through global atomics.
template <typename T, int ORDER, bool TWO>
__device__ __forceinline__ void deposit_one(const double xo[3], const double xn[3], const Mesh& m,
                                            const TileGeom& tg, const TileWin& w, unsigned long long* jh,
                                            unsigned long long* jl, const TileScale& ts, double c1, double c2,
                                            double c3, T* const Jg[3]) {
  constexpr int K = ORDER + 2;  // stencil nodes per direction
  const int n[3] = {m.n1, m.n2, m.n3};
  const ShapeK<K> sh[3] = {shape_o<ORDER>(xo[0], xn[0], m.idx1, m.L1), shape_o<ORDER>(xo[1], xn[1], m.idx2, m.L2),
                           shape_o<ORDER>(xo[2], xn[2], m.idx3, m.L3)};
  // stencil origin relative to the LDS current tile (periodic images folded in)
  int rel[3];
  bool inside = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int bb = sh[d].base - w.lo[d];
    if (bb < -(n[d] / 2)) bb += n[d];
    if (bb > n[d] / 2) bb -= n[d];
    rel[d] = bb + tg.m[d] + 1;
    inside = inside && rel[d] >= 0 && rel[d] + K - 1 < tg.r[d];
  }
  if (inside) {
    const int o = (rel[2] * w.r1 + rel[1]) * w.r0 + rel[0];
    // FP32 grids: coefficients in units of the quantum (power-of-two
    // scalings, exact), so that each contribution is one product
    const double k = TWO ? 1.0 : ts.s;
    auto add = [&](int comp, int a, int b, int c, double v) {
      const int i = comp * w.R + o + (c * w.r1 + b) * w.r0 + a;
      acc_add<TWO>(&jh[i], &jl[i], v, ts);
    };
    // along a direction in which no particle of the wave changes cell, every
    // stencil's last node is empty there, and a smaller loop skips it
    int full = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      full |= __builtin_amdgcn_ballot_w64(sh[d].s0[K - 1] != 0.0 || sh[d].ds[K - 1] != 0.0) ? 1 << d : 0;
    const double k1 = c1 * k, k2 = c2 * k, k3 = c3 * k;
    // one-word (FP32 grid) accumulators add exact zeros faster than they
    // test for them; two-word ones skip them
    switch (full) {
      case 0: esirkepov<K, K - 1, K - 1, K - 1, TWO>(sh[0], sh[1], sh[2], k1, k2, k3, add); break;
      case 1: esirkepov<K, K, K - 1, K - 1, TWO>(sh[0], sh[1], sh[2], k1, k2, k3, add); break;
      case 2: esirkepov<K, K - 1, K, K - 1, TWO>(sh[0], sh[1], sh[2], k1, k2, k3, add); break;
      case 3: esirkepov<K, K, K, K - 1, TWO>(sh[0], sh[1], sh[2], k1, k2, k3, add); break;
      case 4: esirkepov<K, K - 1, K - 1, K, TWO>(sh[0], sh[1], sh[2], k1, k2, k3, add); break;
      case 5: esirkepov<K, K, K - 1, K, TWO>(sh[0], sh[1], sh[2], k1, k2, k3, add); break;
      case 6: esirkepov<K, K - 1, K, K, TWO>(sh[0], sh[1], sh[2], k1, k2, k3, add); break;
      default: esirkepov<K, K, K, K, TWO>(sh[0], sh[1], sh[2], k1, k2, k3, add); break;
    }
  } else {
    const size_t pl = (size_t)m.n1 * m.n2;
    int gw[3][K];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int k = 0; k < K; ++k) gw[d][k] = wrapn(sh[d].base + k, n[d]);
    esirkepov<K>(sh[0], sh[1], sh[2], c1, c2, c3, [&](int comp, int a, int b, int c, double v) {
      atomic_add(&Jg[comp][(size_t)gw[2][c] * pl + (size_t)gw[1][b] * m.n1 + gw[0][a]], v);
    });
  }
}

// Clears the tile's accumulator words (1 or 2 per node and component).
__device__ __forceinline__ void acc_clear(unsigned long long* jh, int words) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) jh[i] = 0;
}

// Flush of a tile's current: one global atomic add per non-zero node, or,
// with ``stage`` (the deterministic mode), a plain store of every node's
// value into the tile's slot of the staging array, which reduce_stage_kernel
// then sums in a fixed order.
template <typename T, bool TWO>
__device__ __forceinline__ void acc_flush(const unsigned long long* jh, const unsigned long long* jl,
                                          const TileScale& ts, const TileWin& w, const TileGeom& tg, const Mesh& m,
                                          int tile, T* const Jg[3], double* stage) {
  const size_t pl = (size_t)m.n1 * m.n2;
  if (!stage && w.r0 <= 64) {
    // one x1 row of the window per L lanes (the row's nodes in its first
    // r0 lanes), so that each lane keeps its x1 node and steps its row
    // indices by carries instead of dividing; row = (comp r2 + c) r1 + b
    const int L = w.r0 <= 16 ? 16 : (w.r0 <= 32 ? 32 : 64);
    const int a = (int)threadIdx.x % L, P = (int)blockDim.x / L, r2 = tg.r[2];
    if (a >= w.r0) return;
    const int gx = wrapn(w.lo[0] + a - tg.m[0] - 1, m.n1);
    // a window row's mesh row lo + b - m - 1 lies in [-n, 2n) when the mesh
    // is at least as wide as the window: one conditional add or subtract
    // wraps it (else the general remainder)
    const bool near = m.n2 >= w.r1 && m.n3 >= r2;
    auto wrap_row = [&](int v, int n) { return near ? (v < 0 ? v + n : (v >= n ? v - n : v)) : wrapn(v, n); };
    int row = (int)threadIdx.x / L;
    int b = row % w.r1, c = (row / w.r1) % r2, comp = row / (w.r1 * r2);
    for (; row < 3 * w.r1 * r2; row += P) {
      const int i = row * w.r0 + a;
      const double v = acc_value<TWO>(jh[i], TWO ? jl[i] : 0ull, ts);
      if (v != 0.0) {
        const int gy = wrap_row(w.lo[1] + b - tg.m[1] - 1, m.n2);
        const int gz = wrap_row(w.lo[2] + c - tg.m[2] - 1, m.n3);
        unsafeAtomicAdd(&Jg[comp][(size_t)gz * pl + (size_t)gy * m.n1 + gx], (T)v);
      }
      b += P;
      while (b >= w.r1) {
        b -= w.r1;
        ++c;
      }
      while (c >= r2) {
        c -= r2;
        ++comp;
      }
    }
    return;
  }
  for (int i = threadIdx.x; i < 3 * w.R; i += blockDim.x) {
    const double v = acc_value<TWO>(jh[i], TWO ? jl[i] : 0ull, ts);
    if (stage) {
      stage[(size_t)tile * 3 * w.R + i] = v;
      continue;
    }
    if (v == 0.0) continue;
    const int comp = i / w.R;
    const int q = i - comp * w.R;
    const int a = q % w.r0, b = (q / w.r0) % w.r1, c = q / (w.r0 * w.r1);
    const int gx = wrapn(w.lo[0] + a - tg.m[0] - 1, m.n1);
    const int gy = wrapn(w.lo[1] + b - tg.m[1] - 1, m.n2);
    const int gz = wrapn(w.lo[2] + c - tg.m[2] - 1, m.n3);
    unsafeAtomicAdd(&Jg[comp][(size_t)gz * pl + (size_t)gy * m.n1 + gx], (T)v);
  }
}

// Workgroups are dealt to the eight XCDs in turn (workgroup b to XCD
// b % 8).  Tile of workgroup b: each XCD takes one contiguous run of tiles,
// so the tiles an XCD holds at once are neighbours whose field rows and
// current nodes share its L2.  (Grids have n1 a multiple of 64, so the tile
// count is a multiple of 8; the formula is a bijection for any count.)
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int x = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + min(x, r) + k;
}

// FP32 linear-shape pushes fit three workgroups per CU in LDS: the Boris and
// Higuera-Cary ones are held to the registers of three waves per SIMD too
template <typename T, int PUSH, int ORDER, bool TWO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(!TWO && ORDER == 1 && PUSH != PIC_PUSH_ANALYTIC ? 3 : 1)))
void tile_push_kernel(
    const T* __restrict__ E1, const T* __restrict__ E2, const T* __restrict__ E3, const T* __restrict__ B1,
    const T* __restrict__ B2, const T* __restrict__ B3, T* __restrict__ J1, T* __restrict__ J2, T* __restrict__ J3,
    Mesh m, TileGeom tg, const int* __restrict__ offsets, const double* sx1, const double* sx2, const double* sx3,
    const double* su1, const double* su2, const double* su3, const int64_t* sid, double* dx1, double* dx2,
    double* dx3, double* du1, double* du2, double* du3, int64_t* did, const int* __restrict__ perm, double qm,
    double qw, double dt, double* stage, int* __restrict__ keys, int* __restrict__ counts) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const TileWin w = tile_window(tile, tg);
  unsigned long long* jh = reinterpret_cast<unsigned long long*>(lds_raw);
  unsigned long long* jl = jh + 3 * w.R;
  const int beg = offsets[tile * tg.sub], end = offsets[(tile + 1) * tg.sub];
  T* const Jg[3] = {J1, J2, J3};
  if (end == beg && !stage) return;  // uniform: no particles, nothing to add
  const double c1 = -qw * m.dx1 / dt, c2 = -qw * m.dx2 / dt, c3 = -qw * m.dx3 / dt;
  const TileScale ts = tile_scale<TWO>(end - beg, fmax(fabs(c1), fmax(fabs(c2), fabs(c3))));
  acc_clear(jh, (TWO ? 6 : 3) * w.R);
  __syncthreads();
  // the next particle's position is loaded one iteration ahead, so that its
  // memory latency overlaps this particle's work instead of delaying the
  // gather that depends on it.  Particle i (sorted position) is read from
  // source index perm[i] when the sort left a permutation, else from i.
  double xc[3] = {0.0, 0.0, 0.0};
  int pc = 0;
  if (beg + (int)threadIdx.x < end) {
    pc = perm ? perm[beg + threadIdx.x] : beg + (int)threadIdx.x;
    xc[0] = __builtin_nontemporal_load(sx1 + pc);
    xc[1] = __builtin_nontemporal_load(sx2 + pc);
    xc[2] = __builtin_nontemporal_load(sx3 + pc);
  }
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const double x[3] = {xc[0], xc[1], xc[2]};
    const int si = pc;
    double u[3] = {__builtin_nontemporal_load(su1 + si), __builtin_nontemporal_load(su2 + si),
                   __builtin_nontemporal_load(su3 + si)};
    const int inext = i + blockDim.x;
    if (inext < end) {
      pc = perm ? perm[inext] : inext;
      xc[0] = __builtin_nontemporal_load(sx1 + pc);
      xc[1] = __builtin_nontemporal_load(sx2 + pc);
      xc[2] = __builtin_nontemporal_load(sx3 + pc);
    }
    double E[3], B[3];
    gather_o<T, 3, ORDER>(E1, E2, E3, B1, B2, B3, m, x, E, B);
    if (PUSH == PIC_PUSH_BORIS)
      boris(u, E, B, qm, dt);
    else if (PUSH == PIC_PUSH_HC)
      higuera_cary(u, E, B, qm, dt);
    else
      analytic(u, E, B, qm, dt, m);
    const double ig = dt / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double xn[3] = {wrap_pos(x[0] + ig * u[0], m.L1), wrap_pos(x[1] + ig * u[1], m.L2),
                          wrap_pos(x[2] + ig * u[2], m.L3)};
    __builtin_nontemporal_store(xn[0], dx1 + i);
    __builtin_nontemporal_store(xn[1], dx2 + i);
    __builtin_nontemporal_store(xn[2], dx3 + i);
    __builtin_nontemporal_store(u[0], du1 + i);
    __builtin_nontemporal_store(u[1], du2 + i);
    __builtin_nontemporal_store(u[2], du3 + i);
    if (sid && sid != did) did[i] = sid[si];
    if (keys) {  // the next sort's tile key and count, from the new position
      const int key = tile_key_at(xn[0], xn[1], xn[2], m, tg);
      keys[i] = key;
      // one add for the lanes that share the first active lane's key (most
      // of a wave on sorted particles), one per lane for the others
      const int k0 = __builtin_amdgcn_readfirstlane(key);
      const unsigned long long same = __ballot(key == k0);
      if (key != k0)
        atomicAdd(&counts[key], 1);
      else if ((int)(threadIdx.x & 63) == __ffsll((long long)same) - 1)
        atomicAdd(&counts[k0], __popcll(same));
    }
    deposit_one<T, ORDER, TWO>(x, xn, m, tg, w, jh, jl, ts, c1, c2, c3, Jg);
  }
  __syncthreads();
  acc_flush<T, TWO>(jh, jl, ts, w, tg, m, tile, Jg, stage);
}

// The deposit alone (pic_deposit_J): particles sorted by the tile of their
// old position, old positions in xo, new ones in xn.
template <typename T, int ORDER, bool TWO>
__global__ __launch_bounds__(256) void tile_deposit_kernel(T* __restrict__ J1, T* __restrict__ J2,
                                                           T* __restrict__ J3, Mesh m, TileGeom tg,
                                                           const int* __restrict__ offsets, const double* xo1,
                                                           const double* xo2, const double* xo3, const double* xn1,
                                                           const double* xn2, const double* xn3, double qw, double dt,
                                                           double* stage, const int* __restrict__ perm) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const TileWin w = tile_window(tile, tg);
  unsigned long long* jh = reinterpret_cast<unsigned long long*>(lds_raw);
  unsigned long long* jl = jh + 3 * w.R;
  const int beg = offsets[tile * tg.sub], end = offsets[(tile + 1) * tg.sub];
  T* const Jg[3] = {J1, J2, J3};
  if (end == beg && !stage) return;
  const double c1 = -qw * m.dx1 / dt, c2 = -qw * m.dx2 / dt, c3 = -qw * m.dx3 / dt;
  const TileScale ts = tile_scale<TWO>(end - beg, fmax(fabs(c1), fmax(fabs(c2), fabs(c3))));
  acc_clear(jh, (TWO ? 6 : 3) * w.R);
  __syncthreads();
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const int si = perm ? perm[i] : i;  // the pair at sorted position i
    const double xo[3] = {__builtin_nontemporal_load(xo1 + si), __builtin_nontemporal_load(xo2 + si),
                          __builtin_nontemporal_load(xo3 + si)};
    const double xn[3] = {__builtin_nontemporal_load(xn1 + si), __builtin_nontemporal_load(xn2 + si),
                          __builtin_nontemporal_load(xn3 + si)};
    deposit_one<T, ORDER, TWO>(xo, xn, m, tg, w, jh, jl, ts, c1, c2, c3, Jg);
  }
  __syncthreads();
  acc_flush<T, TWO>(jh, jl, ts, w, tg, m, tile, Jg, stage);
}

// Deterministic mode: J[node] += the staged tile values that land on the
// node, summed in FP64 over the covering tiles in increasing tile index (per
// direction) and, within a tile, over its periodic images in increasing
// window index.  One thread per node and component.
__device__ __forceinline__ int cover(int i, int d, const TileGeom& tg, int n, int* tl, int* ws, int& nw) {
  // tiles along direction d whose window holds node i, and the window
  // indices of every image of i in each; returns the number of tiles
  const int t = tg.t[d], nt = tg.nt[d], r = tg.r[d], mg = tg.m[d];
  const int reach = (mg + 2 + t - 1) / t + 1;
  int ntl = 0;
  nw = 0;
  const int c = i / t;
  const bool all = nt <= 2 * reach + 1;
  const int first = all ? 0 : c - reach, last = all ? nt - 1 : c + reach;
  for (int k = first; k <= last; ++k) {
    const int tt = all ? k : ((k % nt) + nt) % nt;
    const int base = tt * t - mg - 1;  // node of window index 0
    int a = ((i - base) % n + n) % n;
    int cnt = 0;
    for (; a < r; a += n) {
      ws[nw + cnt] = a;
      ++cnt;
    }
    if (cnt) {
      tl[2 * ntl] = tt;
      tl[2 * ntl + 1] = cnt;
      nw += cnt;
      ++ntl;
    }
  }
  return ntl;
}

template <typename T>
__global__ __launch_bounds__(256) void reduce_stage_kernel(T* __restrict__ J1, T* __restrict__ J2,
                                                           T* __restrict__ J3, Mesh m, TileGeom tg,
                                                           const double* __restrict__ stage) {
  const int64_t cells = (int64_t)m.n1 * m.n2 * m.n3;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 3 * cells) return;
  const int comp = (int)(g / cells);
  const int64_t cell = g - comp * cells;
  const int i = (int)(cell % m.n1), j = (int)((cell / m.n1) % m.n2), k = (int)(cell / ((int64_t)m.n1 * m.n2));
  constexpr int kMaxT = 16, kMaxW = 64;  // limits checked on the host (ensure_stage)
  int tx[2 * kMaxT], ty[2 * kMaxT], tz[2 * kMaxT], wx[kMaxW], wy[kMaxW], wz[kMaxW];
  int nwx, nwy, nwz;
  const int ntx = cover(i, 0, tg, m.n1, tx, wx, nwx);
  const int nty = cover(j, 1, tg, m.n2, ty, wy, nwy);
  const int ntz = cover(k, 2, tg, m.n3, tz, wz, nwz);
  const int r0 = tg.r[0], r1 = tg.r[1], R = r0 * r1 * tg.r[2];
  double acc = 0.0;
  int oz = 0;
  for (int c = 0; c < ntz; ++c) {
    int oy = 0;
    for (int b = 0; b < nty; ++b) {
      int ox = 0;
      for (int a = 0; a < ntx; ++a) {
        const int tile = (tz[2 * c] * tg.nt[1] + ty[2 * b]) * tg.nt[0] + tx[2 * a];
        const double* s = stage + (size_t)tile * 3 * R + (size_t)comp * R;
        for (int cz = 0; cz < tz[2 * c + 1]; ++cz)
          for (int cy = 0; cy < ty[2 * b + 1]; ++cy)
            for (int cx = 0; cx < tx[2 * a + 1]; ++cx)
              acc += s[(wz[oz + cz] * r1 + wy[oy + cy]) * r0 + wx[ox + cx]];
        ox += tx[2 * a + 1];
      }
      oy += ty[2 * b + 1];
    }
    oz += tz[2 * c + 1];
  }
  T* J = comp == 0 ? J1 : (comp == 1 ? J2 : J3);
  J[cell] = (T)((double)J[cell] + acc);
}

size_t tile_lds(const TileGeom& tg, bool two) {
  return sizeof(unsigned long long) * (two ? 6 : 3) * (size_t)tg.r[0] * tg.r[1] * tg.r[2];
}

template <typename T>
int run_tile_push(const Mesh& m, const TileGeom& tg, void* const E[3], void* const B[3], void* const J[3],
                  const int* offsets, const pic_particles& src, const pic_particles& dst, int pusher, double dt,
                  double* stage, int* keys, int* counts, const int* perm, hipStream_t s) {
  constexpr bool TWO = sizeof(T) == sizeof(double);
  const size_t lds = tile_lds(tg, TWO);
  if (lds > 160 * 1024) return set_error(PIC_EUNSUPPORTED, "plasma tile needs %zu bytes of LDS", lds);
  const bool q2 = m.order == 2;
  auto k = pusher == PIC_PUSH_BORIS ? (q2 ? tile_push_kernel<T, PIC_PUSH_BORIS, 2, TWO>
                                          : tile_push_kernel<T, PIC_PUSH_BORIS, 1, TWO>)
           : pusher == PIC_PUSH_HC  ? (q2 ? tile_push_kernel<T, PIC_PUSH_HC, 2, TWO>
                                          : tile_push_kernel<T, PIC_PUSH_HC, 1, TWO>)
                                    : (q2 ? tile_push_kernel<T, PIC_PUSH_ANALYTIC, 2, TWO>
                                          : tile_push_kernel<T, PIC_PUSH_ANALYTIC, 1, TWO>);
  if (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return set_error(PIC_EHIP, "tile push: cannot reserve %zu bytes of LDS", lds);
  const double qm = src.q / src.m, qw = src.q * src.w;
  hipLaunchKernelGGL(k, dim3(tg.ntiles), dim3(256), lds, s, (const T*)E[0], (const T*)E[1], (const T*)E[2],
                     (const T*)B[0], (const T*)B[1], (const T*)B[2], (T*)J[0], (T*)J[1], (T*)J[2], m, tg, offsets,
                     (const double*)src.x[0], (const double*)src.x[1], (const double*)src.x[2],
                     (const double*)src.u[0], (const double*)src.u[1], (const double*)src.u[2],
                     (const int64_t*)src.id, dst.x[0], dst.x[1], dst.x[2], dst.u[0], dst.u[1], dst.u[2], dst.id, perm,
                     qm, qw, dt, stage, keys, counts);
  if (hipGetLastError() != hipSuccess) return set_error(PIC_EHIP, "tile push launch failed");
  if (stage) {
    const int64_t work = 3 * (int64_t)m.n1 * m.n2 * m.n3;
    hipLaunchKernelGGL(reduce_stage_kernel<T>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, (T*)J[0],
                       (T*)J[1], (T*)J[2], m, tg, (const double*)stage);
    if (hipGetLastError() != hipSuccess) return set_error(PIC_EHIP, "current reduction launch failed");
  }
  return PIC_OK;
}

template <typename T>
int run_tile_deposit(const Mesh& m, const TileGeom& tg, void* const J[3], const int* offsets,
                     const pic_particles& sorted, double dt, double* stage, const int* perm, hipStream_t s) {
  constexpr bool TWO = sizeof(T) == sizeof(double);
  const size_t lds = tile_lds(tg, TWO);
  if (lds > 160 * 1024) return set_error(PIC_EUNSUPPORTED, "deposit tile needs %zu bytes of LDS", lds);
  auto k = m.order == 2 ? tile_deposit_kernel<T, 2, TWO> : tile_deposit_kernel<T, 1, TWO>;
  if (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return set_error(PIC_EHIP, "tile deposit: cannot reserve %zu bytes of LDS", lds);
  const double qw = sorted.q * sorted.w;
  hipLaunchKernelGGL(k, dim3(tg.ntiles), dim3(256), lds, s, (T*)J[0], (T*)J[1], (T*)J[2], m, tg, offsets,
                     (const double*)sorted.x[0], (const double*)sorted.x[1], (const double*)sorted.x[2],
                     (const double*)sorted.u[0], (const double*)sorted.u[1], (const double*)sorted.u[2], qw, dt, stage,
                     perm);
  if (hipGetLastError() != hipSuccess) return set_error(PIC_EHIP, "tile deposit launch failed");
  if (stage) {
    const int64_t work = 3 * (int64_t)m.n1 * m.n2 * m.n3;
    hipLaunchKernelGGL(reduce_stage_kernel<T>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, (T*)J[0],
                       (T*)J[1], (T*)J[2], m, tg, (const double*)stage);
    if (hipGetLastError() != hipSuccess) return set_error(PIC_EHIP, "current reduction launch failed");
  }
  return PIC_OK;
}

}  // namespace

TileGeom make_tile_geom(const Mesh& m, double dt, int sort_every) {
  TileGeom tg;
  const int n[3] = {m.n1, m.n2, m.n3};
  const double dx[3] = {m.dx1, m.dx2, m.dx3};
  tg.ntiles = 1;
  for (int d = 0; d < 3; ++d) {
    tg.t[d] = n[d] < 8 ? n[d] : 8;
    tg.mt[d] = tg.t[d] == 1 ? 0u : (unsigned)((1ull << 32) / (unsigned)tg.t[d] + 1);
    tg.nt[d] = (n[d] + tg.t[d] - 1) / tg.t[d];
    // |v| < 1: at most (S-1) dt/dx cells of drift before the next sort
    tg.m[d] = (int)std::ceil((sort_every - 1) * dt / dx[d] - 1e-12);
    if (tg.m[d] < 0) tg.m[d] = 0;
    // LDS current nodes: the tile, the drift margin each side, and the
    // deposit stencil (3 nodes from min(floor) for the linear shape, 4 from
    // min(round) - 1 for the quadratic one), origin m + 1 nodes below the tile
    tg.r[d] = tg.t[d] + 2 * tg.m[d] + 2 + (m.order == 2 ? 2 : 1);
    tg.ntiles *= tg.nt[d];
  }
  tg.sub = tg.t[2] * ((tg.t[1] + 1) / 2);  // bins per tile: x3 planes times pairs of x2 rows
  tg.nbins = tg.ntiles * tg.sub;
  return tg;
}

int scan_segments(int ntiles) { return (ntiles + kScanSeg - 1) / kScanSeg; }

int launch_tile_sort(const Mesh& m, const TileGeom& tg, const pic_particles& p, const pic_particles& scratch,
                     int* keys, int* counts, int* offsets, int* cursors, int* segsum, void* stream, bool counted,
                     int* perm) {
  hipStream_t s = (hipStream_t)stream;
  if (p.np == 0) return PIC_OK;
  const dim3 grid((unsigned)((p.np + 255) / 256));
  if (!counted) {
    if (hipMemsetAsync(counts, 0, sizeof(int) * tg.nbins, s) != hipSuccess)
      return set_error(PIC_EHIP, "tile sort: clear counts");
    hipLaunchKernelGGL(tile_count_kernel, grid, dim3(256), 0, s, p.x[0], p.x[1], p.x[2], p.np, m, tg, keys, counts);
  }
  const int nseg = (tg.nbins + kScanSeg - 1) / kScanSeg;
  hipLaunchKernelGGL(tile_segsum_kernel, dim3(nseg), dim3(1024), 0, s, counts, tg.nbins, segsum);
  hipLaunchKernelGGL(tile_segscan_kernel, dim3(nseg), dim3(1024), 0, s, counts, tg.nbins, segsum, nseg, offsets,
                     cursors);
  if (perm)
    hipLaunchKernelGGL(tile_rank_kernel, dim3((unsigned)((p.np + 256 * kRankGroups - 1) / (256 * kRankGroups))),
                       dim3(256), 0, s, keys, offsets, cursors, p.np, perm);
  else
    hipLaunchKernelGGL(tile_scatter_kernel, grid, dim3(256), 0, s, p.x[0], p.x[1], p.x[2], p.u[0], p.u[1], p.u[2],
                       p.id, keys, offsets, cursors, p.np, scratch.x[0], scratch.x[1], scratch.x[2], scratch.u[0],
                       scratch.u[1], scratch.u[2], scratch.id);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "tile sort launch failed");
}

// ---------------------------------------------------------------------------
// Tile-ordered copies of a species for the vacuum step loop: the copy carries
// each particle's original index, through which it is scattered back.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void iota_kernel(int64_t* __restrict__ ids, int64_t np) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) ids[p] = p;
}

__global__ __launch_bounds__(256) void unsort_kernel(const double* __restrict__ x1, const double* __restrict__ x2,
                                                     const double* __restrict__ x3, const double* __restrict__ u1,
                                                     const double* __restrict__ u2, const double* __restrict__ u3,
                                                     const int64_t* __restrict__ ids, int64_t np,
                                                     double* __restrict__ dx1, double* __restrict__ dx2,
                                                     double* __restrict__ dx3, double* __restrict__ du1,
                                                     double* __restrict__ du2, double* __restrict__ du3) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int64_t q = ids[p];
  dx1[q] = x1[p];
  dx2[q] = x2[p];
  dx3[q] = x3[p];
  du1[q] = u1[p];
  du2[q] = u2[p];
  du3[q] = u3[p];
}

int launch_iota(int64_t* ids, int64_t np, void* stream) {
  if (np == 0) return PIC_OK;
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, (hipStream_t)stream, ids, np);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "iota launch failed");
}

int launch_unsort(const pic_particles& sorted, const int64_t* ids, const pic_particles& dst, void* stream) {
  if (sorted.np == 0) return PIC_OK;
  hipLaunchKernelGGL(unsort_kernel, dim3((unsigned)((sorted.np + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     sorted.x[0], sorted.x[1], sorted.x[2], sorted.u[0], sorted.u[1], sorted.u[2], ids, sorted.np,
                     dst.x[0], dst.x[1], dst.x[2], dst.u[0], dst.u[1], dst.u[2]);
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "unsort launch failed");
}

int launch_tile_push(int prec, const Mesh& m, const TileGeom& tg, void* const E[3], void* const B[3],
                     void* const J[3], const int* offsets, const pic_particles& src, const pic_particles& dst,
                     int pusher, double dt, double* stage, void* stream, int* keys, int* counts, const int* perm) {
  hipStream_t s = (hipStream_t)stream;
  if (src.np == 0) return PIC_OK;
  if (keys && hipMemsetAsync(counts, 0, sizeof(int) * tg.nbins, s) != hipSuccess)
    return set_error(PIC_EHIP, "tile push: clear counts");
  return prec == PIC_FP64
             ? run_tile_push<double>(m, tg, E, B, J, offsets, src, dst, pusher, dt, stage, keys, counts, perm, s)
             : run_tile_push<float>(m, tg, E, B, J, offsets, src, dst, pusher, dt, stage, keys, counts, perm, s);
}

int launch_tile_deposit(int prec, const Mesh& m, const TileGeom& tg, void* const J[3], const int* offsets,
                        const pic_particles& sorted, double dt, double* stage, void* stream, const int* perm) {
  hipStream_t s = (hipStream_t)stream;
  if (sorted.np == 0) return PIC_OK;
  return prec == PIC_FP64 ? run_tile_deposit<double>(m, tg, J, offsets, sorted, dt, stage, perm, s)
                          : run_tile_deposit<float>(m, tg, J, offsets, sorted, dt, stage, perm, s);
}

size_t stage_doubles(const TileGeom& tg) { return (size_t)tg.ntiles * 3 * tg.r[0] * tg.r[1] * tg.r[2]; }

}  // namespace yeepic
