// Internal declarations of the yeepic library (not part of the ABI).
#pragma once

#include <cstdint>

#include "yeepic.h"

namespace yeepic {

// Records a thread-local message for pic_last_error and returns ``code``.
int set_error(int code, const char* fmt, ...);

// Kernel widths: the coefficient count of each x1 operator rounded up to one
// of the compiled stencil widths (zero padding is exact).
constexpr int kWidths[5] = {1, 2, 4, 8, 16};
int round_width(int m);

// Mesh geometry and the grid's kernel settings, passed to every kernel.
struct Mesh {
  int n1, n2, n3;
  int ndim;
  int order;  // particle shape: 1 linear, 2 quadratic B-spline
  double dx1, dx2, dx3;
  double idx1, idx2, idx3;  // 1/dx: positions become cell coordinates by a multiply
  double L1, L2, L3;
  int exact_iters;  // iteration cap of the exact pusher's proper-time solve
  int* noconv;      // device counter of exact pushes whose solve hit the cap
};

// Field kernels (field_kernels.hip).  ``h`` is the time over which Faraday's
// law is applied (dt/2 for a half step); coefficients are the raw C_j.
template <typename T>
struct FieldSet {
  T* E[3];
  T* B[3];
};

// B step out of place: Bout = B - h curl_E E (Bout may be B).
int launch_advance_b(int prec, const Mesh& m, void* const E[3], void* const B[3], void* const Bout[3],
                     const double* CE, int ME, double h, void* stream);
int launch_advance_e(int prec, const Mesh& m, void* const E[3], void* const B[3],
                     void* const J[3], const double* CB, int MB, double dt, void* stream);
// Fused B-half / E / B-half sweep from (Ein, Bin) to (Eout, Bout); J may be
// all-null; Bh, if not NULL, also receives B^{n+1/2}.  In and out must not
// alias.
// x1 current correction (Sec. 3.3): out = periodic convolution along x1 of
// J1 with the symmetric taps h[0..kw] (h[-m] = h[m]); kw is 8, 16, 24, 32, 40, 48 or 64
int launch_correct_j1(int prec, const Mesh& m, const void* J1, void* out, const double* taps, int kw,
                      void* stream);
int launch_sweep(int prec, const Mesh& m, void* const Ein[3], void* const Bin[3],
                 void* const J[3], void* const Eout[3], void* const Bout[3], void* const Bh[3],
                 const double* CE, int ME, const double* CB, int MB, double dt, void* stream);

// Particle kernels (particle_kernels.hip).
int launch_gather_push(int prec, const Mesh& m, void* const E[3], void* const B[3],
                       const pic_particles& p, int pusher, double dt, double* const x_old[3],
                       void* stream);
int launch_deposit(int prec, const Mesh& m, void* const J[3], const pic_particles& p,
                   double* const x_old[3], double dt, void* stream);
// Spatial tiles of the sorted plasma path (plasma_kernels.hip).
struct TileGeom {
  int t[3];   // tile size in cells
  int nt[3];  // tiles per direction
  int m[3];   // drift margin in cells
  int r[3];   // nodes of the on-chip current tile per direction
  int ntiles;
  int sub;    // sort bins per tile: one per x3 cell plane and pair of x2 cell rows of the tile
  unsigned mt[3];  // cell / t[d] == umulhi(cell, mt[d]): floor(2^32 / t) + 1 (0 for t = 1, where cell is 0)
  int nbins;  // ntiles * sub: the sort's keys
};
TileGeom make_tile_geom(const Mesh& m, double dt, int sort_every);
// counting sort of p by tile into scratch; segsum holds scan_segments(ntiles)
// ints.  ``counted``: keys and counts of p already hold every particle's tile
// and the tiles' counts (written by the push that produced p).  With
// ``perm`` (np ints) nothing is moved: perm[q] receives the index in p of the
// particle whose sorted position is q, and scratch is not used.
int scan_segments(int ntiles);
int launch_tile_sort(const Mesh& m, const TileGeom& tg, const pic_particles& p, const pic_particles& scratch,
                     int* keys, int* counts, int* offsets, int* cursors, int* segsum, void* stream,
                     bool counted = false, int* perm = nullptr);
// ids[i] = i; dst[ids[i]] = sorted[i] for x and u (3D)
int launch_iota(int64_t* ids, int64_t np, void* stream);
int launch_unsort(const pic_particles& sorted, const int64_t* ids, const pic_particles& dst, void* stream);
// ``stage`` (deterministic mode, else nullptr) holds stage_doubles(tg) doubles:
// the tiles' currents are then stored there and summed per node in a fixed
// order instead of being added to J with atomics.
// ``keys``, ``counts`` (or nullptr): also write each pushed particle's tile
// key (indexed as dst) and the tiles' counts, for a sort of dst right after.
// ``perm`` (or nullptr): the particle at sorted position i is read from src
// at perm[i] (a sort's permutation; src and dst must then not alias), else
// from src at i.
int launch_tile_push(int prec, const Mesh& m, const TileGeom& tg, void* const E[3], void* const B[3],
                     void* const J[3], const int* offsets, const pic_particles& src, const pic_particles& dst,
                     int pusher, double dt, double* stage, void* stream, int* keys = nullptr,
                     int* counts = nullptr, const int* perm = nullptr);
// Esirkepov current of particles sorted by the tile of their old position:
// sorted.x holds the old positions, sorted.u the new ones; with ``perm`` the
// pair at sorted position i is read at perm[i].
int launch_tile_deposit(int prec, const Mesh& m, const TileGeom& tg, void* const J[3], const int* offsets,
                        const pic_particles& sorted, double dt, double* stage, void* stream,
                        const int* perm = nullptr);
size_t stage_doubles(const TileGeom& tg);

// Adjoint kernels (adjoint_kernels.hip).  launch_coef_grad adds
// scale * sum_i (la_i D_j fa_i - lb_i D_j fb_i) to g[j], j < M, where D_j is
// the Faraday (form 0) or Ampere (form 1) difference of lag j; ``partial``
// holds coef_partial_blocks(m) * PIC_MAX_M doubles.
int coef_partial_blocks(const Mesh& m);
int launch_coef_grad(const Mesh& m, int form, const double* la, const double* fa, const double* lb,
                     const double* fb, double scale, int M, double* partial, double* g, void* stream);
// Fused reverse of one 2D vacuum sweep with a one-coefficient Ampere
// stencil (C^B = cb1 e1): (lE, lB) at t^{n+1} -> (lEo, lBo) at t^n, out of
// place, from E^{n+1}, B^{n+1/2} and E^n; adds dL/dC^E and dL/dC^B (M
// entries).  ``partial`` holds adjoint_sweep2d_blocks(m) * 2 * PIC_MAX_M doubles
// (at most 256 workgroups).  adjoint_sweep2d_fits: the mesh is within the
// kernel's index range (a plane below 2^31 cells).
bool adjoint_sweep2d_fits(const Mesh& m);
int64_t adjoint_sweep2d_blocks(const Mesh& m);
int launch_adjoint_sweep2d(const Mesh& m, void* const lE[3], void* const lB[3], void* const lEo[3],
                           void* const lBo[3], const void* const Enext[3], const void* const Bhalf[3],
                           void* const En[3], const double* CE, int ME, double cb1, double dt, int M,
                           double* partial, double* gCE, double* gCB, void* stream);
int launch_adjoint_push(const Mesh& m, void* const E[3], void* const B[3], void* const lE[3], void* const lB[3],
                        const pic_particles& p, const pic_particles& lam, int pusher, double dt, void* stream);

// Moving window (window_kernels.hip).  launch_zero_columns clears columns
// [c0, c0 + s) mod n1 of every row of ``narrays`` (<= 9) field arrays;
// launch_window_count writes per-block survivor counts (window_blocks(np)
// ints) and their exclusive scan offs[0..nb] (offs[nb] = survivors) for a
// move of s columns from ring origin ``origin``; launch_window_scatter copies
// the survivors of src, in order, to dst[0 .. offs[nb]).
int launch_zero_columns(int prec, const Mesh& m, void* const* arrays, int narrays, int64_t c0, int64_t s,
                        void* stream);
int64_t window_blocks(int64_t np);
// Absorbing layers: damps E and B in the 2W window columns at the two x1
// ends (window cell s in array column (origin + s) mod n1); W = 0 does nothing.
int launch_damp_columns(int prec, const Mesh& m, void* const E[3], void* const B[3], int64_t origin, int W,
                        double sigma, void* stream);
int launch_window_count(const Mesh& m, const pic_particles& p, int64_t origin, int64_t s, int* counts,
                        int64_t* offs, void* stream);
int launch_window_scatter(const Mesh& m, const pic_particles& src, const pic_particles& dst, int64_t origin,
                          int64_t s, const int64_t* offs, void* stream);
int launch_check(int prec, const Mesh& m, void* const E[3], void* const B[3],
                 const pic_particles* p, int* d_flag, void* stream);

}  // namespace yeepic
