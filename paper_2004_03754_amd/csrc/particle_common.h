// Device helpers shared by the particle kernels: staggered linear-shape
// gather (App. A), Boris and exact constant-field pushers (Sec. 1, 4.1),
// periodic position wrap, Esirkepov shapes (Sec. 3.3).  All double precision.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "yeepic_internal.h"

namespace yeepic {
namespace pdev {

// Linear-shape nodes and weights along one direction for the component
// offset ``off`` (0 or 1/2 cell): u = x/dx - off, i0 = floor(u),
// w1 = u - i0 (App. A); x/dx is formed as x * (1/dx) (the linear shape is
// continuous, so the rounding of the cell coordinate only moves results by
// rounding).  The index is clamped into [-1, n] before the periodic wrap so
// that no input can address outside the mesh.
struct Axis {
  int i0, i1;
  double w0, w1;
};

__device__ __forceinline__ Axis axis(double x, double idx, double off, int n) {
  const double u = x * idx - off;
  double fl = floor(u);
  fl = fmin(fmax(fl, -1.0), (double)n);
  Axis a;
  a.w1 = u - fl;
  a.w0 = 1.0 - a.w1;
  int i = (int)fl;
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  a.i0 = i;
  a.i1 = (i + 1 == n) ? 0 : i + 1;
  return a;
}

// The two x1 nodes of row ``r``.  PAIR (the caller has checked that no
// lane's pair wraps around the periodic x1 edge): one load of two adjacent
// elements, which needs only element alignment (global memory on this part
// takes unaligned multi-dword loads).
template <bool PAIR, typename T>
__device__ __forceinline__ void row_pair(const T* __restrict__ r, const Axis& a, double& f0, double& f1) {
  if (PAIR) {
    struct P {
      T v[2];
    } p;
    __builtin_memcpy(&p, r + a.i0, sizeof(P));
    f0 = (double)p.v[0];
    f1 = (double)p.v[1];
  } else {
    f0 = (double)r[a.i0];
    f1 = (double)r[a.i1];
  }
}

template <bool PAIR = false, typename T>
__device__ __forceinline__ double interp3(const T* __restrict__ f, const Axis& a, const Axis& b, const Axis& c,
                                          int n1, size_t plane) {
  const size_t r00 = (size_t)c.i0 * plane + (size_t)b.i0 * n1;
  const size_t r01 = (size_t)c.i0 * plane + (size_t)b.i1 * n1;
  const size_t r10 = (size_t)c.i1 * plane + (size_t)b.i0 * n1;
  const size_t r11 = (size_t)c.i1 * plane + (size_t)b.i1 * n1;
  double f000, f001, f010, f011, f100, f101, f110, f111;
  row_pair<PAIR>(f + r00, a, f000, f001);
  row_pair<PAIR>(f + r01, a, f010, f011);
  row_pair<PAIR>(f + r10, a, f100, f101);
  row_pair<PAIR>(f + r11, a, f110, f111);
  return c.w0 * (b.w0 * (a.w0 * f000 + a.w1 * f001) + b.w1 * (a.w0 * f010 + a.w1 * f011)) +
         c.w1 * (b.w0 * (a.w0 * f100 + a.w1 * f101) + b.w1 * (a.w0 * f110 + a.w1 * f111));
}

// A 2D mesh with n3 > 1 is a stack of n3 independent 2D meshes (no coupling
// along x3); in 2D a particle's x3 holds the index of its plane (dx3 = 1 in
// 2D), floor(x3) clamped into [0, n3).  Returns the plane's element offset.
__device__ __forceinline__ size_t plane_offset(const Mesh& m, double x3) {
  if (m.n3 == 1) return 0;
  const double k = fmin(fmax(floor(x3), 0.0), (double)(m.n3 - 1));
  return (size_t)k * m.n1 * m.n2;
}

template <typename T>
__device__ __forceinline__ double interp2(const T* __restrict__ f, const Axis& a, const Axis& b, int n1) {
  const size_t r0 = (size_t)b.i0 * n1, r1 = (size_t)b.i1 * n1;
  return b.w0 * (a.w0 * (double)f[r0 + a.i0] + a.w1 * (double)f[r0 + a.i1]) +
         b.w1 * (a.w0 * (double)f[r1 + a.i0] + a.w1 * (double)f[r1 + a.i1]);
}

// ---------------------------------------------------------------------------
// Boris (Sec. 1): half E kick, rotation about B, half E kick.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void boris(double u[3], const double E[3], const double B[3], double qm, double dt) {
  const double eps = 0.5 * qm * dt;
  double um[3] = {u[0] + eps * E[0], u[1] + eps * E[1], u[2] + eps * E[2]};
  const double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  const double eg = eps / g;
  const double t[3] = {eg * B[0], eg * B[1], eg * B[2]};
  const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  const double f = 2.0 / (1.0 + tt);
  const double s[3] = {f * t[0], f * t[1], f * t[2]};
  const double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                        um[2] + (um[0] * t[1] - um[1] * t[0])};
  u[0] = um[0] + (up[1] * s[2] - up[2] * s[1]) + eps * E[0];
  u[1] = um[1] + (up[2] * s[0] - up[0] * s[2]) + eps * E[1];
  u[2] = um[2] + (up[0] * s[1] - up[1] * s[0]) + eps * E[2];
}

// Higuera-Cary push (Sec. 1, Sec. 4.1: the published method the paper cites):
// the Boris splitting with the rotation vector t = tau/gamma_r, tau =
// (q dt/2m) B, at the Lorentz factor
//   gamma_r^2 = (sigma + sqrt(sigma^2 + 4 (tau^2 + (u-.tau)^2)))/2,
//   sigma = 1 + u-^2 - tau^2,
// then u+ = (u- + (u-.t) t + u- x t)/(1 + t^2) and u = u+ + (q dt/2m) E + u+ x t.
__device__ __forceinline__ void higuera_cary(double u[3], const double E[3], const double B[3], double qm,
                                             double dt) {
  const double eps = 0.5 * qm * dt;
  const double um[3] = {u[0] + eps * E[0], u[1] + eps * E[1], u[2] + eps * E[2]};
  const double tau[3] = {eps * B[0], eps * B[1], eps * B[2]};
  const double tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
  const double ust = um[0] * tau[0] + um[1] * tau[1] + um[2] * tau[2];
  const double sigma = 1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2] - tau2;
  const double gr = sqrt(0.5 * (sigma + sqrt(sigma * sigma + 4.0 * (tau2 + ust * ust))));
  const double t[3] = {tau[0] / gr, tau[1] / gr, tau[2] / gr};
  const double s = 1.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  const double ut = um[0] * t[0] + um[1] * t[1] + um[2] * t[2];
  const double up[3] = {s * (um[0] + ut * t[0] + (um[1] * t[2] - um[2] * t[1])),
                        s * (um[1] + ut * t[1] + (um[2] * t[0] - um[0] * t[2])),
                        s * (um[2] + ut * t[2] + (um[0] * t[1] - um[1] * t[0]))};
  u[0] = up[0] + eps * E[0] + (up[1] * t[2] - up[2] * t[1]);
  u[1] = up[1] + eps * E[1] + (up[2] * t[0] - up[0] * t[2]);
  u[2] = up[2] + eps * E[2] + (up[0] * t[1] - up[1] * t[0]);
}

// ---------------------------------------------------------------------------
// Exact push for fields constant over the step (Sec. 1, Sec. 4.1).
//
// With F = (q/m) Lambda(E, B) acting on U = (gamma, u), U(tau) = exp(F tau) U0
// in proper time.  F has eigenvalues +-kappa, +-i omega with
//   kappa^2 - omega^2 = (q/m)^2 (E^2 - B^2),  kappa omega = (q/m)^2 |E.B|,
// so by Cayley-Hamilton exp(F tau) = a0 + a1 F + a2 F^2 + a3 F^3 and the
// lab time is t(tau) = e0 . (A0 + A1 F + A2 F^2 + A3 F^3) U0 with
// A_k = int_0^tau a_k.  With X = (kappa tau)^2, Y = (omega tau)^2 every
// coefficient is an entire function of (X, -Y):
//   a0 = 1 + XY G4, a1 = tau (1 + XY G5), a2 = tau^2 G2, a3 = tau^3 G3,
//   A0 = a1, A1 = tau^2 (1/2 + XY G6), A2 = a3, A3 = tau^4 G4,
//   G_m = sum_k h_k(X, -Y)/(2k+m)!,  h_k = complete homogeneous polynomial.
// For max(X, Y) <= 1 the series is summed; otherwise the hyperbolic /
// trigonometric closed forms are used, written without cancellation where a
// cancellation-free form exists.  t(tau) = dt is solved by bracketed Newton
// (t increases with dt/dtau = gamma >= 1, root between 0 and dt) from a
// first guess on the Taylor polynomial of t: plain Newton near the root, on
// log(t/dt) far from it, stopping when the correction is below the rounding
// of tau.
// ---------------------------------------------------------------------------
struct ExpCoef {
  double a0, a1, a2, a3, A1, A3;  // A0 = a1, A2 = a3
};

// 1/n! for n = 0..32, evaluated at compile time: the series reads
// 1/(2k + m)! for k < 14, m = 2..6 as constants (no divisions at run time).
struct InvFact {
  double v[33];
  constexpr InvFact() : v() {
    double f = 1.0;
    v[0] = 1.0;
    for (int n = 1; n < 33; ++n) {
      f *= n;
      v[n] = 1.0 / f;
    }
  }
};
__device__ constexpr InvFact kInvFact{};

__device__ __forceinline__ ExpCoef exp_coef(double k2, double w2, double tau) {
  const double t2 = tau * tau;
  const double X = k2 * t2, Y = w2 * t2;
  ExpCoef e;
  if (X <= 1.0 && Y <= 1.0) {
    // G_m for m = 2..6 from h_k(X, Z), Z = -Y; 14 terms reach below 1e-19
    const double Z = -Y;
    double h = 1.0, zk = 1.0;
    double G[7] = {0, 0, 0, 0, 0, 0, 0};
    // terms beyond k are below v^k/(2k+2)! with v = max(X, Y): 14 terms reach
    // 1e-19 at v = 1, 8 at v <= 1/16, 5 at v <= 1/256
    const double v = fmax(X, Y);
    const int nk = v > 0.0625 ? 14 : (v > 0.00390625 ? 8 : 5);
#pragma unroll
    for (int k = 0; k < 14; ++k) {
      if (k >= nk) break;
      G[2] += h * kInvFact.v[2 * k + 2];
      G[3] += h * kInvFact.v[2 * k + 3];
      G[4] += h * kInvFact.v[2 * k + 4];
      G[5] += h * kInvFact.v[2 * k + 5];
      G[6] += h * kInvFact.v[2 * k + 6];
      zk *= Z;
      h = X * h + zk;  // h_{k+1} = X h_k + Z^{k+1}
    }
    const double XY = X * Y;
    e.a0 = 1.0 + XY * G[4];
    e.a1 = tau * (1.0 + XY * G[5]);
    e.a2 = t2 * G[2];
    e.a3 = t2 * tau * G[3];
    e.A1 = t2 * (0.5 + XY * G[6]);
    e.A3 = t2 * t2 * G[4];
    return e;
  }
  const double kap = sqrt(k2), om = sqrt(w2);
  const double x = kap * tau, y = om * tau;
  // sinh(x)/kappa, (cosh x - 1)/kappa^2, sin(y)/omega, (1 - cos y)/omega^2
  double sh, ch1, sn, cs1;
  if (fabs(x) < 1e-4) {
    sh = tau * (1.0 + X / 6.0 * (1.0 + X / 20.0));
    ch1 = t2 * 0.5 * (1.0 + X / 12.0 * (1.0 + X / 30.0));
  } else {
    sh = sinh(x) / kap;
    const double s = sinh(0.5 * x) / kap;
    ch1 = 2.0 * s * s;
  }
  if (fabs(y) < 1e-4) {
    sn = tau * (1.0 - Y / 6.0 * (1.0 - Y / 20.0));
    cs1 = t2 * 0.5 * (1.0 - Y / 12.0 * (1.0 - Y / 30.0));
  } else {
    sn = sin(y) / om;
    const double s = sin(0.5 * y) / om;
    cs1 = 2.0 * s * s;
  }
  const double inv = 1.0 / (k2 + w2);
  const double chx = 1.0 + k2 * ch1, cy = 1.0 - w2 * cs1;  // cosh x, cos y
  e.a0 = (w2 * chx + k2 * cy) * inv;
  e.a1 = (w2 * sh + k2 * sn) * inv;
  e.a2 = (k2 * ch1 + w2 * cs1) * inv;
  e.a3 = (sh - sn) * inv;
  e.A1 = (w2 * ch1 + k2 * cs1) * inv;
  e.A3 = (ch1 - cs1) * inv;
  return e;
}

__device__ __forceinline__ void apply_F(const double E[3], const double B[3], double qm, const double v[4],
                                        double o[4]) {
  o[0] = qm * (E[0] * v[1] + E[1] * v[2] + E[2] * v[3]);
  o[1] = qm * (E[0] * v[0] + B[2] * v[2] - B[1] * v[3]);
  o[2] = qm * (E[1] * v[0] - B[2] * v[1] + B[0] * v[3]);
  o[3] = qm * (E[2] * v[0] + B[1] * v[1] - B[0] * v[2]);
}

// The exact push's state before the exponential: invariants kappa^2,
// omega^2, U0 = (gamma, u) and F U0, F^2 U0, F^3 U0.
struct ExactState {
  double k2, w2;
  double U0[4], V1[4], V2[4], V3[4];
};

// Solves t(tau) = dt for the exact push of u in (E, B); returns tau and the
// state the exponential is applied to.  ``conv`` is set false when the solve
// ends by exhausting ``max_iter`` iterations instead of by one of its
// stopping tests.
__device__ __forceinline__ double analytic_solve(const double u[3], const double E[3], const double B[3], double qm,
                                                 double dt, ExactState& st, int max_iter, bool& conv) {
  const double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
  const double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const double EB = E[0] * B[0] + E[1] * B[1] + E[2] * B[2];
  const double q2 = qm * qm;
  const double P = 0.5 * (E2 - B2);
  const double Q = sqrt(P * P + EB * EB);
  double k2, w2;  // kappa^2, omega^2 without cancellation
  if (P >= 0) {
    k2 = q2 * (P + Q);
    w2 = (P + Q) > 0 ? q2 * (EB * EB) / (P + Q) : 0.0;
  } else {
    w2 = q2 * (Q - P);
    k2 = q2 * (EB * EB) / (Q - P);
  }
  st.k2 = k2;
  st.w2 = w2;
  double* U0 = st.U0;
  double* V1 = st.V1;
  double* V2 = st.V2;
  double* V3 = st.V3;
  U0[0] = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  U0[1] = u[0];
  U0[2] = u[1];
  U0[3] = u[2];
  apply_F(E, B, qm, U0, V1);
  apply_F(E, B, qm, V1, V2);
  apply_F(E, B, qm, V2, V3);
  double lo = fmin(0.0, dt), hi = fmax(0.0, dt);
  // First guess: from dt/gamma, two Newton steps on the Taylor polynomial
  // t(tau) ~ gamma tau + (F U)^0 tau^2/2 + (F^2 U)^0 tau^3/6 + (F^3 U)^0 tau^4/24
  // (exact where F^4 U = 0, e.g. a null field), kept only while it rises and
  // stays in the bracket; then pulled in so that exp(sqrt(k2 + w2) tau)
  // stays finite.
  const double kw = sqrt(k2 + w2);
  double tau = dt / U0[0];
  {
    const double c1 = 0.5 * V1[0], c2 = V2[0] / 6.0, c3 = V3[0] / 24.0;
    for (int s = 0; s < 2; ++s) {
      const double p = (((c3 * tau + c2) * tau + c1) * tau + U0[0]) * tau - dt;
      const double dp = ((4.0 * c3 * tau + 3.0 * c2) * tau + 2.0 * c1) * tau + U0[0];
      const double nt = tau - p / dp;
      if (!(dp > 0.0) || !(nt > lo && nt < hi)) break;
      tau = nt;
    }
  }
  if (kw * fabs(tau) > 50.0) tau = copysign(50.0 / kw, dt);
  conv = false;
  // the last two step lengths: a step that is not below half of the one
  // before the last one is replaced by bisection, so that steps that cross
  // the root back and forth (Newton on log t can cycle between the two ends
  // of the bracket when t rises steeply past the root) still halve the
  // bracket every other iteration
  double dx = hi - lo, dxold = dx;
  for (int it = 0; it < max_iter; ++it) {
    const ExpCoef e = exp_coef(k2, w2, tau);
    const double t = e.a1 * U0[0] + e.A1 * V1[0] + e.a3 * V2[0] + e.A3 * V3[0];
    const double g = e.a0 * U0[0] + e.a1 * V1[0] + e.a2 * V2[0] + e.a3 * V3[0];
    const bool fin = isfinite(t) && isfinite(g) && g > 0.0;
    const double f = t - dt;
    if (fin && fabs(f) <= 1e-16 * fabs(dt)) {
      conv = true;
      break;
    }
    // keep the root bracketed; a non-finite value lies beyond it, away from 0
    if (fin ? f > 0.0 : dt > 0.0) hi = tau; else lo = tau;
    // Far from the root (t/dt outside (1/2, 2)) the step is Newton on
    // log(t/dt): where t grows exponentially log t is close to linear, and for
    // a particle accelerated from rest it is concave, so the step does not
    // overshoot (a plain Newton step on the steep, convex t does, far past the
    // root).  Near the root plain Newton is as fast and needs no logarithm:
    // from t = dt/2 it reaches at most e/2 dt.  The bracket guards the rest.
    const double ratio = t / dt;
    double nx;
    if (!fin || !(ratio > 0.0)) {
      nx = 0.5 * (lo + hi);
    } else if (ratio > 0.5 && ratio < 2.0) {
      // a Newton correction below the rounding of tau ends the solve: t is
      // then at its rounding floor, which can stay above 1e-16 dt
      const double step = f / g;
      if (fabs(step) <= 1e-15 * fabs(tau)) {
        conv = true;
        break;
      }
      nx = tau - step;
    } else {
      nx = tau - log(ratio) * (t / g);
    }
    if (!(nx > lo && nx < hi) || fabs(nx - tau) > 0.5 * dxold) nx = 0.5 * (lo + hi);
    dxold = dx;
    dx = fabs(nx - tau);
    const bool small = fabs(nx - tau) <= 1e-15 * fabs(tau);
    tau = nx;
    if (small) {
      conv = true;
      break;
    }
  }
  return tau;
}

// Counts an exact push whose proper-time solve did not converge (read and
// cleared by pic_check).
__device__ __forceinline__ void note_noconv(const Mesh& m) {
  if (m.noconv) atomicAdd(m.noconv, 1);
}

__device__ __forceinline__ void analytic(double u[3], const double E[3], const double B[3], double qm, double dt,
                                         const Mesh& m) {
  ExactState st;
  bool conv;
  const double tau = analytic_solve(u, E, B, qm, dt, st, m.exact_iters, conv);
  if (!conv) note_noconv(m);
  const ExpCoef e = exp_coef(st.k2, st.w2, tau);
  for (int d = 0; d < 3; ++d)
    u[d] = e.a0 * st.U0[d + 1] + e.a1 * st.V1[d + 1] + e.a2 * st.V2[d + 1] + e.a3 * st.V3[d + 1];
}

// periodic wrap of an advanced position (the oracle's rule)
__device__ __forceinline__ double wrap_pos(double x, double L) {
  if (x < 0.0) {
    x += L;
    if (x >= L) x = 0.0;
  } else if (x >= L) {
    x -= L;
  }
  return x;
}

// ---------------------------------------------------------------------------
// Esirkepov deposit (Sec. 3.3).  Local K-node stencils per direction: linear
// shape K = 3 starting at min(floor(X0), floor(X1)); quadratic B-spline
// (the Sec. 4.2 run's shape) K = 4 starting one node left of the smaller of
// the nearest nodes round(X0), round(X1).  J_d is the running sum of W_d
// along d times -q w dx_d/dt.
// ---------------------------------------------------------------------------
template <int K>
struct ShapeK {
  int base;
  double s0[K], ds[K];
};
using Shape3 = ShapeK<3>;
using Shape4 = ShapeK<4>;

__device__ __forceinline__ Shape3 shape3(double xo, double xn, double idx, double L) {
  double d = xn - xo;  // minimum image
  if (d > 0.5 * L) d -= L;
  if (d < -0.5 * L) d += L;
  const double X0 = xo * idx, X1 = (xo + d) * idx;
  const double f0 = floor(X0), f1 = floor(X1);
  const double b = fmin(f0, f1);
  const double r0 = X0 - f0, r1 = X1 - f1;
  int a0 = (int)(f0 - b), a1 = (int)(f1 - b);
  a0 = a0 < 0 ? 0 : (a0 > 1 ? 1 : a0);
  a1 = a1 < 0 ? 0 : (a1 > 1 ? 1 : a1);
  Shape3 s;
  double s1[3] = {0, 0, 0};
  s.s0[0] = s.s0[1] = s.s0[2] = 0;
  s.s0[a0] = 1.0 - r0;
  s.s0[a0 + 1] = r0;
  s1[a1] = 1.0 - r1;
  s1[a1 + 1] = r1;
  for (int q = 0; q < 3; ++q) s.ds[q] = s1[q] - s.s0[q];
  s.base = (int)fmin(fmax(b, -2.0), 1e9);
  return s;
}

// quadratic B-spline weights at offset d = X - round(X) from the nearest node
__device__ __forceinline__ void bspline2(double d, double w[3]) {
  w[0] = 0.5 * (0.5 - d) * (0.5 - d);
  w[1] = 0.75 - d * d;
  w[2] = 0.5 * (0.5 + d) * (0.5 + d);
}

__device__ __forceinline__ Shape4 shape4(double xo, double xn, double idx, double L) {
  double d = xn - xo;  // minimum image
  if (d > 0.5 * L) d -= L;
  if (d < -0.5 * L) d += L;
  const double X0 = xo * idx, X1 = (xo + d) * idx;
  const double i0 = floor(X0 + 0.5), i1 = floor(X1 + 0.5);
  const double b = fmin(i0, i1) - 1.0;
  int a0 = (int)(i0 - 1.0 - b), a1 = (int)(i1 - 1.0 - b);
  a0 = a0 < 0 ? 0 : (a0 > 1 ? 1 : a0);
  a1 = a1 < 0 ? 0 : (a1 > 1 ? 1 : a1);
  double w0[3], w1[3];
  bspline2(X0 - i0, w0);
  bspline2(X1 - i1, w1);
  Shape4 s;
#pragma unroll
  for (int k = 0; k < 4; ++k) {  // selects, not indexed stores: the arrays stay in registers
    const double s0 = k == a0 ? w0[0] : (k == a0 + 1 ? w0[1] : (k == a0 + 2 ? w0[2] : 0.0));
    const double s1 = k == a1 ? w1[0] : (k == a1 + 1 ? w1[1] : (k == a1 + 2 ? w1[2] : 0.0));
    s.s0[k] = s0;
    s.ds[k] = s1 - s0;
  }
  s.base = (int)fmin(fmax(b, -3.0), 1e9);
  return s;
}

__device__ __forceinline__ int wrapn(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, double v) {
  unsafeAtomicAdd(p, (T)v);
}


}  // namespace pdev
}  // namespace yeepic

namespace yeepic {
namespace pdev {

// E^n and B^n at x from the six staggered component arrays (App. A).
template <typename T, int NDIM>
__device__ __forceinline__ void gather6(const T* __restrict__ E1, const T* __restrict__ E2, const T* __restrict__ E3,
                                        const T* __restrict__ B1, const T* __restrict__ B2, const T* __restrict__ B3,
                                        const Mesh& m, const double x[3], double E[3], double B[3]) {
  const Axis a0 = axis(x[0], m.idx1, 0.0, m.n1), ah = axis(x[0], m.idx1, 0.5, m.n1);
  const Axis b0 = axis(x[1], m.idx2, 0.0, m.n2), bh = axis(x[1], m.idx2, 0.5, m.n2);
  if (NDIM == 3) {
    const Axis c0 = axis(x[2], m.idx3, 0.0, m.n3), ch = axis(x[2], m.idx3, 0.5, m.n3);
    const size_t pl = (size_t)m.n1 * m.n2;
    // FP64 fields: pairs of x1 nodes in one 16-byte load when no lane of the
    // wave wraps in x1 (only waves at the last x1 cell column do).  FP32
    // pairs would be unaligned 8-byte loads, measured slower than two loads
    // in the plasma push.
    if (sizeof(T) == 8 && __builtin_amdgcn_ballot_w64(a0.i1 == 0 || ah.i1 == 0) == 0) {
      E[0] = interp3<true>(E1, ah, b0, c0, m.n1, pl);
      E[1] = interp3<true>(E2, a0, bh, c0, m.n1, pl);
      E[2] = interp3<true>(E3, a0, b0, ch, m.n1, pl);
      B[0] = interp3<true>(B1, a0, bh, ch, m.n1, pl);
      B[1] = interp3<true>(B2, ah, b0, ch, m.n1, pl);
      B[2] = interp3<true>(B3, ah, bh, c0, m.n1, pl);
    } else {
      E[0] = interp3(E1, ah, b0, c0, m.n1, pl);
      E[1] = interp3(E2, a0, bh, c0, m.n1, pl);
      E[2] = interp3(E3, a0, b0, ch, m.n1, pl);
      B[0] = interp3(B1, a0, bh, ch, m.n1, pl);
      B[1] = interp3(B2, ah, b0, ch, m.n1, pl);
      B[2] = interp3(B3, ah, bh, c0, m.n1, pl);
    }
  } else {
    const size_t o = plane_offset(m, x[2]);
    E[0] = interp2(E1 + o, ah, b0, m.n1);
    E[1] = interp2(E2 + o, a0, bh, m.n1);
    E[2] = interp2(E3 + o, a0, b0, m.n1);
    B[0] = interp2(B1 + o, a0, bh, m.n1);
    B[1] = interp2(B2 + o, ah, b0, m.n1);
    B[2] = interp2(B3 + o, ah, bh, m.n1);
  }
}

// Quadratic B-spline gather (the Sec. 4.2 run's shape): the three nodes
// around the nearest one, round(X), along each direction, wrapped
// periodically (positions outside the box are clamped as in ``axis``).
struct AxisQ {
  int i[3];
  double w[3];
};

__device__ __forceinline__ AxisQ axisq(double x, double idx, double off, int n) {
  const double u = x * idx - off;
  double c = floor(u + 0.5);
  c = fmin(fmax(c, -1.0), (double)n);
  AxisQ a;
  bspline2(u - c, a.w);
  const int ic = (int)c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int i = (ic - 1 + k) % n;
    a.i[k] = i < 0 ? i + n : i;
  }
  return a;
}

template <typename T>
__device__ __forceinline__ double interp3q(const T* __restrict__ f, const AxisQ& a, const AxisQ& b, const AxisQ& c,
                                           int n1, size_t plane) {
  double acc = 0;
#pragma unroll
  for (int kc = 0; kc < 3; ++kc) {
    double accb = 0;
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) {
      const T* r = f + (size_t)c.i[kc] * plane + (size_t)b.i[kb] * n1;
      accb += b.w[kb] * (a.w[0] * (double)r[a.i[0]] + a.w[1] * (double)r[a.i[1]] + a.w[2] * (double)r[a.i[2]]);
    }
    acc += c.w[kc] * accb;
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ double interp2q(const T* __restrict__ f, const AxisQ& a, const AxisQ& b, int n1) {
  double acc = 0;
#pragma unroll
  for (int kb = 0; kb < 3; ++kb) {
    const T* r = f + (size_t)b.i[kb] * n1;
    acc += b.w[kb] * (a.w[0] * (double)r[a.i[0]] + a.w[1] * (double)r[a.i[1]] + a.w[2] * (double)r[a.i[2]]);
  }
  return acc;
}

template <typename T, int NDIM>
__device__ __forceinline__ void gather6q(const T* __restrict__ E1, const T* __restrict__ E2, const T* __restrict__ E3,
                                         const T* __restrict__ B1, const T* __restrict__ B2, const T* __restrict__ B3,
                                         const Mesh& m, const double x[3], double E[3], double B[3]) {
  const AxisQ a0 = axisq(x[0], m.idx1, 0.0, m.n1), ah = axisq(x[0], m.idx1, 0.5, m.n1);
  const AxisQ b0 = axisq(x[1], m.idx2, 0.0, m.n2), bh = axisq(x[1], m.idx2, 0.5, m.n2);
  if (NDIM == 3) {
    const AxisQ c0 = axisq(x[2], m.idx3, 0.0, m.n3), ch = axisq(x[2], m.idx3, 0.5, m.n3);
    const size_t pl = (size_t)m.n1 * m.n2;
    E[0] = interp3q(E1, ah, b0, c0, m.n1, pl);
    E[1] = interp3q(E2, a0, bh, c0, m.n1, pl);
    E[2] = interp3q(E3, a0, b0, ch, m.n1, pl);
    B[0] = interp3q(B1, a0, bh, ch, m.n1, pl);
    B[1] = interp3q(B2, ah, b0, ch, m.n1, pl);
    B[2] = interp3q(B3, ah, bh, c0, m.n1, pl);
  } else {
    const size_t o = plane_offset(m, x[2]);
    E[0] = interp2q(E1 + o, ah, b0, m.n1);
    E[1] = interp2q(E2 + o, a0, bh, m.n1);
    E[2] = interp2q(E3 + o, a0, b0, m.n1);
    B[0] = interp2q(B1 + o, a0, bh, m.n1);
    B[1] = interp2q(B2 + o, ah, b0, m.n1);
    B[2] = interp2q(B3 + o, ah, bh, m.n1);
  }
}

// the gather of shape order ORDER (1 linear, 2 quadratic)
template <typename T, int NDIM, int ORDER>
__device__ __forceinline__ void gather_o(const T* __restrict__ E1, const T* __restrict__ E2, const T* __restrict__ E3,
                                         const T* __restrict__ B1, const T* __restrict__ B2, const T* __restrict__ B3,
                                         const Mesh& m, const double x[3], double E[3], double B[3]) {
  if constexpr (ORDER == 2)
    gather6q<T, NDIM>(E1, E2, E3, B1, B2, B3, m, x, E, B);
  else
    gather6<T, NDIM>(E1, E2, E3, B1, B2, B3, m, x, E, B);
}

// the deposit stencil of shape order ORDER
template <int ORDER>
__device__ __forceinline__ ShapeK<ORDER + 2> shape_o(double xo, double xn, double idx, double L) {
  if constexpr (ORDER == 2)
    return shape4(xo, xn, idx, L);
  else
    return shape3(xo, xn, idx, L);
}

// Esirkepov 3D decomposition (Sec. 3.3, cited method): for each node
// (a, b, c) of the K x K x K local stencil, add the current contributions
// J_d = -q w (dx_d/dt) * (running sum of W_d along d).  ``add(comp, a, b, c, v)``
// receives stencil-local node indices.  N1, N2, N3 < K: only the first K - 1
// nodes along that direction, for particles known not to change cell
// (nearest node, at the quadratic shape) along it, whose last node there
// carries no weight.  SKIP: exactly zero contributions are not passed to
// ``add`` when some direction takes its full stencil (for adds that cost
// more than the test: global atomics, two-word accumulators).
template <int K, int N1 = K, int N2 = K, int N3 = K, bool SKIP = true, typename Add>
__device__ __forceinline__ void esirkepov(const ShapeK<K>& sx, const ShapeK<K>& sy, const ShapeK<K>& sz, double c1,
                                          double c2, double c3, Add add) {
  static_assert((N1 == K || N1 == K - 1) && (N2 == K || N2 == K - 1) && (N3 == K || N3 == K - 1), "node count");
  // The running sum of W_d along d is (prefix sum of the shape differences
  // up to the node) times the transverse weight.  With SKIP, exactly zero
  // contributions are skipped when some direction takes its full stencil
  // (where every particle without a cell change along it leaves a row of
  // them), never on the short one, where they are rare.  A particle that
  // stays in its cell along d has an empty last node there, so the prefix sum
  // up to the node before it is exactly zero; it is set so (the differences'
  // rounding would leave a residue), which makes the full loop give the same
  // contributions as the short one for such a particle.
  constexpr bool kSkipZero = SKIP && (N1 == K || N2 == K || N3 == K);
  auto prefix = [](const ShapeK<K>& sh, auto& cs, auto nn) {
    constexpr int N = decltype(nn)::value;
    cs[0] = sh.ds[0];
#pragma unroll
    for (int n = 1; n < N - 1; ++n) cs[n] = cs[n - 1] + sh.ds[n];
    if (N == K && sh.s0[K - 1] == 0.0 && sh.ds[K - 1] == 0.0) cs[N - 2] = 0.0;
  };
  double cx[N1 > 1 ? N1 - 1 : 1], cy[N2 > 1 ? N2 - 1 : 1], cz[N3 > 1 ? N3 - 1 : 1];
  prefix(sx, cx, std::integral_constant<int, N1>{});
  prefix(sy, cy, std::integral_constant<int, N2>{});
  prefix(sz, cz, std::integral_constant<int, N3>{});
  // The transverse weight of W_d at nodes (p, q) of the two other directions,
  //   S0_p S0_q + (dS_p S0_q + S0_p dS_q)/2 + dS_p dS_q/3,
  // taken as S0_p h_q + dS_p k_q with h = S0 + dS/2, k = S0/2 + dS/3 (the
  // same quantity, two operations per node)
  double hy[N2], ky[N2], hz[N3], kz[N3];
#pragma unroll
  for (int n = 0; n < N2; ++n) {
    hy[n] = sy.s0[n] + 0.5 * sy.ds[n];
    ky[n] = 0.5 * sy.s0[n] + (1.0 / 3.0) * sy.ds[n];
  }
#pragma unroll
  for (int n = 0; n < N3; ++n) {
    hz[n] = sz.s0[n] + 0.5 * sz.ds[n];
    kz[n] = 0.5 * sz.s0[n] + (1.0 / 3.0) * sz.ds[n];
  }
#pragma unroll
  for (int b = 0; b < N2; ++b)
#pragma unroll
    for (int c = 0; c < N3; ++c) {
      const double w = sy.s0[b] * hz[c] + sy.ds[b] * kz[c];
#pragma unroll
      for (int a = 0; a < N1 - 1; ++a) {
        const double run = cx[a] * w;
        if (!kSkipZero || run != 0.0) add(0, a, b, c, c1 * run);
      }
    }
#pragma unroll
  for (int a = 0; a < N1; ++a)
#pragma unroll
    for (int c = 0; c < N3; ++c) {
      const double w = sx.s0[a] * hz[c] + sx.ds[a] * kz[c];
#pragma unroll
      for (int b = 0; b < N2 - 1; ++b) {
        const double run = cy[b] * w;
        if (!kSkipZero || run != 0.0) add(1, a, b, c, c2 * run);
      }
    }
#pragma unroll
  for (int a = 0; a < N1; ++a)
#pragma unroll
    for (int b = 0; b < N2; ++b) {
      const double w = sx.s0[a] * hy[b] + sx.ds[a] * ky[b];
#pragma unroll
      for (int c = 0; c < N3 - 1; ++c) {
        const double run = cz[c] * w;
        if (!kSkipZero || run != 0.0) add(2, a, b, c, c3 * run);
      }
    }
}

}  // namespace pdev
}  // namespace yeepic
