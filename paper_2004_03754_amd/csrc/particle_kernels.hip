// Particle kernels (gfx950): staggered linear-shape gather, Boris and exact
// constant-field pushers, leapfrog position update, Esirkepov deposit.
// All particle arithmetic is double precision; field values are promoted.
#include <hip/hip_runtime.h>

#include "particle_common.h"

namespace yeepic {
namespace {

using namespace pdev;


template <typename T, int PUSH, int NDIM, int ORDER>
__global__ __launch_bounds__(256) void gather_push_kernel(const T* __restrict__ E1, const T* __restrict__ E2,
                                                          const T* __restrict__ E3, const T* __restrict__ B1,
                                                          const T* __restrict__ B2, const T* __restrict__ B3,
                                                          Mesh m, double* __restrict__ x1, double* __restrict__ x2,
                                                          double* __restrict__ x3, double* __restrict__ u1,
                                                          double* __restrict__ u2, double* __restrict__ u3,
                                                          int64_t np, double qm, double dt,
                                                          double* __restrict__ o1, double* __restrict__ o2,
                                                          double* __restrict__ o3) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  // particle state is streamed once: non-temporal loads and stores keep it
  // from evicting the field lines the gathers share in L2
  double x[3] = {__builtin_nontemporal_load(x1 + p), __builtin_nontemporal_load(x2 + p),
                 (NDIM == 3 || m.n3 > 1) ? __builtin_nontemporal_load(x3 + p) : 0.0};
  double u[3] = {__builtin_nontemporal_load(u1 + p), __builtin_nontemporal_load(u2 + p),
                 __builtin_nontemporal_load(u3 + p)};
  double E[3], B[3];
  gather_o<T, NDIM, ORDER>(E1, E2, E3, B1, B2, B3, m, x, E, B);
  if (PUSH == PIC_PUSH_BORIS)
    boris(u, E, B, qm, dt);
  else if (PUSH == PIC_PUSH_HC)
    higuera_cary(u, E, B, qm, dt);
  else
    analytic(u, E, B, qm, dt, m);
  const double ig = dt / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  if (o1) {
    __builtin_nontemporal_store(x[0], o1 + p);
    __builtin_nontemporal_store(x[1], o2 + p);
    if (NDIM == 3 && o3) __builtin_nontemporal_store(x[2], o3 + p);
  }
  __builtin_nontemporal_store(wrap_pos(x[0] + ig * u[0], m.L1), x1 + p);
  __builtin_nontemporal_store(wrap_pos(x[1] + ig * u[1], m.L2), x2 + p);
  if (NDIM == 3) __builtin_nontemporal_store(wrap_pos(x[2] + ig * u[2], m.L3), x3 + p);
  __builtin_nontemporal_store(u[0], u1 + p);
  __builtin_nontemporal_store(u[1], u2 + p);
  __builtin_nontemporal_store(u[2], u3 + p);
}

template <typename T, int NDIM, int ORDER>
__global__ __launch_bounds__(256) void deposit_kernel(T* __restrict__ J1, T* __restrict__ J2, T* __restrict__ J3,
                                                      Mesh m, const double* __restrict__ x1,
                                                      const double* __restrict__ x2, const double* __restrict__ x3,
                                                      const double* __restrict__ xo1,
                                                      const double* __restrict__ xo2,
                                                      const double* __restrict__ xo3,
                                                      const double* __restrict__ u1, const double* __restrict__ u2,
                                                      const double* __restrict__ u3, int64_t np, double qw,
                                                      double dt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  constexpr int K = ORDER + 2;  // stencil nodes per direction
  const ShapeK<K> sx = shape_o<ORDER>(xo1[p], x1[p], m.idx1, m.L1);
  const ShapeK<K> sy = shape_o<ORDER>(xo2[p], x2[p], m.idx2, m.L2);
  const size_t pl = (size_t)m.n1 * m.n2;
  const double c1 = -qw * m.dx1 / dt, c2 = -qw * m.dx2 / dt;
  if (NDIM == 3) {
    const ShapeK<K> sz = shape_o<ORDER>(xo3[p], x3[p], m.idx3, m.L3);
    const double c3 = -qw * m.dx3 / dt;
    int ia[K], jb[K], kc[K];
    for (int q = 0; q < K; ++q) {
      ia[q] = wrapn(sx.base + q, m.n1);
      jb[q] = wrapn(sy.base + q, m.n2);
      kc[q] = wrapn(sz.base + q, m.n3);
    }
    T* Jg[3] = {J1, J2, J3};
    esirkepov<K>(sx, sy, sz, c1, c2, c3, [&](int comp, int a, int b, int c, double v) {
      atomic_add(&Jg[comp][(size_t)kc[c] * pl + (size_t)jb[b] * m.n1 + ia[a]], v);
    });
  } else {
    int ia[K], jb[K];
    for (int q = 0; q < K; ++q) {
      ia[q] = wrapn(sx.base + q, m.n1);
      jb[q] = wrapn(sy.base + q, m.n2);
    }
    if (m.n3 > 1) {  // the particle's plane of a stack of 2D meshes
      const size_t o = plane_offset(m, x3[p]);
      J1 += o;
      J2 += o;
      J3 += o;
    }
    const double g = sqrt(1.0 + u1[p] * u1[p] + u2[p] * u2[p] + u3[p] * u3[p]);
    const double c3 = qw * u3[p] / g;
    for (int b = 0; b < K; ++b) {
      const double w = sy.s0[b] + 0.5 * sy.ds[b];
      double run = 0;
      for (int a = 0; a < K - 1; ++a) {
        run += sx.ds[a] * w;
        if (run != 0.0) atomic_add(&J1[(size_t)jb[b] * m.n1 + ia[a]], c1 * run);
      }
    }
    for (int a = 0; a < K; ++a) {
      const double w = sx.s0[a] + 0.5 * sx.ds[a];
      double run = 0;
      for (int b = 0; b < K - 1; ++b) {
        run += sy.ds[b] * w;
        if (run != 0.0) atomic_add(&J2[(size_t)jb[b] * m.n1 + ia[a]], c2 * run);
      }
    }
    if (c3 != 0.0)
      for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
          const double w = sx.s0[a] * sy.s0[b] + 0.5 * sx.ds[a] * sy.s0[b] + 0.5 * sx.s0[a] * sy.ds[b] +
                           sx.ds[a] * sy.ds[b] * (1.0 / 3.0);
          if (w != 0.0) atomic_add(&J3[(size_t)jb[b] * m.n1 + ia[a]], c3 * w);
        }
  }
}

// non-finite fields or out-of-box positions -> *flag = 1
template <typename T>
__global__ __launch_bounds__(256) void check_fields_kernel(const T* __restrict__ f, size_t n, int* flag) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite((double)f[i])) atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void check_particles_kernel(const double* __restrict__ x, const double* __restrict__ u,
                                                              int64_t np, double L, int* flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const double xi = x ? x[i] : 0.0;
    if (!(xi >= 0.0 && xi < L) || !isfinite(u[i])) atomicOr(flag, 2);
  }
}

template <typename T>
int run_gather_push(const Mesh& m, void* const E[3], void* const B[3], const pic_particles& p, int pusher,
                    double dt, double* const xo[3], hipStream_t s) {
  if (p.np == 0) return PIC_OK;
  const int bs = 256;
  const dim3 grid((unsigned)((p.np + bs - 1) / bs));
  const double qm = p.q / p.m;
  double* o1 = xo ? xo[0] : nullptr;
  double* o2 = xo ? xo[1] : nullptr;
  double* o3 = xo ? xo[2] : nullptr;
#define YP_GP1(PUSH, ND, ORD)                                                                                  \
  hipLaunchKernelGGL((gather_push_kernel<T, PUSH, ND, ORD>), grid, dim3(bs), 0, s, (const T*)E[0],            \
                     (const T*)E[1], (const T*)E[2], (const T*)B[0], (const T*)B[1], (const T*)B[2], m, p.x[0], \
                     p.x[1], p.x[2], p.u[0], p.u[1], p.u[2], p.np, qm, dt, o1, o2, o3)
#define YP_GP(PUSH, ND)            \
  do {                             \
    if (m.order == 2)              \
      YP_GP1(PUSH, ND, 2);         \
    else                           \
      YP_GP1(PUSH, ND, 1);         \
  } while (0)
  if (m.ndim == 3) {
    if (pusher == PIC_PUSH_BORIS) YP_GP(PIC_PUSH_BORIS, 3);
    else if (pusher == PIC_PUSH_HC) YP_GP(PIC_PUSH_HC, 3);
    else YP_GP(PIC_PUSH_ANALYTIC, 3);
  } else {
    if (pusher == PIC_PUSH_BORIS) YP_GP(PIC_PUSH_BORIS, 2);
    else if (pusher == PIC_PUSH_HC) YP_GP(PIC_PUSH_HC, 2);
    else YP_GP(PIC_PUSH_ANALYTIC, 2);
  }
#undef YP_GP
#undef YP_GP1
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "gather_push launch failed");
}

template <typename T>
int run_deposit(const Mesh& m, void* const J[3], const pic_particles& p, double* const xo[3], double dt,
                hipStream_t s) {
  if (p.np == 0) return PIC_OK;
  const int bs = 256;
  const dim3 grid((unsigned)((p.np + bs - 1) / bs));
  const double qw = p.q * p.w;
#define YP_DEP(ND, ORD, X3, XO3)                                                                                 \
  hipLaunchKernelGGL((deposit_kernel<T, ND, ORD>), grid, dim3(bs), 0, s, (T*)J[0], (T*)J[1], (T*)J[2], m, p.x[0], \
                     p.x[1], X3, xo[0], xo[1], XO3, p.u[0], p.u[1], p.u[2], p.np, qw, dt)
  if (m.ndim == 3) {
    if (m.order == 2) YP_DEP(3, 2, p.x[2], xo[2]);
    else YP_DEP(3, 1, p.x[2], xo[2]);
  } else {
    if (m.order == 2) YP_DEP(2, 2, p.x[2], nullptr);
    else YP_DEP(2, 1, p.x[2], nullptr);
  }
#undef YP_DEP
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "deposit launch failed");
}

}  // namespace

int launch_gather_push(int prec, const Mesh& m, void* const E[3], void* const B[3], const pic_particles& p,
                       int pusher, double dt, double* const x_old[3], void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return prec == PIC_FP64 ? run_gather_push<double>(m, E, B, p, pusher, dt, x_old, s)
                          : run_gather_push<float>(m, E, B, p, pusher, dt, x_old, s);
}

int launch_deposit(int prec, const Mesh& m, void* const J[3], const pic_particles& p, double* const x_old[3],
                   double dt, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return prec == PIC_FP64 ? run_deposit<double>(m, J, p, x_old, dt, s) : run_deposit<float>(m, J, p, x_old, dt, s);
}

int launch_check(int prec, const Mesh& m, void* const E[3], void* const B[3], const pic_particles* p, int* d_flag,
                 void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)m.n1 * m.n2 * m.n3;
  const dim3 grid(1024), block(256);
  for (int c = 0; c < 3; ++c) {
    if (prec == PIC_FP64) {
      hipLaunchKernelGGL(check_fields_kernel<double>, grid, block, 0, s, (const double*)E[c], n, d_flag);
      hipLaunchKernelGGL(check_fields_kernel<double>, grid, block, 0, s, (const double*)B[c], n, d_flag);
    } else {
      hipLaunchKernelGGL(check_fields_kernel<float>, grid, block, 0, s, (const float*)E[c], n, d_flag);
      hipLaunchKernelGGL(check_fields_kernel<float>, grid, block, 0, s, (const float*)B[c], n, d_flag);
    }
  }
  if (p && p->np > 0) {
    const double L[3] = {m.L1, m.L2, m.L3};
    for (int d = 0; d < 3; ++d) {
      const double* x = (d < m.ndim || (d == 2 && m.n3 > 1)) ? p->x[d] : nullptr;
      hipLaunchKernelGGL(check_particles_kernel, grid, block, 0, s, x, p->u[d], p->np, L[d], d_flag);
    }
  }
  return hipGetLastError() == hipSuccess ? PIC_OK : set_error(PIC_EHIP, "check launch failed");
}

}  // namespace yeepic
