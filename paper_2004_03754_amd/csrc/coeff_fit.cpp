// Customized x1 stencil coefficients (App. B of the paper), host only.
//
// The least-squares fit of the k-space targets of Eq. (new_op) is extremely
// ill-conditioned (the normal-equation matrix A of App. B has condition number
// ~1e19 at M = 16), so this solves the same constrained minimisation without
// forming A: the weighted integral is discretised by composite Gauss-Legendre
// quadrature, the constraint M C = e1 is eliminated with a QR factorisation
// of M^T (null-space method), and the remaining unconstrained least-squares
// problem is solved by Householder QR.  All arithmetic is binary128
// (__float128 with libquadmath), which leaves the coefficients accurate to
// ~1e-24 -- far below double rounding.
#include <quadmath.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "yeepic_internal.h"

namespace {

using q128 = __float128;

const q128 kPi = M_PIq;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton on the Legendre
// three-term recurrence.
void gauss_legendre(int G, std::vector<q128>& x, std::vector<q128>& w) {
  x.assign(G, 0);
  w.assign(G, 0);
  for (int i = 0; i < G; ++i) {
    q128 z = cosq(kPi * (i + 0.75Q) / (G + 0.5Q));
    q128 dp = 1;
    for (int it = 0; it < 100; ++it) {
      q128 p0 = 1, p1 = z;
      for (int k = 2; k <= G; ++k) {
        q128 p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = G * (z * p1 - p0) / (z * z - 1);
      q128 dz = p1 / dp;
      z -= dz;
      if (fabsq(dz) < 1e-40Q) break;
    }
    q128 p0 = 1, p1 = z;
    for (int k = 2; k <= G; ++k) {
      q128 p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = G * (z * p1 - p0) / (z * z - 1);
    x[i] = z;
    w[i] = 2 / ((1 - z * z) * dp * dp);
  }
}

q128 target_value(int kind, q128 kappa, q128 r) {
  switch (kind) {
    case PIC_TARGET_E: return tanq(kPi * kappa * r) / (kPi * r);
    case PIC_TARGET_B: return sinq(2 * kPi * kappa * r) / (2 * kPi * r);
    // Yee t-stagger (Sec. 4): Eq. (new_op) with the Yee symbol in place of [k]_{1,t}
    case PIC_TARGET_YEET_E: return sinq(kPi * kappa) / (kPi * cosq(kPi * kappa * r));
    case PIC_TARGET_YEET_B: return sinq(kPi * kappa) * cosq(kPi * kappa * r) / kPi;
    default: return sinq(kPi * kappa * r) / (kPi * r);
  }
}

}  // namespace

// Dense Householder least squares with explicit R (small sizes; clarity over
// speed).  Solves min ||A z - b|| for column-major A (m x n), m >= n.
static int lsq_solve(std::vector<q128> A, int m, int n, std::vector<q128> b,
                     std::vector<q128>& z) {
  std::vector<q128> R((size_t)n * n, 0);
  for (int k = 0; k < n; ++k) {
    q128* col = &A[(size_t)k * m];
    q128 norm = 0;
    for (int i = k; i < m; ++i) norm += col[i] * col[i];
    norm = sqrtq(norm);
    if (norm == 0) return -1;
    q128 alpha = col[k] > 0 ? -norm : norm;
    col[k] -= alpha;
    q128 vv = 0;
    for (int i = k; i < m; ++i) vv += col[i] * col[i];
    q128 beta = vv > 0 ? 2 / vv : 0;
    for (int j = k + 1; j < n; ++j) {
      q128* cj = &A[(size_t)j * m];
      q128 s = 0;
      for (int i = k; i < m; ++i) s += col[i] * cj[i];
      s *= beta;
      for (int i = k; i < m; ++i) cj[i] -= s * col[i];
    }
    q128 s = 0;
    for (int i = k; i < m; ++i) s += col[i] * b[i];
    s *= beta;
    for (int i = k; i < m; ++i) b[i] -= s * col[i];
    R[(size_t)k * n + k] = alpha;
    for (int j = k + 1; j < n; ++j) R[(size_t)k * n + j] = A[(size_t)j * m + k];
  }
  z.assign(n, 0);
  for (int k = n - 1; k >= 0; --k) {
    q128 s = b[k];
    for (int j = k + 1; j < n; ++j) s -= R[(size_t)k * n + j] * z[j];
    z[k] = s / R[(size_t)k * n + k];
  }
  return 0;
}

extern "C" int pic_design_coeffs(int M, double r_d, int target, int p, int n, double wk1_d,
                                 double width_factor_d, double* out) {
  using namespace yeepic;
  if (!out) return set_error(PIC_EINVAL, "pic_design_coeffs: out is NULL");
  if (M < 1 || M > PIC_MAX_M) return set_error(PIC_EINVAL, "pic_design_coeffs: M outside 1..16");
  if (p < 2 || (p & 1) || p / 2 > M) return set_error(PIC_EINVAL, "pic_design_coeffs: bad order p");
  if (!(r_d > 0 && r_d < 1)) return set_error(PIC_EINVAL, "pic_design_coeffs: r = dt/dx1 must be in (0, 1)");
  if (n < 1 || !(wk1_d > 0) || !(width_factor_d > 0))
    return set_error(PIC_EINVAL, "pic_design_coeffs: bad weight parameters");
  if (target < PIC_TARGET_E || target > PIC_TARGET_YEET_B)
    return set_error(PIC_EINVAL, "pic_design_coeffs: bad target");

  const int nc = p / 2;             // constraint rows
  const int panels = 48, G = 40;    // composite Gauss-Legendre on [0, 1/2]
  const int N = panels * G;
  const q128 r = r_d, wk1 = wk1_d, wf = width_factor_d;
  std::vector<q128> gx, gw;
  gauss_legendre(G, gx, gw);

  // sqrt(weight)-scaled design matrix Phi (N x M, column-major) and target
  std::vector<q128> Phi((size_t)N * M), T(N);
  const q128 h = 0.5Q / panels, ln2 = logq(2.0Q);
  for (int pn = 0; pn < panels; ++pn) {
    for (int g = 0; g < G; ++g) {
      const int row = pn * G + g;
      const q128 kap = pn * h + (gx[g] + 1) * h / 2;
      const q128 wq = gw[g] * h / 2 * expq(-ln2 * powq(wf * kap / wk1, n));
      const q128 sw = sqrtq(wq);
      for (int j = 0; j < M; ++j) Phi[(size_t)j * N + row] = sw * sinq((2 * j + 1) * kPi * kap) / kPi;
      T[row] = sw * target_value(target, kap, r);
    }
  }

  // constraint matrix Mc (nc x M): (2j-1)^(2i-1)/(2i-1)!
  std::vector<q128> Mc((size_t)nc * M);
  for (int i = 0; i < nc; ++i) {
    q128 fact = 1;
    for (int f = 2; f <= 2 * i + 1; ++f) fact *= f;
    for (int j = 0; j < M; ++j) Mc[(size_t)i * M + j] = powq((q128)(2 * j + 1), 2 * i + 1) / fact;
  }

  // QR of Mc^T (M x nc) with explicit Q (M x M) to split range / null space
  std::vector<q128> Q((size_t)M * M, 0), At((size_t)M * nc);
  for (int i = 0; i < M; ++i) Q[(size_t)i * M + i] = 1;
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < M; ++j) At[(size_t)i * M + j] = Mc[(size_t)i * M + j];  // column i = row i of Mc
  std::vector<q128> Rm((size_t)nc * nc, 0);
  for (int k = 0; k < nc; ++k) {
    q128* col = &At[(size_t)k * M];
    q128 norm = 0;
    for (int i = k; i < M; ++i) norm += col[i] * col[i];
    norm = sqrtq(norm);
    q128 alpha = col[k] > 0 ? -norm : norm;
    std::vector<q128> v(M, 0);
    for (int i = k; i < M; ++i) v[i] = col[i];
    v[k] -= alpha;
    q128 vv = 0;
    for (int i = k; i < M; ++i) vv += v[i] * v[i];
    q128 beta = vv > 0 ? 2 / vv : 0;
    for (int j = k; j < nc; ++j) {  // apply to remaining columns of At
      q128* cj = &At[(size_t)j * M];
      q128 s = 0;
      for (int i = k; i < M; ++i) s += v[i] * cj[i];
      s *= beta;
      for (int i = k; i < M; ++i) cj[i] -= s * v[i];
    }
    // accumulate Q = H_0 H_1 ... explicitly (row-major Q[row*M + col])
    for (int row = 0; row < M; ++row) {
      q128 s = 0;
      for (int i = k; i < M; ++i) s += Q[(size_t)row * M + i] * v[i];
      s *= beta;
      for (int i = k; i < M; ++i) Q[(size_t)row * M + i] -= s * v[i];
    }
    for (int j = k; j < nc; ++j) Rm[(size_t)k * nc + j] = At[(size_t)j * M + k];
  }
  // particular solution C_p = Q1 R^{-T} e1
  std::vector<q128> y(nc, 0);
  for (int i = 0; i < nc; ++i) {
    q128 s = (i == 0) ? 1 : 0;
    for (int k = 0; k < i; ++k) s -= Rm[(size_t)k * nc + i] * y[k];
    y[i] = s / Rm[(size_t)i * nc + i];
  }
  std::vector<q128> C(M, 0);
  for (int row = 0; row < M; ++row)
    for (int i = 0; i < nc; ++i) C[row] += Q[(size_t)row * M + i] * y[i];

  const int nf = M - nc;  // free directions
  if (nf > 0) {
    // reduced problem: (Phi Q2) z ~ T - Phi C_p
    std::vector<q128> A2((size_t)N * nf, 0), b2(N);
    for (int row = 0; row < N; ++row) {
      q128 s = T[row];
      for (int j = 0; j < M; ++j) s -= Phi[(size_t)j * N + row] * C[j];
      b2[row] = s;
    }
    for (int c = 0; c < nf; ++c)
      for (int j = 0; j < M; ++j) {
        const q128 qj = Q[(size_t)j * M + nc + c];
        if (qj == 0) continue;
        for (int row = 0; row < N; ++row) A2[(size_t)c * N + row] += Phi[(size_t)j * N + row] * qj;
      }
    std::vector<q128> z;
    if (lsq_solve(A2, N, nf, b2, z) != 0)
      return set_error(PIC_EINVAL, "pic_design_coeffs: singular least-squares system");
    for (int j = 0; j < M; ++j)
      for (int c = 0; c < nf; ++c) C[j] += Q[(size_t)j * M + nc + c] * z[c];
  }
  for (int j = 0; j < M; ++j) out[j] = (double)C[j];
  return PIC_OK;
}
