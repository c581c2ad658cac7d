// Reference-cell tables for the DPG local solve: Gauss-Legendre quadrature,
// the first-kind Nedelec test basis (orthonormal shifted-Legendre tensor
// products), the DG Lagrange trial basis at Gauss-Lobatto nodes, the
// hierarchical Nedelec trace basis, and the matrices that the covariant
// Piola map leaves geometry-independent:
//   C_ij  = int_K curl psi_i . psi_j         = int_[0,1]^3 curl psi_hat_i . psi_hat_j
//   Rt_ij = int_f (n x psi_i) . psi_j dS     = int_f_hat (n_hat x psi_hat_i) . psi_hat_j
//   T_ij  = int_f psi_i . (n x theta_j) dS  = int_f_hat psi_hat_i . (n_hat x theta_hat_j)
// (psi = J^{-T} psi_hat, curl psi = J curl psi_hat / det J and
// n dS = det J J^{-T} n_hat dS_hat, so the metric cancels pointwise).
#include "dpg_tables.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace dpg {

namespace {

// Legendre P_0..P_n at t and their derivatives (Bonnet recurrence).
void legendre(int n, double t, std::vector<double>& P, std::vector<double>& dP) {
  P.assign(n + 1, 0.0);
  dP.assign(n + 1, 0.0);
  P[0] = 1.0;
  if (n >= 1) { P[1] = t; dP[1] = 1.0; }
  for (int k = 1; k < n; ++k) {
    P[k + 1] = ((2 * k + 1) * t * P[k] - k * P[k - 1]) / (k + 1);
    dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
  }
}

// n-point Gauss-Legendre rule mapped to [0,1], ascending nodes.
void gauss01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  std::vector<double> P, dP;
  for (int i = 0; i < n; ++i) {
    // i-th root from the largest; Tricomi-style start, then Newton
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, P, dP);
      double dt = P[n] / dP[n];
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    legendre(n, t, P, dP);
    double wt = 2.0 / ((1.0 - t * t) * dP[n] * dP[n]);
    x[n - 1 - i] = 0.5 * (t + 1.0);
    w[n - 1 - i] = 0.5 * wt;
  }
}

// n >= 2 Gauss-Lobatto nodes on [0,1].
std::vector<double> lobatto01(int n) {
  std::vector<double> z(n);
  z[0] = 0.0;
  z[n - 1] = 1.0;
  int m = n - 1;
  std::vector<double> P, dP;
  for (int i = 1; i < n - 1; ++i) {
    double t = -std::cos(M_PI * i / m);
    for (int it = 0; it < 100; ++it) {
      legendre(m, t, P, dP);
      double d2 = (2.0 * t * dP[m] - m * (m + 1.0) * P[m]) / (1.0 - t * t);
      double dt = dP[m] / d2;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    z[i] = 0.5 * (t + 1.0);
  }
  return z;
}

// Orthonormal shifted Legendre q_k(x) = sqrt(2k+1) P_k(2x-1), k = 0..n, and d/dx.
void onb(int n, double x, std::vector<double>& v, std::vector<double>& dv) {
  std::vector<double> P, dP;
  legendre(n, 2.0 * x - 1.0, P, dP);
  v.resize(n + 1);
  dv.resize(n + 1);
  for (int k = 0; k <= n; ++k) {
    double c = std::sqrt(2.0 * k + 1.0);
    v[k] = c * P[k];
    dv[k] = 2.0 * c * dP[k];
  }
}

// Transverse factor of a trace function: kind 0 -> 1-x, 1 -> x, m >= 2 -> bubble b_m.
double transverse(int kind, double x) {
  if (kind == 0) return 1.0 - x;
  if (kind == 1) return x;
  std::vector<double> P, dP;
  legendre(kind, 2.0 * x - 1.0, P, dP);
  return (P[kind] - P[kind - 2]) / std::sqrt(2.0 * (2 * kind - 1));
}

struct TestFn { int comp; int deg[3]; };
struct TraceFn { int comp; int i; int ax_b, kind_b, ax_c, kind_c; };

std::vector<TestFn> test_functions(int s) {
  std::vector<TestFn> out;
  for (int a = 0; a < 3; ++a) {
    int hi[3] = {s, s, s};
    hi[a] = s - 1;
    for (int d2 = 0; d2 <= hi[2]; ++d2)
      for (int d1 = 0; d1 <= hi[1]; ++d1)
        for (int d0 = 0; d0 <= hi[0]; ++d0) out.push_back({a, {d0, d1, d2}});
  }
  return out;
}

std::vector<TraceFn> trace_functions(int r) {
  std::vector<TraceFn> out;
  for (int a = 0; a < 3; ++a) {                 // 12 edges: 4 per direction
    int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
    for (int vc = 0; vc < 2; ++vc)
      for (int vb = 0; vb < 2; ++vb)
        for (int i = 0; i < r; ++i) out.push_back({a, i, b, vb, c, vc});
  }
  for (int f = 0; f < 6; ++f) {                 // face functions
    int nax = f / 2, side = f % 2;
    int t1 = (nax == 0) ? 1 : 0, t2 = (nax == 2) ? 1 : 2;
    for (int g = 0; g < 2; ++g) {
      int comp = g == 0 ? t1 : t2, other = g == 0 ? t2 : t1;
      for (int m = 2; m <= r; ++m)
        for (int i = 0; i < r; ++i) out.push_back({comp, i, nax, side, other, m});
    }
  }
  return out;
}

// Test function value (nonzero component) and curl at reference point xi.
void eval_test(const TestFn& t, int s, const double* xi, double& val, double curl[3]) {
  std::vector<double> v[3], dv[3];
  for (int ax = 0; ax < 3; ++ax) onb(s, xi[ax], v[ax], dv[ax]);
  const int* d = t.deg;
  val = v[0][d[0]] * v[1][d[1]] * v[2][d[2]];
  double g[3] = {dv[0][d[0]] * v[1][d[1]] * v[2][d[2]], v[0][d[0]] * dv[1][d[1]] * v[2][d[2]],
                 v[0][d[0]] * v[1][d[1]] * dv[2][d[2]]};
  // curl(f e_a) = grad f x e_a
  double e[3] = {0, 0, 0};
  e[t.comp] = 1.0;
  curl[0] = g[1] * e[2] - g[2] * e[1];
  curl[1] = g[2] * e[0] - g[0] * e[2];
  curl[2] = g[0] * e[1] - g[1] * e[0];
}

void eval_trace(const TraceFn& t, int r, const double* xi, double out[3]) {
  std::vector<double> v, dv;
  onb(r - 1, xi[t.comp], v, dv);
  out[0] = out[1] = out[2] = 0.0;
  out[t.comp] = v[t.i] * transverse(t.kind_b, xi[t.ax_b]) * transverse(t.kind_c, xi[t.ax_c]);
}

double lagrange(const std::vector<double>& z, int i, double x) {
  double v = 1.0;
  for (size_t j = 0; j < z.size(); ++j)
    if ((int)j != i) v *= (x - z[j]) / (z[i] - z[j]);
  return v;
}

inline void cross(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

}  // namespace

Dims make_dims(int p, int dp) {
  if (p < 1 || p > 4 || dp < 1 || dp > 2) throw std::invalid_argument("unsupported (p, dp)");
  Dims d;
  d.p = p;
  d.dp = dp;
  d.s = p + dp + 1;
  d.r = p + 1;
  d.n1 = p + dp + 2;
  d.nq = d.n1 * d.n1 * d.n1;
  d.nfq = d.n1 * d.n1;
  d.N = 3 * d.s * (d.s + 1) * (d.s + 1);
  d.Np = (d.N + 31) / 32 * 32;
  d.m1 = (p + 1) * (p + 1) * (p + 1);
  d.nu = 6 * d.m1;
  d.nt1 = 12 * d.r * d.r;
  d.nt = 2 * d.nt1;
  d.k = d.nu + d.nt;
  d.kaug = d.k + 2;
  d.kp = (d.kaug + 63) / 64 * 64;
  d.nvp = 2 * d.Np;
  d.nrows = d.nvp + d.kp;
  return d;
}

RefTables build_tables(int p, int dp) {
  RefTables T;
  T.d = make_dims(p, dp);
  const Dims& d = T.d;
  std::vector<double> gx, gw;
  gauss01(d.n1, gx, gw);
  auto tf = test_functions(d.s);
  auto trf = trace_functions(d.r);
  auto zl = lobatto01(p + 1);

  // volume points, x fastest
  T.vol_pts.resize(d.nq * 3);
  T.vol_w.resize(d.nq);
  for (int k = 0; k < d.n1; ++k)
    for (int j = 0; j < d.n1; ++j)
      for (int i = 0; i < d.n1; ++i) {
        int q = i + d.n1 * (j + d.n1 * k);
        T.vol_pts[3 * q + 0] = gx[i];
        T.vol_pts[3 * q + 1] = gx[j];
        T.vol_pts[3 * q + 2] = gx[k];
        T.vol_w[q] = gw[i] * gw[j] * gw[k];
      }
  T.comp.assign(d.Np, 0);
  for (int i = 0; i < d.N; ++i) T.comp[i] = (int8_t)tf[i].comp;
  T.vol_v.assign((size_t)d.nq * d.Np, 0.0);
  T.vol_c.assign((size_t)d.nq * d.Np * 3, 0.0);
  for (int q = 0; q < d.nq; ++q)
    for (int i = 0; i < d.N; ++i) {
      double v, c[3];
      eval_test(tf[i], d.s, &T.vol_pts[3 * q], v, c);
      T.vol_v[(size_t)q * d.Np + i] = v;
      for (int u = 0; u < 3; ++u) T.vol_c[((size_t)q * d.Np + i) * 3 + u] = c[u];
    }
  // 1D factors of the test basis for the sum-factorised formation
  T.sf_tab.assign((size_t)2 * (d.s + 1) * d.n1, 0.0);
  T.sf_side.assign((size_t)2 * (d.s + 1), 0.0);
  for (int q = 0; q < d.n1; ++q) {
    std::vector<double> v, dv;
    onb(d.s, gx[q], v, dv);
    for (int k = 0; k <= d.s; ++k) {
      T.sf_tab[(size_t)k * d.n1 + q] = v[k];
      T.sf_tab[(size_t)(d.s + 1 + k) * d.n1 + q] = dv[k];
    }
  }
  for (int side = 0; side < 2; ++side) {
    std::vector<double> v, dv;
    onb(d.s, (double)side, v, dv);
    for (int k = 0; k <= d.s; ++k) T.sf_side[(size_t)side * (d.s + 1) + k] = v[k];
  }
  T.sf_phi.assign((size_t)(p + 1) * d.n1, 0.0);
  T.sf_phis.assign((size_t)2 * (p + 1), 0.0);
  for (int k = 0; k <= p; ++k) {
    for (int q = 0; q < d.n1; ++q) T.sf_phi[(size_t)k * d.n1 + q] = lagrange(zl, k, gx[q]);
    for (int side = 0; side < 2; ++side) T.sf_phis[(size_t)side * (p + 1) + k] = lagrange(zl, k, (double)side);
  }
  auto phi_at = [&](const double* xi, double* out) {
    int n = p + 1;
    for (int kk = 0; kk < n; ++kk)
      for (int jj = 0; jj < n; ++jj)
        for (int ii = 0; ii < n; ++ii)
          out[ii + n * (jj + n * kk)] = lagrange(zl, ii, xi[0]) * lagrange(zl, jj, xi[1]) * lagrange(zl, kk, xi[2]);
  };
  T.vol_phi.resize((size_t)d.nq * d.m1);
  for (int q = 0; q < d.nq; ++q) phi_at(&T.vol_pts[3 * q], &T.vol_phi[(size_t)q * d.m1]);

  // face points: tangential axes t1 < t2, t1 fastest
  T.face_pts.resize(6 * d.nfq * 3);
  T.face_w.resize(6 * d.nfq);
  T.face_v.assign((size_t)6 * d.nfq * d.Np, 0.0);
  T.face_phi.resize((size_t)6 * d.nfq * d.m1);
  for (int f = 0; f < 6; ++f) {
    int nax = f / 2, side = f % 2;
    int t1 = (nax == 0) ? 1 : 0, t2 = (nax == 2) ? 1 : 2;
    for (int b = 0; b < d.n1; ++b)
      for (int a = 0; a < d.n1; ++a) {
        int fq = a + d.n1 * b;
        double* X = &T.face_pts[(f * d.nfq + fq) * 3];
        X[t1] = gx[a];
        X[t2] = gx[b];
        X[nax] = (double)side;
        T.face_w[f * d.nfq + fq] = gw[a] * gw[b];
        for (int i = 0; i < d.N; ++i) {
          double v, c[3];
          eval_test(tf[i], d.s, X, v, c);
          T.face_v[((size_t)f * d.nfq + fq) * d.Np + i] = v;
        }
        phi_at(X, &T.face_phi[((size_t)f * d.nfq + fq) * d.m1]);
      }
  }

  // geometry-free reference matrices; the quadrature sums run in long double
  // (a 64-bit significand), so that each entry is the correctly rounded FP64
  // value of the rule's sum of the FP64 basis values (up to thousands of
  // terms at p = 4, where FP64 accumulation would carry several ulps).  Rows
  // are independent: host threads take interleaved rows.
  std::vector<double> fpsi((size_t)6 * d.nfq * d.N * 3, 0.0), fnpsi(fpsi.size()), fnth((size_t)6 * d.nfq * d.nt1 * 3);
  for (int f = 0; f < 6; ++f) {
    double nh[3] = {0, 0, 0};
    nh[f / 2] = (f % 2) ? 1.0 : -1.0;
    for (int fq = 0; fq < d.nfq; ++fq) {
      const size_t o = (size_t)f * d.nfq + fq;
      const double* X = &T.face_pts[o * 3];
      for (int i = 0; i < d.N; ++i) {
        double* ps = &fpsi[(o * d.N + i) * 3];
        ps[tf[i].comp] = T.face_v[o * d.Np + i];
        cross(nh, ps, &fnpsi[(o * d.N + i) * 3]);
      }
      for (int j = 0; j < d.nt1; ++j) {
        double th[3];
        eval_trace(trf[j], d.r, X, th);
        cross(nh, th, &fnth[(o * d.nt1 + j) * 3]);
      }
    }
  }
  T.Cref.assign((size_t)d.N * d.N, 0.0);
  T.Rt.assign((size_t)6 * d.N * d.N, 0.0);
  T.T.assign((size_t)6 * d.N * d.nt1, 0.0);
  auto rows = [&](int i0, int step) {
    std::vector<long double> acc((size_t)std::max(d.N, d.nt1));
    for (int i = i0; i < d.N; i += step) {
      std::fill(acc.begin(), acc.end(), 0.0L);
      for (int q = 0; q < d.nq; ++q) {
        const long double wc = (long double)T.vol_w[q];
        const double* ci = &T.vol_c[((size_t)q * d.Np + i) * 3];
        const double* vq = &T.vol_v[(size_t)q * d.Np];
        for (int j = 0; j < d.N; ++j) acc[j] += wc * (long double)ci[tf[j].comp] * (long double)vq[j];
      }
      for (int j = 0; j < d.N; ++j) T.Cref[(size_t)i * d.N + j] = (double)acc[j];
      for (int f = 0; f < 6; ++f) {
        std::fill(acc.begin(), acc.end(), 0.0L);
        for (int fq = 0; fq < d.nfq; ++fq) {
          const size_t o = (size_t)f * d.nfq + fq;
          const long double w = (long double)T.face_w[o];
          const double* ni = &fnpsi[(o * d.N + i) * 3];
          for (int j = 0; j < d.N; ++j) {
            const double* pj = &fpsi[(o * d.N + j) * 3];
            acc[j] += w * ((long double)ni[0] * pj[0] + (long double)ni[1] * pj[1] + (long double)ni[2] * pj[2]);
          }
        }
        for (int j = 0; j < d.N; ++j) T.Rt[((size_t)f * d.N + i) * d.N + j] = (double)acc[j];
        std::fill(acc.begin(), acc.end(), 0.0L);
        for (int fq = 0; fq < d.nfq; ++fq) {
          const size_t o = (size_t)f * d.nfq + fq;
          const long double w = (long double)T.face_w[o];
          const double* pi = &fpsi[(o * d.N + i) * 3];
          for (int j = 0; j < d.nt1; ++j) {
            const double* nj = &fnth[(o * d.nt1 + j) * 3];
            acc[j] += w * ((long double)pi[0] * nj[0] + (long double)pi[1] * nj[1] + (long double)pi[2] * nj[2]);
          }
        }
        for (int j = 0; j < d.nt1; ++j) T.T[((size_t)f * d.N + i) * d.nt1 + j] = (double)acc[j];
      }
    }
  };
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back(rows, t, nth);
  rows(0, nth);
  for (auto& th : pool) th.join();
  return T;
}

}  // namespace dpg
