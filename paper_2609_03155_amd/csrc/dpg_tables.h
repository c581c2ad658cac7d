// Reference-cell tables of one (p, dp) pair: quadrature, test/trial/trace
// basis values and the geometry-independent reference matrices.
#pragma once
#include <cstdint>
#include <vector>

namespace dpg {

// Sizes of the local spaces and of the padded device layout for one (p, dp).
struct Dims {
  int p, dp;
  int s, r, n1, nq, nfq;  // test FEEC index, trace FEEC index, Gauss pts/dir, volume and face points
  int N, Np;              // test functions per field, padded to a multiple of 32
  int m1, nu, nt1, nt;    // DG functions per component, interior unknowns, trace fns per field, trace unknowns
  int k, kaug, kp;        // unknowns per cell, +2 (load, residual), padded to 64
  int nvp, nrows;         // padded test rows (2 Np), rows of the augmented workspace (nvp + kp)
};

Dims make_dims(int p, int dp);

// Host tables; the device copies live in DeviceTables (dpg_api).
struct RefTables {
  Dims d;
  std::vector<double> vol_pts, vol_w;     // [nq][3], [nq]   (x fastest)
  std::vector<double> vol_v;              // [nq][Np]  nonzero component of psi_hat_i
  std::vector<double> vol_c;              // [nq][Np][3] curl of psi_hat_i
  std::vector<int8_t> comp;               // [Np] component of psi_hat_i (pad: 0)
  std::vector<double> vol_phi;            // [nq][m1] DG Lagrange functions
  std::vector<double> face_pts, face_w;   // [6][nfq][3], [6][nfq]
  std::vector<double> face_v;             // [6][nfq][Np]
  std::vector<double> sf_tab;             // [2][s+1][n1]: orthonormal shifted Legendre q_k and q_k' at the Gauss points
  std::vector<double> sf_side;            // [2][s+1]: q_k(0), q_k(1) (the normal factor on the faces)
  std::vector<double> sf_phi;             // [p+1][n1]: 1D Lagrange factors of the DG basis at the Gauss points
  std::vector<double> sf_phis;            // [2][p+1]: the same at 0 and 1
  std::vector<double> face_phi;           // [6][nfq][m1]
  std::vector<double> Cref;               // [N][N]  int curl psi_hat_i . psi_hat_j
  std::vector<double> Rt;                 // [6][N][N] int_f (n_hat x psi_hat_i) . psi_hat_j
  std::vector<double> T;                  // [6][N][nt1] int_f psi_hat_i . (n_hat x theta_hat_j)
};

RefTables build_tables(int p, int dp);

}  // namespace dpg
