// HIP kernels (gfx950) of the DPG per-cell local solve.
//
// Per degree group and chunk of cells the pipeline is
//   k_cell_scale  geometry check and Jacobi scaling d_i = G_ii^{-1/2}
//   k_form_SM     G_FF, G_II from S, M (volume) and the Robin face mass, by
//                 sum factorisation over the tensor-product test basis
//   k_form_IF     G_IF from the geometry-free C and Rt (Sec. 2.2 test norm)
//   k_form_pad    identity/zero padding of the test space
//   k_form_B      rows of B_f^H, l^H and r^H = (B_f x - l)^H (Sec. 2.2 forms,
//                 entries of Sec. 2.3; r for the error representation)
//   k_chol_diag / k_chol_panel   left-looking blocked Cholesky of the
//                 augmented Hermitian matrix [[D G D, D B],[B^H D, 0]]: the
//                 lower rows of its factor are W^H = (L^{-1} D B_f)^H
//   k_herk        K_aug = W^H W -> K_e, l_e, eta (Sec. 2.3)
// Workspace of a cell: column-major complex matrix Z with nrows = nvp + kp
// rows and nvp columns; rows [0,nvp) hold the lower triangle of D G D (F
// test functions at [0,Np), I at [Np,2Np)), rows [nvp, nvp+kp) hold
// (D B_f)^H, (D l)^H, (D r)^H and zero padding.
#include "dpg_kernels.h"

#include <math.h>

namespace dpg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;   // threads per workgroup (4 wave64)
constexpr int TB = 64;    // tile of the blocked factorisation
constexpr int KC = 16;    // k-chunk staged through LDS
constexpr int LDP = 65;   // LDS row pitch (doubles) of staged panels: odd, so that
                          // column-wise (transposed) writes hit distinct banks

__device__ __forceinline__ int sym3(int a, int b) {
  // packed index of a symmetric 3x3: (0,0)(1,1)(2,2)(0,1)(0,2)(1,2)
  return a == b ? a : (a + b + 2);
}

// XCD-aware decode of a (cell, tile) grid: consecutive workgroup ids are
// dispatched round-robin over the 8 XCDs, so cell c is given to XCD c % 8 and
// all tiles of a cell run on the same XCD (its L2 holds the shared panels).
__device__ __forceinline__ bool decode_cell_tile(int64_t ncells, int ntiles, int64_t& cell, int& tile) {
  const int64_t w = blockIdx.x;
  const int x = (int)(w & 7);
  const int64_t slot = w >> 3;
  const int64_t cl = slot / ntiles;
  tile = (int)(slot - cl * ntiles);
  cell = cl * 8 + x;
  return cell < ncells;
}

__host__ inline unsigned grid_cells_tiles(int64_t ncells, int ntiles) {
  return (unsigned)(((ncells + 7) / 8) * 8 * ntiles);
}

// ---------------------------------------------------------------- geometry
struct Geo {
  double J[3][3];    // J[a][b] = d x_a / d xi_b
  double Ji[3][3];   // inverse
  double det;
  double x[3];
};

__device__ inline void trilinear(const double (*X)[3], double x0, double x1, double x2, Geo& g) {
  for (int a = 0; a < 3; ++a) {
    g.x[a] = 0.0;
    g.J[a][0] = g.J[a][1] = g.J[a][2] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int i = v & 1, j = (v >> 1) & 1, k = v >> 2;
    const double fx = i ? x0 : 1.0 - x0, fy = j ? x1 : 1.0 - x1, fz = k ? x2 : 1.0 - x2;
    const double dx = i ? 1.0 : -1.0, dy = j ? 1.0 : -1.0, dz = k ? 1.0 : -1.0;
    const double n = fx * fy * fz, n0 = dx * fy * fz, n1 = fx * dy * fz, n2 = fx * fy * dz;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      g.x[a] += n * X[v][a];
      g.J[a][0] += n0 * X[v][a];
      g.J[a][1] += n1 * X[v][a];
      g.J[a][2] += n2 * X[v][a];
    }
  }
  const double (*J)[3] = g.J;
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  g.det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const double id = 1.0 / g.det;
  g.Ji[0][0] = c00 * id;
  g.Ji[1][0] = c01 * id;
  g.Ji[2][0] = c02 * id;
  g.Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  g.Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  g.Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  g.Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  g.Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  g.Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
}

// Volume metrics at one point: Gc = w J^T J / det (curl-curl), Gm = w det J^{-1} J^{-T}
// (rows of J^{-1} are the covariant images of the reference unit vectors).
__device__ inline void vol_metrics(const Geo& g, double w, double* Gc, double* Gm) {
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      double c = 0.0, m = 0.0;
      for (int e = 0; e < 3; ++e) {
        c += g.J[e][a] * g.J[e][b];
        m += g.Ji[a][e] * g.Ji[b][e];
      }
      Gc[sym3(a, b)] = w * c / g.det;
      Gm[sym3(a, b)] = w * g.det * m;
    }
}

// Face quantities at one point of reference face f: outward unit normal n and
// area factor s (n dS = det J J^{-T} n_hat dS_hat).
__device__ inline void face_normal(const Geo& g, int f, double n[3], double& s) {
  const int ax = f >> 1;
  const double sg = (f & 1) ? 1.0 : -1.0;
  double v[3];
  // (row ax of J^{-1} by selects: a runtime index would put g in scratch memory)
  for (int a = 0; a < 3; ++a) v[a] = sg * g.det * (ax == 0 ? g.Ji[0][a] : (ax == 1 ? g.Ji[1][a] : g.Ji[2][a]));
  s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int a = 0; a < 3; ++a) n[a] = v[a] / s;
}

// Face mass metric Q_ab = w s (n x r_a).(n x r_b), r_a = row a of J^{-1}.
__device__ inline void face_metric(const Geo& g, const double n[3], double ws, double* Q) {
  double rn[3];
  for (int a = 0; a < 3; ++a) rn[a] = g.Ji[a][0] * n[0] + g.Ji[a][1] * n[1] + g.Ji[a][2] * n[2];
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      double d = g.Ji[a][0] * g.Ji[b][0] + g.Ji[a][1] * g.Ji[b][1] + g.Ji[a][2] * g.Ji[b][2];
      Q[sym3(a, b)] = ws * (d - rn[a] * rn[b]);
    }
}

__device__ inline bool is_robin(int8_t k) { return k == 2 || k == 3; }

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Structure of the augmented rows [r0, r0 + nr) in the F columns: the
// rows of the E-hat trace unknowns pair with no F test function (zero there,
// so are the padding rows), those of H-hat only through the real trace table
// (real); the interior, load and residual rows and the I test rows are complex.
enum { FROWS_COMPLEX = 0, FROWS_REAL = 1, FROWS_ZERO = 2 };
__device__ inline int frows_class(const DevTables& T, int r0, int nr = 32) {
  const int eh0 = T.nvp + T.nu, hh0 = eh0 + T.nt1, lr0 = T.nvp + T.k, pad0 = lr0 + 2;
  const int r1 = r0 + nr;
  if (r0 < eh0 || (r0 < pad0 && r1 > lr0)) return FROWS_COMPLEX;
  if (r0 < lr0 && r1 > hh0) return FROWS_REAL;
  return FROWS_ZERO;
}

// First column of the sum W_a^H W_b over the test columns: the F columns
// contribute nothing when either 64-row block of W^H is zero there.
__device__ inline int herk_k0(const DevTables& T, int a, int b) {
  auto zero_f = [&](int blk) {
    const int r0 = T.nvp + blk * TB;
    return frows_class(T, r0) == FROWS_ZERO && frows_class(T, r0 + 32) == FROWS_ZERO;
  };
  return zero_f(a) || zero_f(b) ? (T.Np / TB) * TB : 0;
}

// Trace-row entries of the workspace that the formation leaves unwritten
// because they are zero and no kernel reads them: the E-hat rows in the
// columns of the real F block (c < 64 nF) inside a 64-row block of W whose F
// columns are all zero.  Their F-column tiles are skipped, the sums of their
// step tiles and of the HERK start after the F block, and no other tile reads
// these rows.  None without an F block (the condensation and reconstruction
// matrices).
__device__ inline bool trace_unwritten(const DevTables& T, int r, int c) {
  const int eh0 = T.nvp + T.nu, hh0 = eh0 + T.nt1;
  if (T.Np <= 0 || r < eh0 || r >= hh0 || c >= (T.Np / TB) * TB) return false;
  const int b0 = T.nvp + (r - T.nvp) / TB * TB;
  return frows_class(T, b0) == FROWS_ZERO && frows_class(T, b0 + 32) == FROWS_ZERO;
}

// Three-term bf16 splits of a complex value: v ~ h0 + h1 + h2 for its real and
// imaginary parts, each term the remainder of the previous ones rounded to
// bf16 (through float, round to nearest even; about 24 significant bits in
// total).  p[t] holds the t-th terms, the real part's bits in the low half and
// the imaginary part's in the high half: one packed conversion makes both.
__device__ inline void split3_bf16_pair(double vr, double vi, uint32_t p[3]) {
  double rr = vr, ri = vi;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    // both halves in one packed conversion (rounding to nearest even); the
    // float values are rounded from the doubles first, as written
    const float fr = (float)rr, fi = (float)ri;
    __asm__("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(p[t]) : "v"(fr), "v"(fi));
    rr -= (double)__uint_as_float(p[t] << 16);
    ri -= (double)__uint_as_float(p[t] & 0xffff0000u);
  }
}

// TE_mn fields of Sec. 4.1 at non-dimensional point x.
__device__ inline void te_fields(const ProbArgs& P, double omega, const double x[3], double2 E[3], double2 H[3]) {
  const double c1 = cos(P.pk1 * x[0]), s1 = sin(P.pk1 * x[0]);
  const double c2 = cos(P.pk2 * x[1]), s2 = sin(P.pk2 * x[1]);
  // e^{i k3 x3} with complex k3
  const double amp = exp(-P.pk3im * x[2]);
  const double2 ph = make_double2(amp * cos(P.pk3re * x[2]), amp * sin(P.pk3re * x[2]));
  // pre = i omega mu / kc^2
  const double2 pre = make_double2(-omega * P.pmu_im / P.pkc2, omega * P.pmu_re / P.pkc2);
  const double2 ex = cmul(pre, make_double2(-P.pk2 * c1 * s2, 0.0));
  const double2 ey = cmul(pre, make_double2(P.pk1 * s1 * c2, 0.0));
  E[0] = cmul(ex, ph);
  E[1] = cmul(ey, ph);
  E[2] = make_double2(0.0, 0.0);
  // -i k3 k1 / kc^2 : (-i)(k3re + i k3im) = k3im - i k3re
  const double2 mik3 = make_double2(P.pk3im / P.pkc2, -P.pk3re / P.pkc2);
  H[0] = cmul(cmul(mik3, make_double2(P.pk1 * s1 * c2, 0.0)), ph);
  H[1] = cmul(cmul(mik3, make_double2(P.pk2 * c1 * s2, 0.0)), ph);
  H[2] = cmul(make_double2(c1 * c2, 0.0), ph);
}

__device__ inline void load_cell_vertices(const ProbArgs& P, int64_t gc, double (*sX)[3]) {
  const int t = threadIdx.x;
  if (t < 24) {
    const int v = t / 3, a = t % 3;
    const int64_t vid = P.cells[gc * 8 + v];
    sX[v][a] = P.vertices[vid * 3 + a] * P.inv_len;
  }
}

// ================================================================ scaling
__global__ __launch_bounds__(NT) void k_cell_scale(DevTables T, ProbArgs P, ChunkArgs C) {
  const int64_t cell = blockIdx.x;
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  __shared__ double sX[8][3];
  __shared__ int s_bad;
  extern __shared__ double smem[];
  double* sGc = smem;                         // [nq][6]
  double* sGm = sGc + 6 * T.nq;               // [nq][6]
  double* sQ = sGm + 6 * T.nq;                // [6][nfq][6]
  load_cell_vertices(P, gc, sX);
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  double* gm = C.met + cell * met_stride(T);
  for (int q = threadIdx.x; q < T.nq; q += NT) {
    Geo g;
    trilinear(sX, T.vol_pts[3 * q], T.vol_pts[3 * q + 1], T.vol_pts[3 * q + 2], g);
    if (!(g.det > 0.0) || !isfinite(g.det)) atomicOr(&s_bad, 1);
    vol_metrics(g, T.vol_w[q], &sGc[6 * q], &sGm[6 * q]);
    // the maps of the trial-to-test contractions: w det J^{-T} (covariant test
    // functions times the volume element) and w J (their curls times det J)
    double* pj = gm + 12 * T.nq + 36 * T.nfq + 9 * q;
    double* qj = gm + 21 * T.nq + 36 * T.nfq + 9 * q;
    const double wd = T.vol_w[q] * g.det, w = T.vol_w[q];
    for (int e = 0; e < 9; ++e) {
      pj[e] = wd * g.Ji[e / 3][e % 3];
      qj[e] = w * g.J[e / 3][e % 3];
    }
  }
  int8_t fk[6];
  for (int f = 0; f < 6; ++f) fk[f] = P.face_kind[gc * 6 + f];
  for (int f = 0; f < 6; ++f) {
    if (!is_robin(fk[f])) continue;
    for (int fq = threadIdx.x; fq < T.nfq; fq += NT) {
      const double* xi = &T.face_pts[(f * T.nfq + fq) * 3];
      Geo g;
      trilinear(sX, xi[0], xi[1], xi[2], g);
      double n[3], s;
      face_normal(g, f, n, s);
      face_metric(g, n, T.face_w[f * T.nfq + fq] * s, &sQ[(f * T.nfq + fq) * 6]);
    }
  }
  __syncthreads();
  const double2 eps = make_double2(P.eps[2 * gc], P.eps[2 * gc + 1]);
  const double2 mu = make_double2(P.mu[2 * gc], P.mu[2 * gc + 1]);
  const double om2 = P.omega * P.omega;
  const double cF = om2 * (eps.x * eps.x + eps.y * eps.y) + P.alpha;
  const double cI = om2 * (mu.x * mu.x + mu.y * mu.y) + P.alpha;
  double z2[6];
  for (int f = 0; f < 6; ++f) {
    const double zr = P.zinv[(gc * 6 + f) * 2], zi = P.zinv[(gc * 6 + f) * 2 + 1];
    z2[f] = zr * zr + zi * zi;
  }
  double* d = C.dscale + cell * (int64_t)T.nvp;
  for (int i = threadIdx.x; i < T.Np; i += NT) {
    double dF = 1.0, dI = 1.0;
    if (i < T.N) {
      const int a = T.comp[i];
      double S = 0.0, M = 0.0;
      for (int q = 0; q < T.nq; ++q) {
        const double* c = &T.vol_c[((size_t)q * T.Np + i) * 3];
        const double* G = &sGc[6 * q];
        const double v = T.vol_v[(size_t)q * T.Np + i];
        S += c[0] * (G[0] * c[0] + 2.0 * G[3] * c[1] + 2.0 * G[4] * c[2]) +
             c[1] * (G[1] * c[1] + 2.0 * G[5] * c[2]) + c[2] * G[2] * c[2];
        M += v * v * sGm[6 * q + a];
      }
      double mtF = 0.0, mtI = 0.0;
      for (int f = 0; f < 6; ++f) {
        if (!is_robin(fk[f])) continue;
        double mt = 0.0;
        for (int fq = 0; fq < T.nfq; ++fq) {
          const double v = T.face_v[((size_t)f * T.nfq + fq) * T.Np + i];
          mt += v * v * sQ[(f * T.nfq + fq) * 6 + a];
        }
        mtF += z2[f] * mt;
        mtI += mt;
      }
      dF = 1.0 / sqrt(S + cF * M + mtF);
      dI = 1.0 / sqrt(S + cI * M + mtI);
    }
    d[i] = dF;
    d[T.Np + i] = dI;
  }
  // keep the point metrics for the formation kernels
  for (int e = threadIdx.x; e < 12 * T.nq + 36 * T.nfq; e += NT) gm[e] = smem[e];
  if (threadIdx.x == 0) C.info[gc - C.cell_base] = s_bad ? -1 : 0;
}

// ================================================================ G_IF
// G_IF(i,j) = conj(G_FI(j,i)) = -i w mu C_ji - i w conj(eps) C_ij + sum_R conj(z) Rt_ij,
// from the geometry-free C and Rt; also zero in the F-pad columns / I-pad rows.
__global__ __launch_bounds__(NT) void k_form_IF(DevTables T, ProbArgs P, ChunkArgs C) {
  const int nt = (T.Np + 63) / 64;
  int64_t cell;
  int tile;
  if (!decode_cell_tile(C.n, nt * nt, cell, tile)) return;
  const int64_t gc = C.cell_ids[cell];
  const int I0 = (tile / nt) * 64, J0 = (tile % nt) * 64;
  const double2 eps = make_double2(P.eps[2 * gc], P.eps[2 * gc + 1]);
  const double2 mu = make_double2(P.mu[2 * gc], P.mu[2 * gc + 1]);
  const double om = P.omega;
  double2 zc[6];
  int8_t fk[6];
  for (int f = 0; f < 6; ++f) {
    fk[f] = P.face_kind[gc * 6 + f];
    zc[f] = make_double2(P.zinv[(gc * 6 + f) * 2], -P.zinv[(gc * 6 + f) * 2 + 1]);
  }
  const double* __restrict__ d = C.dscale + cell * (int64_t)T.nvp;
  double2* __restrict__ Z = C.Z + cell * T.zstride;
  const double* __restrict__ Cref = T.Cref;
  const double* __restrict__ CrefT = T.CrefT;
  const int64_t ld = T.ldz;
  const int il = threadIdx.x & 63;
  const int i = I0 + il;
  if (i >= T.Np) return;
  // the wave's columns jl = wave + 4 n in batches of NB = 4: the table loads
  // of a batch are in flight together (all sixteen at once take too many
  // registers: 3 waves per SIMD, slower)
  constexpr int NB = 4;
  const int wv = threadIdx.x >> 6;
  const double di = d[T.Np + i];
  for (int jb = J0 + wv; jb < J0 + 64 && jb < T.Np; jb += NB * (NT / 64)) {
    double cji[NB], cij[NB], dj[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      const int j = jb + n * (NT / 64);
      const bool ok = i < T.N && j < T.N;
      cji[n] = ok ? Cref[(size_t)j * T.N + i] : 0.0;
      cij[n] = ok ? CrefT[(size_t)j * T.N + i] : 0.0;
      dj[n] = j < T.Np ? d[j] : 0.0;
    }
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      const int j = jb + n * (NT / 64);
      if (j >= T.Np || j >= J0 + 64) break;
      double2 v = make_double2(0.0, 0.0);
      if (i < T.N && j < T.N) {
        // -i w mu cji = w (mu.y, -mu.x) cji ; -i w conj(eps) cij = w (-eps.y, -eps.x) cij
        v.x = om * (mu.y * cji[n] - eps.y * cij[n]);
        v.y = om * (-mu.x * cji[n] - eps.x * cij[n]);
        for (int f = 0; f < 6; ++f) {
          if (!is_robin(fk[f])) continue;
          const double rt = T.RtT[((size_t)f * T.N + j) * T.N + i];
          v.x += zc[f].x * rt;
          v.y += zc[f].y * rt;
        }
        const double sc = di * dj[n];
        v.x *= sc;
        v.y *= sc;
      }
      Z[(int64_t)j * ld + T.Np + i] = v;
    }
  }
}

// Identity/zero padding of the test space (rows N..Np-1 of each field block),
// consecutive threads along the rows of one column (contiguous stores).
__global__ __launch_bounds__(NT) void k_form_pad(DevTables T, ChunkArgs C) {
  const int64_t cell = blockIdx.x;
  if (cell >= C.n) return;
  double2* Z = C.Z + cell * T.zstride;
  const int64_t ld = T.ldz;
  const int npad = T.Np - T.N;
  const int nfb = (T.Np / TB) * TB;     // the real F block lives in its compact copy
  double* fr = C.fr + cell * fr_stride(T);
  const int64_t ldf = fr_ld(T);
  for (int blk = 0; blk < 2; ++blk) {
    const int base = blk * T.Np;
    for (int e = threadIdx.x; e < npad * T.Np; e += NT) {
      const int row = base + T.N + e % npad;
      const int col = base + e / npad;
      if (col > row) continue;
      const double v = col == row ? 1.0 : 0.0;
      if (row < nfb) fr[(int64_t)col * ldf + row] = v;
      else Z[(int64_t)col * ld + row] = make_double2(v, 0.0);
    }
  }
}

// ================================================================ B_f^H by sum factorisation
// The DG trial functions are tensor products of 1D Lagrange factors at the
// Gauss-Lobatto nodes, phi_m = l_{m0}(xi_0) l_{m1}(xi_1) l_{m2}(xi_2), m0
// fastest.  For the test functions of component a and the trial component c,
//   D_c(i,m) = sum_q w det (J^{-1})_{ac} v_i phi_m,
//   R_c(i,m) = sum_q w (J chat_i)_c phi_m
//            = sum_q w [J_{c,a+1} d_{a+2} f_i - J_{c,a+2} d_{a+1} f_i] phi_m
// are three sum-factorisable terms with the weights w det J^{-1}_{ac},
// w J_{c,a+1} and -w J_{c,a+2}.  As for G: T1 over q2 (blocks (i2, m2)), T2
// over q1 (columns (m1, i1)), then an f64 MFMA GEMM with rows (m0, i0) and
// K = (term, q0), whose row operand does not depend on the cell.  Every B
// entry fills four places of (D B_f)^H:
//   column F_i:  row E_cm  conj(dF (i w eps D)),   row H_cm  dF R,
//   column I_i:  row E_cm  dI R,                   row H_cm  conj(dI (-i w mu D)).
// The Robin-face part of B(F, E) (k_form_Bt), the trace rows, the padding
// and the residual row (k_form_T, k_form_resid) are written by other kernels.
// One workgroup per (cell, a, c); a is a compile-time parameter.
template <int Q1, int P1, int CAP>
struct SfbShape {
  static constexpr int S = Q1 - 1;
  static constexpr int NQ = Q1 * Q1 * Q1;
  static constexpr int KD = (Q1 + 3) / 4;         // k-steps of D (rows q0, zero padded)
  static constexpr int KR = (2 * Q1 + 3) / 4;     // k-steps of the two R terms (rows 4 KD + t' Q1 + q0)
  static constexpr int KS = KD + KR;
  __host__ __device__ static constexpr int n(int comp, int dir) { return comp == dir ? S : Q1; }
  __host__ __device__ static constexpr int rows(int a) { return n(a, 0) * P1; }
  __host__ __device__ static constexpr int rtiles(int a) { return (rows(a) + 15) / 16; }
  __host__ __device__ static constexpr int ncb(int a) { return n(a, 1) * P1; }
  // column tiles per chunk: at most 16 tiles in all and at most CAP columns
  // tiles (the tile shape the autotuner picks), but at least one (i2, m2) block
  __host__ __device__ static constexpr int ctiles(int a) {
    return (ncb(a) + 15) / 16 > (16 / rtiles(a) < CAP ? 16 / rtiles(a) : CAP)
               ? (ncb(a) + 15) / 16
               : (16 / rtiles(a) < CAP ? 16 / rtiles(a) : CAP);
  }
  __host__ __device__ static constexpr int cc(int a) { return 16 * ctiles(a); }
  __host__ __device__ static constexpr int nbc(int a) { return cc(a) / ncb(a); }
  __host__ __device__ static constexpr int ccmax() {
    int m = 0;
    for (int a = 0; a < 3; ++a) m = cc(a) > m ? cc(a) : m;
    return m;
  }
  __host__ __device__ static constexpr int nbmax() {
    int m = 0;
    for (int a = 0; a < 3; ++a) m = nbc(a) > m ? nbc(a) : m;
    return m;
  }
  static constexpr int CCP = ccmax();
  // LDS (doubles): q_k, q_k' at the points [k][q]; l_m [m][q]; weights [3][NQ];
  // T1 [3][nbmax][Q1^2]; T2 [4 KS][CCP]; row operands [rtiles][KS][64]
  static constexpr int oV = 0, oD = Q1 * Q1, oP = 2 * Q1 * Q1, oW = oP + P1 * Q1, oT1 = oW + 3 * NQ,
                       oT2 = oT1 + 3 * nbmax() * Q1 * Q1, oA = oT2 + 4 * KS * CCP, total = oA + 4 * KS * 64;
  static_assert(total * 8 <= 80 * 1024, "two workgroups per CU");
};

// test-side 1D factor of B term t (0: D, values; 1: d/dxi_{a+2}; 2: d/dxi_{a+1}) in direction d
__device__ __forceinline__ const double* sfb_tab(int t, int a, int d, const double* sV, const double* sD) {
  const bool der = (t == 1 && d == (a + 2) % 3) || (t == 2 && d == (a + 1) % 3);
  return der ? sD : sV;
}

template <int Q1, int P1, int CAP, int a>
__device__ __forceinline__ void sfb_block(const DevTables& T, const ProbArgs& P, const ChunkArgs& C, int64_t cell,
                                          int c, double* smem) {
  using SH = SfbShape<Q1, P1, CAP>;
  constexpr int NQ = SH::NQ, KD = SH::KD, KS = SH::KS, CCP = SH::CCP, NBM = SH::nbmax();
  constexpr int na0 = SH::n(a, 0), na1 = SH::n(a, 1), na2 = SH::n(a, 2);
  constexpr int R = SH::rows(a), Rt = SH::rtiles(a), ctl = SH::ctiles(a), CC = 16 * ctl, Tn = Rt * ctl;
  constexpr int ncb = SH::ncb(a), nbc = SH::nbc(a), nblk = na2 * P1;
  const int64_t gc = C.cell_ids[cell];
  double* sV = smem + SH::oV;
  double* sD = smem + SH::oD;
  double* sP = smem + SH::oP;
  double* sW = smem + SH::oW;
  double* sT1 = smem + SH::oT1;
  double* sT2 = smem + SH::oT2;
  double* sA = smem + SH::oA;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double* gmet = C.met + cell * met_stride(T);
  const double* wdj = gmet + 12 * NQ + 36 * T.nfq;   // [q][9] w det J^{-1}
  const double* wj = wdj + 9 * NQ;                   // [q][9] w J
  for (int e = tid; e < 2 * Q1 * Q1; e += NT) smem[SH::oV + e] = T.sf_tab[e];
  for (int e = tid; e < P1 * Q1; e += NT) sP[e] = T.sf_phi[e];
  constexpr int u1 = (a + 1) % 3, u2 = (a + 2) % 3;
  for (int q = tid; q < NQ; q += NT) {
    sW[q] = wdj[9 * q + 3 * a + c];
    sW[NQ + q] = wj[9 * q + 3 * c + u1];
    sW[2 * NQ + q] = -wj[9 * q + 3 * c + u2];
  }
  // zero rows of T2: D rows Q1 .. 4 KD, R rows 4 KD + 2 Q1 .. 4 KS
  for (int e = tid; e < (4 * KD - Q1) * CCP; e += NT) sT2[Q1 * CCP + e] = 0.0;
  for (int e = tid; e < (4 * KS - 4 * KD - 2 * Q1) * CCP; e += NT) sT2[(4 * KD + 2 * Q1) * CCP + e] = 0.0;
  __syncthreads();
  // row operands: row (m0, i0) = rt 16 + (lane & 15), m0 fastest; k = 4 ks + (lane >> 4)
  for (int e = tid; e < Rt * KS * 64; e += NT) {
    const int ln = e & 63, ks = (e >> 6) % KS, rt = e / (64 * KS);
    const int row = rt * 16 + (ln & 15), kk = 4 * ks + (ln >> 4);
    int t, q0;
    if (ks < KD) {
      t = 0;
      q0 = kk;
    } else {
      const int r = kk - 4 * KD;
      t = 1 + r / Q1;
      q0 = r - (t - 1) * Q1;
    }
    const int m0 = row % P1, i0 = row / P1;
    const double* ft = sfb_tab(t < 3 ? t : 0, a, 0, sV, sD);
    sA[e] = row < R && t < 3 && q0 < Q1 ? ft[i0 * Q1 + q0] * sP[m0 * Q1 + q0] : 0.0;
  }
  const double2 eps = make_double2(P.eps[2 * gc], P.eps[2 * gc + 1]);
  const double2 mu = make_double2(P.mu[2 * gc], P.mu[2 * gc + 1]);
  const double om = P.omega;
  const double* dsc = C.dscale + cell * (int64_t)T.nvp;
  double2* Z = C.Z + cell * T.zstride;
  const int64_t ld = T.ldz;
  const int m1t = T.m1;
  const int64_t rowE = T.nvp + (int64_t)c * m1t, rowH = T.nvp + (int64_t)(3 + c) * m1t;

  for (int g0 = 0; g0 < nblk; g0 += nbc) {
    const int nb = min(nbc, nblk - g0);
    // ---- T1(t, blk; q0, q1) = sum_q2 X2 W_t, block (m2, i2) = (g % P1, g / P1)
    for (int e = tid; e < 3 * nb * Q1 * Q1; e += NT) {
      const int q0 = e % Q1, q1 = (e / Q1) % Q1, r = e / (Q1 * Q1);
      const int blk = r % nb, t = r / nb;
      const int g = g0 + blk, m2 = g % P1, i2 = g / P1;
      const double* ft = sfb_tab(t, a, 2, sV, sD);
      const double* wv = sW + t * NQ + q0 + Q1 * q1;
      double acc = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < Q1; ++q2) acc = fma(ft[i2 * Q1 + q2] * sP[m2 * Q1 + q2], wv[Q1 * Q1 * q2], acc);
      sT1[(t * NBM + blk) * Q1 * Q1 + q1 * Q1 + q0] = acc;
    }
    __syncthreads();
    // ---- T2(t q0; col) = sum_q1 X1 T1, column (m1, i1, blk), m1 fastest
    for (int e = tid; e < 3 * CC; e += NT) {
      const int t = e / CC, col = e - t * CC;
      const int blk = col / ncb, cc = col - blk * ncb;
      double out[Q1];
#pragma unroll
      for (int q0 = 0; q0 < Q1; ++q0) out[q0] = 0.0;
      if (blk < nb) {
        const int m1 = cc % P1, i1 = cc / P1;
        const double* ft = sfb_tab(t, a, 1, sV, sD);
        const double* t1 = sT1 + (t * NBM + blk) * Q1 * Q1;
#pragma unroll 2
        for (int q1 = 0; q1 < Q1; ++q1) {
          const double x = ft[i1 * Q1 + q1] * sP[m1 * Q1 + q1];
#pragma unroll
          for (int q0 = 0; q0 < Q1; ++q0) out[q0] = fma(x, t1[q1 * Q1 + q0], out[q0]);
        }
      }
      const int row0 = t == 0 ? 0 : 4 * KD + (t - 1) * Q1;
#pragma unroll
      for (int q0 = 0; q0 < Q1; ++q0) sT2[(row0 + q0) * CCP + col] = out[q0];
    }
    __syncthreads();
    // ---- D (rows of term 0) and R (terms 1, 2)
    d4 acD[4], acR[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acD[k] = acR[k] = d4{0, 0, 0, 0};
    auto kstep = [&](int ks, d4* acc) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int tau = w + 4 * k;
        if (tau < Tn) {
          const double av = sA[((tau % Rt) * KS + ks) * 64 + lane];
          const double bv = sT2[(4 * ks + (lane >> 4)) * CCP + (tau / Rt) * 16 + (lane & 15)];
          acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[k], 0, 0, 0);
        }
      }
    };
#pragma unroll
    for (int ks = 0; ks < KD; ++ks) kstep(ks, acD);
#pragma unroll 2
    for (int ks = KD; ks < KS; ++ks) kstep(ks, acR);
    // ---- the four entries of every (i, m) (the scale factors are all
    // loaded before the first store: a wait for a load also waits for the
    // stores issued before it)
    double sF[4][4], sI[4][4];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int tau = w + 4 * k;
        if (tau >= Tn) continue;
        const int col = (tau / Rt) * 16 + (lane & 15);
        const int blk = col / ncb, cc = col - blk * ncb;
        if (blk >= nb) continue;
        const int g = g0 + blk, m2 = g % P1, i2 = g / P1;
        const int ib = a * T.nc + na0 * ((cc / P1) + na1 * i2), mb = P1 * ((cc % P1) + P1 * m2);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int row = (tau % Rt) * 16 + (lane >> 4) + 4 * it;
          if (row >= R) continue;
          const int i = ib + row / P1, m = mb + row % P1;
          if (pass == 0) {
            sF[k][it] = dsc[i];
            sI[k][it] = dsc[T.Np + i];
            continue;
          }
          const double D = acD[k][it], Rv = acR[k][it];
          const double dF = sF[k][it], dI = sI[k][it];
          double2* zf = Z + (int64_t)i * ld;
          double2* zi = Z + (int64_t)(T.Np + i) * ld;
          zf[rowE + m] = make_double2(-dF * om * eps.y * D, -dF * om * eps.x * D);
          zf[rowH + m] = make_double2(dF * Rv, 0.0);
          zi[rowE + m] = make_double2(dI * Rv, 0.0);
          zi[rowH + m] = make_double2(dI * om * mu.y * D, dI * om * mu.x * D);
        }
      }
  }
}

template <int Q1, int P1, int CAP>
__global__ __launch_bounds__(NT, 2) void k_form_Bsf(DevTables T, ProbArgs P, ChunkArgs C) {
  int64_t cell;
  int ac;
  if (!decode_cell_tile(C.n, 9, cell, ac)) return;
  extern __shared__ double smem[];
  const int c = ac % 3;
  switch (ac / 3) {
    case 0: sfb_block<Q1, P1, CAP, 0>(T, P, C, cell, c, smem); break;
    case 1: sfb_block<Q1, P1, CAP, 1>(T, P, C, cell, c, smem); break;
    default: sfb_block<Q1, P1, CAP, 2>(T, P, C, cell, c, smem); break;
  }
}

// ================================================================ residual row
// The volume part of D B_f x for every test function, without forming B:
// the trial coefficients are interpolated to the points (three 1D passes
// over the DG factors), combined pointwise with the metric into the fields
// that the test functions of component a meet,
//   F rows:  g0 = i w eps sum_c w det J^{-1}_{ac} E_c,  g1 = sum_c w J_{c,a+1} H_c,  g2 = -sum_c w J_{c,a+2} H_c,
//   I rows:  g0 = -i w mu sum_c w det J^{-1}_{ac} H_c,  g1 = sum_c w J_{c,a+1} E_c,  g2 = -sum_c w J_{c,a+2} E_c,
// (E_c, H_c the interpolated trial fields), and integrated against them with
// three 1D passes over the test factors (g1 meets d_{a+2} f_i, g2 meets
// d_{a+1} f_i).  Writes d (B_f x)_i, unconjugated, to the residual row of
// columns i < N; k_form_Bt adds the Robin-face part and k_form_T the trace
// part and takes the conjugate.  One workgroup per cell; fixed summation order.
template <int Q1, int P1>
struct SfrShape {
  static constexpr int NQ = Q1 * Q1 * Q1, M1 = P1 * P1 * P1;
  // interpolation: 12 real fields (E_c, H_c; re, im)
  static constexpr int nA = 12 * P1 * P1 * Q1, nB = 12 * P1 * Q1 * Q1;
  // test integration of one (a, side): fields [3][2][NQ], T1 [3][2][Q1][Q1^2], T2 [3][2][Q1^2][Q1]
  static constexpr int nG = 6 * NQ, nT1 = 6 * Q1 * Q1 * Q1;
  static constexpr int nR1 = nA + nB > nG + nT1 ? nA + nB : nG + nT1;
  static constexpr int oV = 0, oD = Q1 * Q1, oP = 2 * Q1 * Q1, oX = oP + P1 * Q1, oU = oX + 12 * M1,
                       oR1 = oU + 12 * NQ, total = oR1 + nR1;
  static_assert(total * 8 <= 160 * 1024, "fits the LDS of a CU");
};

template <int Q1, int P1>
__global__ __launch_bounds__(NT) void k_form_resid(DevTables T, ProbArgs P, ChunkArgs C) {
  using SH = SfrShape<Q1, P1>;
  constexpr int NQ = SH::NQ, M1 = SH::M1, S = Q1 - 1;
  const int64_t cell = blockIdx.x;
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  extern __shared__ double smem[];
  double* sV = smem + SH::oV;
  double* sD = smem + SH::oD;
  double* sP = smem + SH::oP;
  double* sX = smem + SH::oX;     // [12][M1], field f = 2 (3 h + c) + reim
  double* sU = smem + SH::oU;     // [12][NQ]
  double* sA = smem + SH::oR1;    // [12][P1 P1][Q1]
  double* sB = sA + SH::nA;       // [12][P1][Q1 Q1]
  double* sG = smem + SH::oR1;    // [3][2][NQ] (after the interpolation)
  double* sT1 = sG + SH::nG;      // [3][2][Q1][Q1 Q1]
  double* sT2 = sG;               // [3][2][Q1 Q1][Q1] (after T1)
  const int tid = threadIdx.x;
  const double2* xc = C.x + (C.v_off[gc] - C.v_base);
  for (int e = tid; e < 2 * Q1 * Q1; e += NT) smem[SH::oV + e] = T.sf_tab[e];
  for (int e = tid; e < P1 * Q1; e += NT) sP[e] = T.sf_phi[e];
  for (int e = tid; e < 6 * M1; e += NT) {
    const double2 v = xc[e];   // x[(3 h + c) m1 + m]
    const int f = e / M1, m = e - f * M1;
    sX[(2 * f) * M1 + m] = v.x;
    sX[(2 * f + 1) * M1 + m] = v.y;
  }
  __syncthreads();
  // ---- interpolation to the points: m0 -> q0, m1 -> q1, m2 -> q2
  for (int e = tid; e < 12 * P1 * P1 * Q1; e += NT) {
    const int q0 = e % Q1, r = e / Q1, mm = r % (P1 * P1), f = r / (P1 * P1);
    double acc = 0.0;
#pragma unroll
    for (int m0 = 0; m0 < P1; ++m0) acc = fma(sP[m0 * Q1 + q0], sX[f * M1 + m0 + P1 * mm], acc);
    sA[(f * P1 * P1 + mm) * Q1 + q0] = acc;
  }
  __syncthreads();
  for (int e = tid; e < 12 * P1 * Q1 * Q1; e += NT) {
    const int q0 = e % Q1, q1 = (e / Q1) % Q1, r = e / (Q1 * Q1), m2 = r % P1, f = r / P1;
    double acc = 0.0;
#pragma unroll
    for (int m1 = 0; m1 < P1; ++m1) acc = fma(sP[m1 * Q1 + q1], sA[(f * P1 * P1 + m1 + P1 * m2) * Q1 + q0], acc);
    sB[((f * P1 + m2) * Q1 + q1) * Q1 + q0] = acc;
  }
  __syncthreads();
  for (int e = tid; e < 12 * NQ; e += NT) {
    const int qq = e % (Q1 * Q1), q2 = (e / (Q1 * Q1)) % Q1, f = e / NQ;
    double acc = 0.0;
#pragma unroll
    for (int m2 = 0; m2 < P1; ++m2) acc = fma(sP[m2 * Q1 + q2], sB[(f * P1 + m2) * Q1 * Q1 + qq], acc);
    sU[e] = acc;
  }
  const double2 eps = make_double2(P.eps[2 * gc], P.eps[2 * gc + 1]);
  const double2 mu = make_double2(P.mu[2 * gc], P.mu[2 * gc + 1]);
  const double om = P.omega;
  // i w eps = w (-eps.y, eps.x);  -i w mu = w (mu.y, -mu.x)
  const double2 cE = make_double2(-om * eps.y, om * eps.x), cH = make_double2(om * mu.y, -om * mu.x);
  const double* gmet = C.met + cell * met_stride(T);
  const double* wdj = gmet + 12 * NQ + 36 * T.nfq;
  const double* wj = wdj + 9 * NQ;
  const double* dsc = C.dscale + cell * (int64_t)T.nvp;
  double2* Z = C.Z + cell * T.zstride;
  const int64_t ld = T.ldz, rrow = T.nvp + T.k + 1;
  for (int pass = 0; pass < 6; ++pass) {
    const int a = pass >> 1, side = pass & 1;   // side 0: F rows (E through D, H through R); 1: I rows
    const int na0 = a == 0 ? S : Q1, na1 = a == 1 ? S : Q1, na2 = a == 2 ? S : Q1;
    const int u1 = (a + 1) % 3, u2 = (a + 2) % 3;
    const int fd = side == 0 ? 0 : 6, fr = side == 0 ? 6 : 0;   // fields met by D, by R
    const double2 cd = side == 0 ? cE : cH;
    __syncthreads();   // U complete; G, T1 free
    for (int q = tid; q < NQ; q += NT) {
      double dr = 0.0, di = 0.0, r1r = 0.0, r1i = 0.0, r2r = 0.0, r2i = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double wd = wdj[9 * q + 3 * a + c], j1 = wj[9 * q + 3 * c + u1], j2 = wj[9 * q + 3 * c + u2];
        const double udr = sU[(fd + 2 * c) * NQ + q], udi = sU[(fd + 2 * c + 1) * NQ + q];
        const double urr = sU[(fr + 2 * c) * NQ + q], uri = sU[(fr + 2 * c + 1) * NQ + q];
        dr = fma(wd, udr, dr);
        di = fma(wd, udi, di);
        r1r = fma(j1, urr, r1r);
        r1i = fma(j1, uri, r1i);
        r2r = fma(-j2, urr, r2r);
        r2i = fma(-j2, uri, r2i);
      }
      sG[0 * NQ + q] = cd.x * dr - cd.y * di;
      sG[1 * NQ + q] = cd.x * di + cd.y * dr;
      sG[2 * NQ + q] = r1r;
      sG[3 * NQ + q] = r1i;
      sG[4 * NQ + q] = r2r;
      sG[5 * NQ + q] = r2i;
    }
    __syncthreads();
    // T1[t][ri][i2][q1 q0] = sum_q2 f_t,2(i2, q2) g_t
    for (int e = tid; e < 6 * na2 * Q1 * Q1; e += NT) {
      const int qq = e % (Q1 * Q1), r = e / (Q1 * Q1), i2 = r % na2, tr = r / na2, t = tr >> 1;
      const double* ft = sfb_tab(t, a, 2, sV, sD);
      double acc = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < Q1; ++q2) acc = fma(ft[i2 * Q1 + q2], sG[tr * NQ + q2 * Q1 * Q1 + qq], acc);
      sT1[(tr * Q1 + i2) * Q1 * Q1 + qq] = acc;
    }
    __syncthreads();
    // T2[t][ri][i1 + na1 i2][q0] = sum_q1 f_t,1(i1, q1) T1
    for (int e = tid; e < 6 * na1 * na2 * Q1; e += NT) {
      const int q0 = e % Q1, r = e / Q1, ii = r % (na1 * na2), tr = r / (na1 * na2), t = tr >> 1;
      const int i1 = ii % na1, i2 = ii / na1;
      const double* ft = sfb_tab(t, a, 1, sV, sD);
      double acc = 0.0;
#pragma unroll
      for (int q1 = 0; q1 < Q1; ++q1) acc = fma(ft[i1 * Q1 + q1], sT1[(tr * Q1 + i2) * Q1 * Q1 + q1 * Q1 + q0], acc);
      sT2[(tr * Q1 * Q1 + ii) * Q1 + q0] = acc;
    }
    __syncthreads();
    // (B x)_i = sum_t sum_q0 f_t,0(i0, q0) T2
    for (int il = tid; il < na0 * na1 * na2; il += NT) {
      const int i0 = il % na0, ii = il / na0;
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const double* ft = sfb_tab(t, a, 0, sV, sD);
#pragma unroll
        for (int q0 = 0; q0 < Q1; ++q0) {
          const double fv = ft[i0 * Q1 + q0];
          sr = fma(fv, sT2[((2 * t) * Q1 * Q1 + ii) * Q1 + q0], sr);
          si = fma(fv, sT2[((2 * t + 1) * Q1 * Q1 + ii) * Q1 + q0], si);
        }
      }
      const int i = a * T.nc + il, col = side * T.Np + i;
      Z[(int64_t)col * ld + rrow] = make_double2(dsc[col] * sr, dsc[col] * si);
    }
  }
}

// ================================================================ Robin part of B(F, E)
// On Robin faces B(F_i, E_cm) also holds -sum_R z Dt_c(i,m),
//   Dt_c(i,m) = sum_fq w s (psi_i - (psi_i . n) n)_c phi_m,
// a sum over the face points only.  Added to the rows that k_form_Bsf wrote,
// and its part of D B_f x to the residual row (after k_form_resid).  One
// workgroup per (cell, 64 test functions); cells without a Robin face return
// at once.  Thread t owns test row il = t/4 and the DG functions m = t%4,
// t%4 + 4, ...; the four shares of a row's residual are added in a fixed
// order.
constexpr int BQC = 16;   // face points per staged chunk
constexpr int BIT = 4;    // DG functions per thread and batch
__global__ __launch_bounds__(NT, 2) void k_form_Bt(DevTables T, ProbArgs P, ChunkArgs C) {
  const int nrt = (T.Np + 63) / 64;
  int64_t cell;
  int tile;
  if (!decode_cell_tile(C.n, nrt, cell, tile)) return;
  const int64_t gc = C.cell_ids[cell];
  int rmask = 0;   // bit f: face f is a Robin face
  for (int f = 0; f < 6; ++f) rmask |= is_robin(P.face_kind[gc * 6 + f]) ? 1 << f : 0;
  if (!rmask) return;
  const int i0 = tile * 64;
  __shared__ double sX[8][3];
  __shared__ double sGeo[BQC][9];          // tangential maps w s (r_a - (r_a . n) n)
  __shared__ double sPt[BQC][64][3];       // w s (psi_hat_i tangential)_c
  __shared__ double2 sRes[64][4];
  extern __shared__ double smem[];
  double* sPhi = smem;                      // [BQC][m1]
  load_cell_vertices(P, gc, sX);
  const double2* xc = C.x ? C.x + (C.v_off[gc] - C.v_base) : nullptr;
  const double* d = C.dscale + cell * (int64_t)T.nvp;
  double2* Z = C.Z + cell * T.zstride;
  const int64_t ld = T.ldz;
  const int m1 = T.m1;
  const int il = threadIdx.x >> 2, sub = threadIdx.x & 3;
  const int i = i0 + il;
  const bool ok = i < T.N;
  const double dF = ok ? d[i] : 0.0;
  double2 rF = make_double2(0.0, 0.0);
  __syncthreads();
  for (int ib = 0; ib < m1; ib += 4 * BIT) {
    double Dtr[BIT][3], Dti[BIT][3];
#pragma unroll
    for (int u = 0; u < BIT; ++u)
#pragma unroll
      for (int c = 0; c < 3; ++c) Dtr[u][c] = Dti[u][c] = 0.0;
    for (int f = 0; f < 6; ++f) {
      if (!((rmask >> f) & 1)) continue;
      const double2 zf = make_double2(P.zinv[(gc * 6 + f) * 2], P.zinv[(gc * 6 + f) * 2 + 1]);
      for (int q0 = 0; q0 < T.nfq; q0 += BQC) {
        const int nqc = min(BQC, T.nfq - q0);
        __syncthreads();
        for (int qq = threadIdx.x; qq < nqc; qq += NT) {
          const int fq = q0 + qq;
          const double* xi = &T.face_pts[(f * T.nfq + fq) * 3];
          Geo g;
          trilinear(sX, xi[0], xi[1], xi[2], g);
          double n[3], sa;
          face_normal(g, f, n, sa);
          const double ws = T.face_w[f * T.nfq + fq] * sa;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double rn = g.Ji[a][0] * n[0] + g.Ji[a][1] * n[1] + g.Ji[a][2] * n[2];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) sGeo[qq][a * 3 + cc] = ws * (g.Ji[a][cc] - rn * n[cc]);
          }
        }
        for (int e = threadIdx.x; e < nqc * m1; e += NT)
          sPhi[e] = T.face_phi[((size_t)f * T.nfq + q0 + e / m1) * m1 + e % m1];
        __syncthreads();
        for (int e = threadIdx.x; e < nqc * 64; e += NT) {
          const int qq = e / 64, jl = e % 64;
          const int ii = min(i0 + jl, T.N - 1);
          const int a = T.comp[ii];
          const double v = T.face_v[((size_t)f * T.nfq + q0 + qq) * T.Np + ii];
          for (int cc = 0; cc < 3; ++cc) sPt[qq][jl][cc] = v * sGeo[qq][a * 3 + cc];
        }
        __syncthreads();
        for (int qq = 0; qq < nqc; ++qq) {
          const double p0 = sPt[qq][il][0], p1 = sPt[qq][il][1], p2 = sPt[qq][il][2];
#pragma unroll
          for (int u = 0; u < BIT; ++u) {
            const int m = ib + sub + 4 * u;
            const double ph = (m < m1) ? sPhi[qq * m1 + m] : 0.0;
            Dtr[u][0] += zf.x * p0 * ph;
            Dtr[u][1] += zf.x * p1 * ph;
            Dtr[u][2] += zf.x * p2 * ph;
            Dti[u][0] += zf.y * p0 * ph;
            Dti[u][1] += zf.y * p1 * ph;
            Dti[u][2] += zf.y * p2 * ph;
          }
        }
      }
    }
    // stored conj(dF (-z Dt)) = (-dF Re(z Dt), dF Im(z Dt)), added to the volume part
    if (ok) {
#pragma unroll
      for (int u = 0; u < BIT; ++u) {
        const int m = ib + sub + 4 * u;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          if (m >= m1) break;
          double2* z = Z + (int64_t)i * ld + T.nvp + cc * m1 + m;
          const double2 dl = make_double2(-dF * Dtr[u][cc], dF * Dti[u][cc]);
          const double2 v = *z;
          *z = make_double2(v.x + dl.x, v.y + dl.y);
          if (xc) {
            // (d B x) += conj(stored) x
            const double2 xe = xc[cc * m1 + m];
            rF.x += dl.x * xe.x + dl.y * xe.y;
            rF.y += dl.x * xe.y - dl.y * xe.x;
          }
        }
      }
    }
  }
  if (!xc) return;
  sRes[il][sub] = rF;
  __syncthreads();
  if (sub == 0 && ok) {
    double2 s = sRes[il][0];
    for (int q = 1; q < 4; ++q) s = make_double2(s.x + sRes[il][q].x, s.y + sRes[il][q].y);
    double2* z = Z + (int64_t)i * ld + T.nvp + T.k + 1;
    const double2 v = *z;
    *z = make_double2(v.x + s.x, v.y + s.y);
  }
}

// ================================================================ trace rows, padding, residual
// Per (cell, 64 test functions):
//   B(F_i, Hhat_j) = sum_{f not Robin} T_f(i,j),  B(I_i, Ehat_j) = sum_f T_f(i,j)
// (real, geometry free: the pairing summed over all faces is a table and
// Robin faces are taken off it for the F rows), the zero rows of the
// padding test functions, the zero load row (k_form_load writes the load on
// port cells) and the residual row conj(D B_f x), whose volume and Robin
// parts k_form_resid and k_form_Bt left in the row.  A wave takes two columns
// at a time, its lanes along the trace rows in chunks of 64 (coalesced
// stores); each lane sums its rows' part of D B_f x over the chunks and the
// wave reduces each column's sum once, in a fixed order.  The zero E-hat
// entries that no kernel reads (trace_unwritten) are not stored.
template <int MCH>   // chunks of 64 trace rows: ceil(nt1 / 64)
__global__ __launch_bounds__(NT) void k_form_T(DevTables T, ProbArgs P, ChunkArgs C) {
  const int nrt = (T.Np + 63) / 64;
  int64_t cell;
  int tile;
  if (!decode_cell_tile(C.n, nrt, cell, tile)) return;
  const int64_t gc = C.cell_ids[cell];
  const int i0 = tile * 64;
  const double2* __restrict__ xc = C.x ? C.x + (C.v_off[gc] - C.v_base) : nullptr;
  int rmask = 0;
  for (int f = 0; f < 6; ++f) rmask |= is_robin(P.face_kind[gc * 6 + f]) ? 1 << f : 0;
  const int nrobin = __builtin_popcount(rmask);
  const double* __restrict__ d = C.dscale + cell * (int64_t)T.nvp;
  double2* __restrict__ Z = C.Z + cell * T.zstride;
  const int64_t ld = T.ldz;
  const int nvp = T.nvp;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ncol = min(64, T.Np - i0);   // columns of this tile
  // interior rows of the padding test functions: zero
  for (int jl = wv; jl < ncol; jl += NT / 64) {
    const int ii = i0 + jl;
    if (ii < T.N) continue;
    for (int r = lane; r < T.nu; r += 64) {
      Z[(int64_t)ii * ld + nvp + r] = make_double2(0.0, 0.0);
      Z[(int64_t)(T.Np + ii) * ld + nvp + r] = make_double2(0.0, 0.0);
    }
  }
  // G columns of the wave at a time (jl = jb + 4 g).  Every load of a batch
  // (table values of all its chunks of trace rows, the residual row's volume
  // part) is issued before its stores, and the x values of the trace rows
  // once per wave: a wait for a load also waits for the stores issued before
  // it.
  constexpr int G = 2;
  const double* __restrict__ Tsum = T.Tsum;
  double2 xe[MCH], xh[MCH];
#pragma unroll
  for (int c = 0; c < MCH; ++c) {
    const int jt = 64 * c + lane;
    const bool ok = xc && jt < T.nt1;
    xe[c] = ok ? xc[T.nu + jt] : make_double2(0.0, 0.0);
    xh[c] = ok ? xc[T.nu + T.nt1 + jt] : make_double2(0.0, 0.0);
  }
  for (int jb = wv; jb < ncol; jb += G * (NT / 64)) {
    double dF[G], dI[G], tI[MCH][G];
    double2 aF[G], aI[G], rF[G], rI[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int jl = min(jb + g * (NT / 64), ncol - 1), ii = i0 + jl;
      dF[g] = d[ii];
      dI[g] = d[T.Np + ii];
      aF[g] = make_double2(0.0, 0.0);
      aI[g] = aF[g];
      // the residual row's volume part (lane 1 carries the row in the tail below)
      const bool rv = xc && lane == 1 && ii < T.N && jb + g * (NT / 64) < ncol;
      const int row = nvp + T.k + 1;
      rF[g] = rv ? Z[(int64_t)ii * ld + row] : make_double2(0.0, 0.0);
      rI[g] = rv ? Z[(int64_t)(T.Np + ii) * ld + row] : make_double2(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < MCH; ++c) {
        const int jt = 64 * c + lane;
        tI[c][g] = (ii < T.N && jt < T.nt1 && jb + g * (NT / 64) < ncol) ? Tsum[(size_t)ii * T.nt1 + jt] : 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < MCH; ++c) {
      const int jt = 64 * c + lane;
      if (64 * c >= T.nt1) break;
      const bool okt = jt < T.nt1;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int jl = jb + g * (NT / 64);
        if (jl >= ncol) break;
        const int ii = i0 + jl;
        const bool okc = ii < T.N && okt;
        double tF = tI[c][g];
        if (nrobin && okc) {
          for (int f = 0; f < 6; ++f)
            if ((rmask >> f) & 1) tF -= T.T[((size_t)f * T.N + ii) * T.nt1 + jt];
        }
        const double tf = dF[g] * tF, ti = dI[g] * tI[c][g];
        if (okt) {
          const int rowEh = nvp + T.nu + jt, rowHh = nvp + T.nu + T.nt1 + jt;
          if (!trace_unwritten(T, rowEh, ii)) Z[(int64_t)ii * ld + rowEh] = make_double2(0.0, 0.0);
          Z[(int64_t)ii * ld + rowHh] = make_double2(tf, 0.0);
          Z[(int64_t)(T.Np + ii) * ld + rowEh] = make_double2(ti, 0.0);
          Z[(int64_t)(T.Np + ii) * ld + rowHh] = make_double2(0.0, 0.0);
          if (xc) {
            aF[g].x += tf * xh[c].x;
            aF[g].y += tf * xh[c].y;
            aI[g].x += ti * xe[c].x;
            aI[g].y += ti * xe[c].y;
          }
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int jl = jb + g * (NT / 64);
      if (jl >= ncol) break;
      const int ii = i0 + jl;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        aF[g].x += __shfl_xor(aF[g].x, off, 64);
        aF[g].y += __shfl_xor(aF[g].y, off, 64);
        aI[g].x += __shfl_xor(aI[g].x, off, 64);
        aI[g].y += __shfl_xor(aI[g].y, off, 64);
      }
      // the rows after the trace rows, by the same wave right after them (one
      // contiguous run per column): zero load row, residual row (its volume
      // part, if any, plus the trace part, conjugated), zero padding
      for (int rr = lane; rr < T.kp - T.k; rr += 64) {
        const int row = nvp + T.k + rr;
        double2 vF = make_double2(0.0, 0.0), vI = vF;
        if (rr == 1 && xc) {
          vF = rF[g];
          vI = rI[g];
          vF.x += aF[g].x;
          vF.y += aF[g].y;
          vI.x += aI[g].x;
          vI.y += aI[g].y;
          vF.y = -vF.y;
          vI.y = -vI.y;
        }
        Z[(int64_t)ii * ld + row] = vF;
        Z[(int64_t)(T.Np + ii) * ld + row] = vI;
      }
    }
  }
}

// Load vector l(F_i) = - sum_port int psi_i . g dS, written to RHS row k as
// conj(d l).  One workgroup per (cell, 64 test functions); no-op for cells
// without a port face.
__global__ __launch_bounds__(NT) void k_form_load(DevTables T, ProbArgs P, ChunkArgs C) {
  const int nrt = (T.Np + 63) / 64;
  int64_t cell;
  int tile;
  if (!decode_cell_tile(C.n, nrt, cell, tile)) return;
  const int64_t gc = C.cell_ids[cell];
  const int i0 = tile * 64;
  __shared__ double sX[8][3];
  extern __shared__ double smem[];
  double2* sRG = reinterpret_cast<double2*>(smem);   // [nfq][3]: w s (r_a . g)
  int8_t fk[6];
  int nport = 0;
  for (int f = 0; f < 6; ++f) {
    fk[f] = P.face_kind[gc * 6 + f];
    nport += (fk[f] == 2);
  }
  if (!P.has_port || nport == 0) return;   // row already zero
  load_cell_vertices(P, gc, sX);
  const int il = threadIdx.x & 63;
  const int i = i0 + il;
  double2 acc = make_double2(0.0, 0.0);
  for (int f = 0; f < 6; ++f) {
    if (fk[f] != 2) continue;
    const double2 z = make_double2(P.zinv[(gc * 6 + f) * 2], P.zinv[(gc * 6 + f) * 2 + 1]);
    __syncthreads();
    for (int fq = threadIdx.x; fq < T.nfq; fq += NT) {
      const double* xi = &T.face_pts[(f * T.nfq + fq) * 3];
      Geo g;
      trilinear(sX, xi[0], xi[1], xi[2], g);
      double n[3], s;
      face_normal(g, f, n, s);
      double2 E[3], H[3];
      te_fields(P, P.omega, g.x, E, H);
      double2 En = make_double2(0, 0);
#pragma unroll
      for (int a = 0; a < 3; ++a) En = make_double2(En.x + E[a].x * n[a], En.y + E[a].y * n[a]);
      double2 gv[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        const double2 nxh = make_double2(n[b] * H[c].x - n[c] * H[b].x, n[b] * H[c].y - n[c] * H[b].y);
        const double2 et = make_double2(E[a].x - En.x * n[a], E[a].y - En.y * n[a]);
        const double2 zet = cmul(z, et);
        gv[a] = make_double2(nxh.x + zet.x, nxh.y + zet.y);
      }
      const double ws = T.face_w[f * T.nfq + fq] * s;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double2 rg = make_double2(0, 0);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          rg.x += g.Ji[a][cc] * gv[cc].x;
          rg.y += g.Ji[a][cc] * gv[cc].y;
        }
        sRG[fq * 3 + a] = make_double2(ws * rg.x, ws * rg.y);
      }
    }
    __syncthreads();
    if (threadIdx.x < 64 && i < T.N) {
      const int a = T.comp[i];
      for (int fq = 0; fq < T.nfq; ++fq) {
        const double v = T.face_v[((size_t)f * T.nfq + fq) * T.Np + i];
        acc.x -= v * sRG[fq * 3 + a].x;
        acc.y -= v * sRG[fq * 3 + a].y;
      }
    }
  }
  if (threadIdx.x < 64 && i < T.N) {
    const double* d = C.dscale + cell * (int64_t)T.nvp;
    double2* Z = C.Z + cell * T.zstride;
    double2* zc = Z + (int64_t)i * T.ldz + T.nvp + T.k;
    zc[0] = make_double2(d[i] * acc.x, -d[i] * acc.y);           // conj(d l)
    if (C.x) zc[1] = make_double2(zc[1].x - d[i] * acc.x, zc[1].y + d[i] * acc.y);   // conj(d (B x - l))
  }
}

// ================================================================ MFMA core
// Complex 64x64 tile product  P += A B^H  with A, B row panels of column-major
// complex matrices, over columns [0, K).  Four waves; wave (wr, wc) owns the
// 32x32 quadrant rows wr*32.., cols wc*32.. as 2x2 blocks of 16x16, each a
// real and an imaginary f64 MFMA accumulator.  Accumulator item v of lane l
// of a 16x16 block holds row (l>>4) + 4v, column l & 15.
struct Acc {
  d4 re[2][2], im[2][2];
};

struct Stage {
  double Are[KC][LDP], Aim[KC][LDP], Bre[KC][LDP], Bim[KC][LDP];
};

__device__ inline void acc_zero(Acc& c) {
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      c.re[u][v] = d4{0, 0, 0, 0};
      c.im[u][v] = d4{0, 0, 0, 0};
    }
}

// Operand kinds of a tile product: both complex, complex x real (B exactly
// real), real x real.  Rows of the factor that belong to the F test block are
// exactly real (G_FF is real), so products with such rows skip the MFMAs
// whose operands are exact zeros.
enum { MM_CC = 0, MM_CR = 1, MM_RR = 2 };

// One k-step of 4 for the wave's 2x2 blocks: re += Ar Br + Ai Bi, im += Ai Br - Ar Bi.
template <int MODE>
__device__ __forceinline__ void cmfma_step(const double* ar, const double* ai, const double* br, const double* bi,
                                           Acc& c) {
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) c.re[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[u], br[v], c.re[u][v], 0, 0, 0);
  if (MODE == MM_RR) return;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) c.im[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[u], br[v], c.im[u][v], 0, 0, 0);
  if (MODE == MM_CR) return;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) c.re[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[u], bi[v], c.re[u][v], 0, 0, 0);
  double nar[2] = {-ar[0], -ar[1]};
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) c.im[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(nar[u], bi[v], c.im[u][v], 0, 0, 0);
}

template <int MODE>
__device__ inline void stage_compute(const Stage& s, Acc& c) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w & 1, wc = w >> 1;
#pragma unroll
  for (int ks = 0; ks < KC / 4; ++ks) {
    const int kk = ks * 4 + (lane >> 4);
    double ar[2], ai[2] = {0.0, 0.0}, br[2], bi[2] = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int row = wr * 32 + u * 16 + (lane & 15);
      ar[u] = s.Are[kk][row];
      if (MODE != MM_RR) ai[u] = s.Aim[kk][row];
      const int col = wc * 32 + u * 16 + (lane & 15);
      br[u] = s.Bre[kk][col];
      if (MODE == MM_CC) bi[u] = s.Bim[kk][col];
    }
    cmfma_step<MODE>(ar, ai, br, bi, c);
  }
}

// P += A[rowA:rowA+64, 0:K] * B[rowB:rowB+64, 0:K]^H ; A, B column-major with leading dim ld.
template <int MODE = MM_CC>
__device__ inline void gemm_abh(const double2* __restrict__ A, const double2* __restrict__ B, int64_t ld, int K,
                                Stage* st, Acc& c) {
  if (K <= 0) return;
  const int t = threadIdx.x;
  const int lr = t & 63, lc = t >> 6;
  double2 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t col = k0 + lc * 4 + u;
      ra[u] = A[col * ld + lr];
      rb[u] = B[col * ld + lr];
    }
  };
  auto lstore = [&](Stage& s) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s.Are[lc * 4 + u][lr] = ra[u].x;
      if (MODE != MM_RR) s.Aim[lc * 4 + u][lr] = ra[u].y;
      s.Bre[lc * 4 + u][lr] = rb[u].x;
      if (MODE == MM_CC) s.Bim[lc * 4 + u][lr] = rb[u].y;
    }
  };
  gload(0);
  lstore(st[0]);
  __syncthreads();
  const int nst = K / KC;
  for (int sidx = 0; sidx < nst; ++sidx) {
    const bool more = sidx + 1 < nst;
    if (more) gload((sidx + 1) * KC);
    stage_compute<MODE>(st[sidx & 1], c);
    if (more) lstore(st[(sidx + 1) & 1]);
    __syncthreads();
  }
}

// Visit the accumulator elements: f(row, col, re, im) with row/col in [0,64).
template <class F>
__device__ inline void acc_for_each(const Acc& c, F&& f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w & 1, wc = w >> 1;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int row = wr * 32 + u * 16 + (lane >> 4) + 4 * it;
        const int col = wc * 32 + v * 16 + (lane & 15);
        f(row, col, c.re[u][v][it], c.im[u][v][it]);
      }
}

// ================================================================ G_FF, G_II
// Sum factorisation.  The test functions of component a are tensor products
//   psi_hat_i = q_{i0}(xi_0) q_{i1}(xi_1) q_{i2}(xi_2) e_a
// of orthonormal shifted Legendre polynomials, degree i_d < n_ad (n_ad = s
// along a, s + 1 across it), numbered i0 fastest; the volume rule is the
// tensor Gauss rule with n1 points per direction, numbered q0 fastest.  With
// curl(f e_a) = grad f x e_a, component a+1 of chat_i is d_{a+2} f and
// component a+2 is -d_{a+1} f (indices mod 3), so for a pair of components
// (a, b) every entry is a sum of terms
//   sum_q X0(i0,j0,q0) X1(i1,j1,q1) X2(i2,j2,q2) W(q),
//   Xd(i,j,q) = f_i(x_q) g_j(x_q),  f, g in {q_k, q_k'},
// one for M (weight Gm_ab, values only) and four for S (weights
// s_u s_v Gc_uv, u = a+1, a+2, v = b+1, b+2; the derivative taken along the
// direction that the curl component differentiates).  W is the point metric
// of the trilinear map: any pointwise weight factors this way, so curved
// and perturbed cells take the same path as affine ones.  The directions
// are contracted one at a time,
//   T1(q0,q1; i2,j2)       = sum_q2 X2 W,
//   T2(q0; i1,j1,i2,j2)    = sum_q1 X1 T1,
//   G(i0,j0; i1,j1,i2,j2) += sum_q0 X0 T2,
// which costs O(N^2 n1) per pair instead of the O(N^2 n1^3) of a sum over all
// points.  The last contraction is a real GEMM with rows (i0, j0), K = (term,
// q0) and columns (i1, j1, i2, j2), run on f64 MFMA; its row operand X0 does
// not depend on the cell and stays in registers.  A Robin face f adds
// sum_fq v_i v_j Q_ab to both blocks, weighted |z|^2 in G_FF: the same
// three contractions with one point (the face's side) in its normal
// direction.
//
// One workgroup per (cell, pair a >= b); the columns (i2, j2 blocks, j2 <= i2
// for a == b) go in chunks of CC = 16 ctiles columns, and the 16-row tiles x
// 16-column tiles of a chunk are dealt to the four waves (tile tau = w + 4k).
template <int Q1, int CAP>
struct SfShape {
  static constexpr int S = Q1 - 1;                // test degree index s: degrees 0..s-1 along a, 0..s across
  static constexpr int NQ = Q1 * Q1 * Q1;
  static constexpr int KSS = Q1;                  // k-steps of the four curl-curl terms (rows t Q1 + q0)
  static constexpr int KSM = (Q1 + 3) / 4;        // k-steps of the mass term (rows 4 Q1 + q0, zero padded)
  static constexpr int KS = KSS + KSM;
  static constexpr int KR = 4 * KS;               // staged T2 rows
  __host__ __device__ static constexpr int n(int comp, int dir) { return comp == dir ? S : Q1; }
  __host__ __device__ static constexpr int rtiles(int a, int b) { return (n(a, 0) * n(b, 0) + 15) / 16; }
  // column tiles per chunk: at most 16 tiles in all and at most CAP column
  // tiles (the tile shape the autotuner picks)
  __host__ __device__ static constexpr int ctiles(int a, int b) {
    return 16 / rtiles(a, b) < CAP ? 16 / rtiles(a, b) : CAP;
  }
  __host__ __device__ static constexpr int cc(int a, int b) { return 16 * ctiles(a, b); }
  __host__ __device__ static constexpr int nbc(int a, int b) { return cc(a, b) / (n(a, 1) * n(b, 1)); }
  __host__ __device__ static constexpr int ccmax() {
    int m = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b <= a; ++b) m = cc(a, b) > m ? cc(a, b) : m;
    return m;
  }
  __host__ __device__ static constexpr int nbmax() {
    int m = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b <= a; ++b) m = nbc(a, b) > m ? nbc(a, b) : m;
    return m;
  }
  static constexpr int CCP = ccmax();             // T2 row pitch
  // LDS offsets (doubles): 1D tables q_k(x_q), q_k'(x_q) [k][q], q_k(0), q_k(1);
  // volume weights [5][NQ]; Robin face weights [6][Q1^2]; T1 [5][nbmax][Q1^2]; T2 [KR][CCP]
  // row operands X0 [rtiles][KS][64 lanes], of a Robin face [rtiles][KSM][64]
  static constexpr int oV = 0, oD = Q1 * Q1, oSide = 2 * Q1 * Q1, oW = oSide + 2 * Q1, oWf = oW + 5 * NQ,
                       oT1 = oWf + 6 * Q1 * Q1, oT2 = oT1 + 5 * nbmax() * Q1 * Q1, oA = oT2 + KR * CCP,
                       oAf = oA + 4 * KS * 64, total = oAf + 4 * KSM * 64;
  static_assert(total * 8 <= 80 * 1024, "two workgroups per CU");
};

// (i2, j2) of block g: all n_a2 x n_b2 (i2 fastest), or j2 <= i2 row by row when tri
__device__ __forceinline__ void sf_block(int g, bool tri, int na2, int& i2, int& j2) {
  if (!tri) {
    i2 = g % na2;
    j2 = g / na2;
    return;
  }
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= g) ++r;
  i2 = r;
  j2 = g - r * (r + 1) / 2;
}

// 1D factors of volume term t (0..3: curl-curl (u, v) = (a+1+(t>>1), b+1+(t&1)), 4: mass) in direction d
__device__ __forceinline__ void sf_tabs(int t, int a, int b, int d, const double* sV, const double* sD,
                                        const double*& fi, const double*& fj) {
  const bool di = t < 4 && d == (a + 2 - (t >> 1)) % 3;
  const bool dj = t < 4 && d == (b + 2 - (t & 1)) % 3;
  fi = di ? sD : sV;
  fj = dj ? sD : sV;
}

// The (a, b) block of one cell; a and b are compile-time, so that the tile
// counts, the chunk shape and the index splits are constants.
template <int Q1, int CAP, int a, int b>
__device__ __forceinline__ void sf_pair_block(const DevTables& T, const ProbArgs& P, const ChunkArgs& C, int64_t cell,
                                              double* smem) {
  using SH = SfShape<Q1, CAP>;
  constexpr int NQ = SH::NQ, KSS = SH::KSS, KS = SH::KS, CCP = SH::CCP, NBM = SH::nbmax();
  const int64_t gc = C.cell_ids[cell];
  double* sV = smem + SH::oV;
  double* sD = smem + SH::oD;
  double* sSide = smem + SH::oSide;
  double* sW = smem + SH::oW;
  double* sWf = smem + SH::oWf;
  double* sT1 = smem + SH::oT1;
  double* sT2 = smem + SH::oT2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int rmask = 0;   // bit f: face f is a Robin face
  for (int f = 0; f < 6; ++f) rmask |= is_robin(P.face_kind[gc * 6 + f]) ? 1 << f : 0;
  const double* gmet = C.met + cell * met_stride(T);
  for (int e = tid; e < 2 * Q1 * Q1; e += NT) smem[SH::oV + e] = T.sf_tab[e];   // values then derivatives
  for (int e = tid; e < 2 * Q1; e += NT) sSide[e] = T.sf_side[e];
  // weights: s_u s_v Gc_uv of the four curl-curl terms, Gm_ab
  for (int e = tid; e < 4 * NQ; e += NT) {
    const int t = e / NQ, q = e - t * NQ;
    const int u = (a + 1 + (t >> 1)) % 3, v = (b + 1 + (t & 1)) % 3;
    const double sg = ((t >> 1) ^ (t & 1)) ? -1.0 : 1.0;
    sW[e] = sg * gmet[6 * q + sym3(u, v)];
  }
  for (int q = tid; q < NQ; q += NT) sW[4 * NQ + q] = gmet[6 * NQ + 6 * q + sym3(a, b)];
  if (rmask)
    for (int e = tid; e < 6 * Q1 * Q1; e += NT)
      sWf[e] = ((rmask >> (e / (Q1 * Q1))) & 1) ? gmet[12 * NQ + 6 * e + sym3(a, b)] : 0.0;
  // mass-term padding rows of T2 (never written by the chunks)
  for (int e = tid; e < (4 * KS - 5 * Q1) * CCP; e += NT) sT2[5 * Q1 * CCP + e] = 0.0;
  __syncthreads();

  constexpr int na0 = SH::n(a, 0), nb0 = SH::n(b, 0), na1 = SH::n(a, 1), nb1 = SH::n(b, 1), na2 = SH::n(a, 2);
  constexpr int R = na0 * nb0, Rt = SH::rtiles(a, b), ctl = SH::ctiles(a, b), CC = 16 * ctl, Tn = Rt * ctl;
  constexpr int ncb = na1 * nb1, nbc = CC / ncb;
  constexpr bool tri = a == b;
  constexpr int nblk = tri ? na2 * (na2 + 1) / 2 : na2 * SH::n(b, 2);
  // row operands X0 of the tiles, in MFMA lane order: row (i0, j0) = rt 16 + (lane & 15),
  // k = 4 ks + (lane >> 4) (the cell-independent products of the q0 factors)
  double* sA = smem + SH::oA;
  for (int e = tid; e < Rt * KS * 64; e += NT) {
    const int ln = e & 63, ks = (e >> 6) % KS, rt = e / (64 * KS);
    const int row = rt * 16 + (ln & 15), kk = 4 * ks + (ln >> 4);
    const int t = ks < KSS ? kk / Q1 : 4;
    const int q0 = ks < KSS ? kk - t * Q1 : kk - 4 * Q1;
    const int i0 = row % na0, j0 = row / na0;
    const double *fi, *fj;
    sf_tabs(t, a, b, 0, sV, sD, fi, fj);
    sA[e] = row < R && q0 < Q1 ? fi[i0 * Q1 + q0] * fj[j0 * Q1 + q0] : 0.0;
  }
  const double2 eps = make_double2(P.eps[2 * gc], P.eps[2 * gc + 1]);
  const double2 mu = make_double2(P.mu[2 * gc], P.mu[2 * gc + 1]);
  const double om2 = P.omega * P.omega;
  const double cF = om2 * (eps.x * eps.x + eps.y * eps.y) + P.alpha;
  const double cI = om2 * (mu.x * mu.x + mu.y * mu.y) + P.alpha;
  const double* dsc = C.dscale + cell * (int64_t)T.nvp;
  double2* Z = C.Z + cell * T.zstride;
  const int64_t ld = T.ldz;
  // the leading 64 floor(Np / 64) rows and columns of G_FF (the real F block
  // the factorisation works on) go to its compact real copy, not to Z
  const int nfb = (T.Np / TB) * TB;
  double* fr = C.fr + cell * fr_stride(T);
  const int64_t ldf = fr_ld(T);

  for (int g0 = 0; g0 < nblk; g0 += nbc) {
    const int nb = min(nbc, nblk - g0);
    // ---- T1(t, blk; q0, q1) = sum_q2 X2 W_t
    for (int e = tid; e < 5 * nb * Q1 * Q1; e += NT) {
      const int q0 = e % Q1, q1 = (e / Q1) % Q1, r = e / (Q1 * Q1);
      const int blk = r % nb, t = r / nb;
      int i2, j2;
      sf_block(g0 + blk, tri, na2, i2, j2);
      const double *fi, *fj;
      sf_tabs(t, a, b, 2, sV, sD, fi, fj);
      const double* wv = sW + t * NQ + q0 + Q1 * q1;
      double acc = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < Q1; ++q2) acc = fma(fi[i2 * Q1 + q2] * fj[j2 * Q1 + q2], wv[Q1 * Q1 * q2], acc);
      sT1[(t * NBM + blk) * Q1 * Q1 + q1 * Q1 + q0] = acc;
    }
    __syncthreads();
    // ---- T2(t q0; c) = sum_q1 X1 T1, column c = (i1, j1, blk), i1 fastest
    for (int e = tid; e < 5 * CC; e += NT) {
      const int t = e / CC, c = e - t * CC;
      const int blk = c / ncb, cc = c - blk * ncb;
      double out[Q1];
#pragma unroll
      for (int q0 = 0; q0 < Q1; ++q0) out[q0] = 0.0;
      if (blk < nb) {
        const int i1 = cc % na1, j1 = cc / na1;
        const double *fi, *fj;
        sf_tabs(t, a, b, 1, sV, sD, fi, fj);
        const double* t1 = sT1 + (t * NBM + blk) * Q1 * Q1;
#pragma unroll 2
        for (int q1 = 0; q1 < Q1; ++q1) {
          const double x = fi[i1 * Q1 + q1] * fj[j1 * Q1 + q1];
#pragma unroll
          for (int q0 = 0; q0 < Q1; ++q0) out[q0] = fma(x, t1[q1 * Q1 + q0], out[q0]);
        }
      }
      const int row0 = t < 4 ? t * Q1 : 4 * Q1;
#pragma unroll
      for (int q0 = 0; q0 < Q1; ++q0) sT2[(row0 + q0) * CCP + c] = out[q0];
    }
    __syncthreads();
    // ---- G(i0 j0; c) = sum_(t, q0) X0 T2: S (curl-curl rows) and M (mass rows)
    d4 acS[4], acM[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acS[k] = acM[k] = d4{0, 0, 0, 0};
    auto kstep = [&](int ks, d4* acc) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int tau = w + 4 * k;
        if (tau < Tn) {
          const double av = sA[((tau % Rt) * KS + ks) * 64 + lane];
          const double bv = sT2[(4 * ks + (lane >> 4)) * CCP + (tau / Rt) * 16 + (lane & 15)];
          acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[k], 0, 0, 0);
        }
      }
    };
#pragma unroll 2
    for (int ks = 0; ks < KSS; ++ks) kstep(ks, acS);
#pragma unroll
    for (int ks = KSS; ks < KS; ++ks) kstep(ks, acM);
    // G_FF = S + cF M (in acS), G_II = S + cI M (in acM)
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const double sv = acS[k][it], mv = acM[k][it];
        acS[k][it] = fma(cF, mv, sv);
        acM[k][it] = fma(cI, mv, sv);
      }
    // ---- Robin faces: one point (the face's side) in the normal direction
#pragma unroll 1
    for (int f = 0; f < 6; ++f) {
      if (!((rmask >> f) & 1)) continue;
      const int nax = f >> 1;
      const double* side = sSide + (f & 1) * Q1;
      const double z2 = P.zinv[(gc * 6 + f) * 2] * P.zinv[(gc * 6 + f) * 2] +
                        P.zinv[(gc * 6 + f) * 2 + 1] * P.zinv[(gc * 6 + f) * 2 + 1];
      // points and 1D factors per direction (ld: stride of k in the table)
      const int nq0 = nax == 0 ? 1 : Q1, nq1 = nax == 1 ? 1 : Q1, nq2 = nax == 2 ? 1 : Q1;
      const double* f0 = nax == 0 ? side : sV;
      const double* f1 = nax == 1 ? side : sV;
      const double* f2 = nax == 2 ? side : sV;
      const int l0 = nax == 0 ? 1 : Q1, l1 = nax == 1 ? 1 : Q1, l2 = nax == 2 ? 1 : Q1;
      const double* wf = sWf + f * Q1 * Q1;   // face points: tangential axes in increasing order, first fastest
      __syncthreads();   // T1, T2 free
#pragma unroll 1
      for (int e = tid; e < nb * nq0 * nq1; e += NT) {
        const int q0 = e % nq0, q1 = (e / nq0) % nq1, blk = e / (nq0 * nq1);
        int i2, j2;
        sf_block(g0 + blk, tri, na2, i2, j2);
        double acc = 0.0;
#pragma unroll 1
        for (int q2 = 0; q2 < nq2; ++q2)
          acc = fma(f2[i2 * l2 + q2] * f2[j2 * l2 + q2], wf[q0 + nq0 * (q1 + nq1 * q2)], acc);
        sT1[blk * Q1 * Q1 + q1 * nq0 + q0] = acc;
      }
      __syncthreads();
      // (rows nq0 .. 4 KSM of T2 are zero)
#pragma unroll 1
      for (int e = tid; e < 4 * SH::KSM * CC; e += NT) {
        const int q0 = e / CC, c = e - q0 * CC;
        const int blk = c / ncb, cc = c - blk * ncb;
        double acc = 0.0;
        if (blk < nb && q0 < nq0) {
          const int i1 = cc % na1, j1 = cc / na1;
          const double* t1 = sT1 + blk * Q1 * Q1 + q0;
#pragma unroll 1
          for (int q1 = 0; q1 < nq1; ++q1) acc = fma(f1[i1 * l1 + q1] * f1[j1 * l1 + q1], t1[q1 * nq0], acc);
        }
        sT2[q0 * CCP + c] = acc;
      }
      double* sAf = smem + SH::oAf;
#pragma unroll 1
      for (int e = tid; e < Rt * SH::KSM * 64; e += NT) {
        const int ln = e & 63, ks = (e >> 6) % SH::KSM, rt = e / (64 * SH::KSM);
        const int row = rt * 16 + (ln & 15), kk = 4 * ks + (ln >> 4);
        const int i0 = row % na0, j0 = row / na0;
        sAf[e] = row < R && kk < nq0 ? f0[i0 * l0 + kk] * f0[j0 * l0 + kk] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < SH::KSM; ++ks) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int tau = w + 4 * k;
          if (tau < Tn) {
            const double av = sAf[((tau % Rt) * SH::KSM + ks) * 64 + lane];
            const double bv = sT2[(4 * ks + (lane >> 4)) * CCP + (tau / Rt) * 16 + (lane & 15)];
            acS[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(z2 * av, bv, acS[k], 0, 0, 0);
            acM[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acM[k], 0, 0, 0);
          }
        }
      }
    }
    // ---- scaled lower triangles of the (a, b) blocks of D G_FF D and D G_II D
    // (the scale factors are all loaded before the first store: a wait for a
    // load also waits for the stores issued before it)
    double sF[4][4], sI[4][4];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int tau = w + 4 * k;
        if (tau >= Tn) continue;
        const int col = (tau / Rt) * 16 + (lane & 15);
        const int blk = col / ncb, cc = col - blk * ncb;
        if (blk >= nb) continue;
        int i2, j2;
        sf_block(g0 + blk, tri, na2, i2, j2);
        const int ic = a * T.nc + na0 * ((cc % na1) + na1 * i2), jc = b * T.nc + nb0 * ((cc / na1) + nb1 * j2);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int row = (tau % Rt) * 16 + (lane >> 4) + 4 * it;
          if (row >= R) continue;
          const int i = ic + row % na0, j = jc + row / na0;
          if (tri && j > i) continue;
          if (pass == 0) {
            sF[k][it] = dsc[i] * dsc[j];
            sI[k][it] = dsc[T.Np + i] * dsc[T.Np + j];
            continue;
          }
          const double gff = sF[k][it] * acS[k][it];
          if (i < nfb && j < nfb) fr[(int64_t)j * ldf + i] = gff;   // the real F block: its compact copy only
          else Z[(int64_t)j * ld + i] = make_double2(gff, 0.0);
          Z[(int64_t)(T.Np + j) * ld + T.Np + i] = make_double2(sI[k][it] * acM[k][it], 0.0);
        }
      }
  }
}

template <int Q1, int CAP>
__global__ __launch_bounds__(NT, 2) void k_form_SM(DevTables T, ProbArgs P, ChunkArgs C) {
  int64_t cell;
  int pr;
  if (!decode_cell_tile(C.n, 6, cell, pr)) return;
  extern __shared__ double smem[];
  switch (pr) {
    case 0: sf_pair_block<Q1, CAP, 0, 0>(T, P, C, cell, smem); break;
    case 1: sf_pair_block<Q1, CAP, 1, 0>(T, P, C, cell, smem); break;
    case 2: sf_pair_block<Q1, CAP, 1, 1>(T, P, C, cell, smem); break;
    case 3: sf_pair_block<Q1, CAP, 2, 0>(T, P, C, cell, smem); break;
    case 4: sf_pair_block<Q1, CAP, 2, 1>(T, P, C, cell, smem); break;
    default: sf_pair_block<Q1, CAP, 2, 2>(T, P, C, cell, smem); break;
  }
}


// ================================================================ Cholesky
// LDS of the factorisation kernels (aliased phases, two workgroups per CU):
//   diagonal block          Cr, Ci [64][65] (then broadcast slots in Cr)
//   split regrouping        one slab of WSP_BYTES per wave
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kFactorSmem = 2 * 64 * 65 * 8;
constexpr size_t kFblockSmem = 64 * 65 * 8;   // the real F block needs no imaginary parts: three workgroups per CU
static_assert(kFactorSmem <= 80 * 1024, "two factorisation workgroups must fit one CU");

// 1/sqrt(d) for the pivots of the tile factorisation (d > 0 and finite, of
// order one after the diagonal scaling): the hardware estimate refined by two
// Newton steps y <- y + y (1 - d y^2) / 2 (measured: at most 0.99 ulp), then
// a third whose residual 1 - d y^2 is formed exactly (d y split into its
// rounded value and remainder by an fma), which rounds correctly to within
// half an ulp (measured: 0.5).  The pivot enters every column of the factor
// and of the diagonal-block inverses, so its error sets much of the
// factorisation's backward error.  The chain is still shorter than an IEEE
// square root followed by a division.
__device__ __forceinline__ double pivot_rsqrt(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  const double h = d * y, hl = fma(d, y, -h);
  const double e = fma(-hl, y, fma(-h, y, 1.0));
  return fma(0.5 * y, e, y);
}

// Cholesky factorisation of the 64x64 Hermitian tile whose lower part is in
// Cr/Ci[r*65+q], stored for the panel solves of the sweep: the tile L = chol
// is cut into 16x16 blocks; the blocks below the block diagonal hold L itself
// and the four diagonal blocks hold the inverses of L's diagonal blocks
// (lower triangular; zeros above the diagonal of the tile).  A panel X is
// then solved against L^H by block substitution over the four blocks with
// those small inverses.  Multiplying by the inverse of the whole 64x64 factor
// instead loses accuracy by the condition of that factor (measured: about
// five times LAPACK's element-wise error on the trace block of K_e); with
// 16x16 inverses the error is that of substitution.
// Blocked, right-looking over the four 16-column blocks kb, two barriers per
// block:
//   A. every wave factorises the diagonal block D = A[kb][kb] in its own
//      registers by column elimination (the same arithmetic in each wave, so
//      no barrier and no broadcast through LDS; values move between lanes by
//      shuffles) and forms its inverse X = L_kk^{-1}: lane (i, g) = (l & 15,
//      l >> 4) holds row i, columns 4e + g (e = 0..3), of D and of X; column
//      c's step takes L_ic / L_cc = D_ic / d_cc, subtracts it times conj(D_qc)
//      from D_iq and times X_cq from X_iq, and the rows of X are scaled by
//      1 / L_ii at the end.  1/sqrt(d_cc) is pivot_rsqrt;
//   B. wave ib > kb forms the panel block L[ib][kb] = A[ib][kb] X^H on f64
//      MFMA (X's registers are already its B operand) and puts it in LDS;
//   C. wave ib subtracts L[ib][kb] L[jb][kb]^H from A[ib][jb], kb < jb <= ib
//      (f64 MFMA, accumulators started from the LDS block).
// Wave kb writes X into the LDS diagonal block after the first barrier; the
// tile then leaves LDS for `out` (and, REAL, for the real column-major tile
// rout of leading dimension ldr if given) in one coalesced pass.  Returns the
// first failing column + 1 (0 if none), the same value in every thread.
// REAL: the tile is real, Ci is never accessed (it need not exist).
template <bool REAL>
__device__ __forceinline__ int chol_inv_tile(double* Cr, double* Ci, double2* __restrict__ out, int64_t ld,
                                             double* __restrict__ rout = nullptr, int64_t ldr = 0) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int i = lane & 15, g4 = lane >> 4;
  int fail = 0;
  for (int kb = 0; kb < 4; ++kb) {
    const int o = 16 * kb;
    // ---- A: D = L_kk L_kk^H and X = L_kk^{-1}, in every wave
    double dr[4], di[4], xr[4], xi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = 4 * e + g4;
      dr[e] = q <= i ? Cr[(o + i) * 65 + o + q] : 0.0;
      di[e] = (!REAL && q <= i) ? Ci[(o + i) * 65 + o + q] : 0.0;
      xr[e] = q == i ? 1.0 : 0.0;
      xi[e] = 0.0;
    }
    double pinv = 1.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int ce = c >> 2, cg = c & 3;   // column c: element ce of the lanes with g4 == cg
      double dcc = __shfl(dr[ce], c + 16 * cg, 64);
      if (!(dcc > 0.0) || !isfinite(dcc)) {
        if (!fail) fail = o + c + 1;
        dcc = 1.0;
      }
      const double inv = pivot_rsqrt(dcc);
      const double inv2 = inv * inv;
      const double cr = __shfl(dr[ce], i + 16 * cg, 64);
      const double ci = REAL ? 0.0 : __shfl(di[ce], i + 16 * cg, 64);
      const double lr = i > c ? cr * inv2 : 0.0, li = i > c ? ci * inv2 : 0.0;   // L_ic / L_cc
      // every read of this step before any of its updates (column c sits in
      // element ce, which the updates below change)
      double qr[4], qi[4], yr[4], yi[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = 4 * e + g4;
        qr[e] = __shfl(dr[ce], q + 16 * cg, 64);            // D_qc
        qi[e] = REAL ? 0.0 : __shfl(di[ce], q + 16 * cg, 64);
        yr[e] = __shfl(xr[e], c + 16 * g4, 64);             // X_cq (before its scaling)
        yi[e] = REAL ? 0.0 : __shfl(xi[e], c + 16 * g4, 64);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        dr[e] = fma(-lr, qr[e], dr[e]);
        xr[e] = fma(-lr, yr[e], xr[e]);
        if (!REAL) {
          dr[e] = fma(-li, qi[e], dr[e]);
          di[e] = fma(-li, qr[e], di[e]);
          di[e] = fma(lr, qi[e], di[e]);
          xr[e] = fma(li, yi[e], xr[e]);
          xi[e] = fma(-lr, yi[e], xi[e]);
          xi[e] = fma(-li, yr[e], xi[e]);
        }
      }
      if (i == c) pinv = inv;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xr[e] *= pinv;
      xi[e] *= pinv;
    }
    // ---- B: L[w][kb] = A[w][kb] X^H  (re = Ar Xr^T + Ai Xi^T, im = Ai Xr^T - Ar Xi^T)
    if (w > kb) {
      d4 cre = d4{0, 0, 0, 0}, cim = d4{0, 0, 0, 0};
      const int ar0 = (16 * w + (lane & 15)) * 65 + o + (lane >> 4);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const double a_r = Cr[ar0 + 4 * ks];
        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r, xr[ks], cre, 0, 0, 0);
        if (!REAL) {
          const double a_i = Ci[ar0 + 4 * ks];
          cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i, xi[ks], cre, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i, xr[ks], cim, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_r, xi[ks], cim, 0, 0, 0);
        }
      }
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int idx = (16 * w + (lane >> 4) + 4 * it) * 65 + o + (lane & 15);
        Cr[idx] = cre[it];
        if (!REAL) Ci[idx] = cim[it];
      }
    }
    __syncthreads();   // panel blocks of column block kb in LDS; diagonal block kb read by every wave
    if (w == kb) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = (o + i) * 65 + o + 4 * e + g4;
        Cr[idx] = xr[e];
        if (!REAL) Ci[idx] = xi[e];
      }
    }
    // ---- C: A[w][jb] -= L[w][kb] L[jb][kb]^H for kb < jb <= w
    //      (re -= Lr_w Lr_j^T + Li_w Li_j^T, im -= Li_w Lr_j^T - Lr_w Li_j^T)
    if (w > kb) {
      const int aw = (16 * w + (lane & 15)) * 65 + o + (lane >> 4);
      for (int jb = kb + 1; jb <= w; ++jb) {
        const int bj = (16 * jb + (lane & 15)) * 65 + o + (lane >> 4);
        d4 cre, cim = d4{0, 0, 0, 0};
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int idx = (16 * w + (lane >> 4) + 4 * it) * 65 + 16 * jb + (lane & 15);
          cre[it] = Cr[idx];
          if (!REAL) cim[it] = Ci[idx];
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const double wr = Cr[aw + 4 * ks], jr = Cr[bj + 4 * ks];
          cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-wr, jr, cre, 0, 0, 0);
          if (!REAL) {
            const double wi = Ci[aw + 4 * ks], ji = Ci[bj + 4 * ks];
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-wi, ji, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(-wi, jr, cim, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(wr, ji, cim, 0, 0, 0);
          }
        }
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int idx = (16 * w + (lane >> 4) + 4 * it) * 65 + 16 * jb + (lane & 15);
          Cr[idx] = cre[it];
          if (!REAL) Ci[idx] = cim[it];
        }
      }
    }
    __syncthreads();   // trailing blocks updated
  }
  // ---- the tile: L below the block diagonal, the inverses on it, zeros above
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int c = e >> 6, r = e & 63;
    const bool keep = (r >> 4) >= (c >> 4);
    const double vr = keep ? Cr[r * 65 + c] : 0.0;
    if (REAL) {
      if (out) out[(int64_t)c * ld + r] = make_double2(vr, 0.0);
      if (rout) rout[(int64_t)c * ldr + r] = vr;
    } else {
      out[(int64_t)c * ld + r] = make_double2(vr, keep ? Ci[r * 65 + c] : 0.0);
    }
  }
  return fail;
}

// Step 0 diagonal block: A_00 = L L^H, stored for the panel solves (chol_inv_tile).
__global__ __launch_bounds__(NT) void k_chol_diag0(DevTables T, ChunkArgs C) {
  const int64_t cell = blockIdx.x;
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  extern __shared__ double smem[];
  double* Cr = smem;
  double* Ci = Cr + 64 * 65;
  const int64_t ld = T.ldz;
  double2* tile = C.Z + cell * T.zstride;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int q = e >> 6, r = e & 63;
    if (q <= r) {
      const double2 a = tile[(int64_t)q * ld + r];
      Cr[r * 65 + q] = a.x;
      Ci[r * 65 + q] = a.y;
    }
  }
  __syncthreads();
  const int fail = T.Np >= TB ? chol_inv_tile<true>(Cr, Ci, tile, ld) : chol_inv_tile<false>(Cr, Ci, tile, ld);
  if (threadIdx.x == 0 && fail && C.info[gc - C.cell_base] == 0) C.info[gc - C.cell_base] = fail;
}

// ---------------------------------------------------------------- one wave, part of a tile
// Register-direct tile product for one wave, which owns the 16 NV rows
// [16 NV h, 16 NV (h + 1)) of a 64x64 output tile: Q -= conj(B_j) A_i^T with B_j the
// 64-row panel of the tile's columns and A_i the wave's rows, over columns
// [0, K) of the panels.  No LDS and no barriers: every operand goes from
// memory to the MFMA source registers.  Block (u, v) of Q (u: rows from panel
// j, v: rows from the wave's half of panel i) is one 16x16 f64 MFMA
// accumulator; item t of lane l holds Q[16u + (l >> 4) + 4t][16v + (l & 15)].
// With that layout item t is at once the B operand (k = row of Q) of a
// following product  M Q, which is how the triangular epilogue consumes it
// without a transpose.  Two waves per SIMD (256 registers each) hide each
// other's load latency.
template <int NV = 2>
struct WAccT {
  d4 re[4][NV], im[4][NV];
};
using WAcc = WAccT<2>;

// Per-wave LDS slab that regroups the bf16 split planes of a 32 x 16 block of
// W^H into 16-byte column runs: [32 rows][6 planes][16 columns], row pitch
// 208 bytes (16-byte aligned rows; 2-way bank aliasing at most).
constexpr int WSP_PITCH = 208;
constexpr int WSP_BYTES = 32 * WSP_PITCH;
static_assert(4 * WSP_BYTES <= kFactorSmem, "four wave slabs fit the step kernel's LDS");
// A wave's LDS region in the F-column kernel: the running total of its
// two-level sums (32 doubles per lane) during the k-loop, then its split slab.
constexpr int WLDS_BYTES = 32 * 64 * 8;
static_assert(WSP_BYTES <= WLDS_BYTES && 4 * WLDS_BYTES <= kFactorSmem, "four wave regions fit the LDS");

template <int NV = 2>
struct WOpsT {
  double2 a[NV], b[4];
};

// Register buffers of the k-step pipeline (prefetch distance NB - 1): the
// fewer MFMAs a k-step has, the deeper the prefetch; sized to what the
// register file holds next to the accumulators without spilling.
template <int MODE, int NV = 2, int TWO = 0>
struct WPipe {
  // a wave of 16 rows (NV = 1) has half the accumulators, so room for twice the
  // buffers, unless the two-level summation takes that room for its run sums
  static constexpr int NB = (NV == 2 || TWO) ? (MODE == MM_RR ? 4 : 2) : (MODE == MM_RR ? 8 : 4);
  // k-steps per buffer (more than one lets a mode with few MFMAs per k-step
  // keep more work in flight): two for complex x real once the running totals
  // are in LDS (TWO == 2; with them in registers two spilled), else one
  static constexpr int KS = (MODE == MM_CR && TWO == 2) ? 2 : 1;
};

// Operands of one k-step: A from the complex panel Ai (leading dimension
// lda) or, when FRA, from a real matrix, B from the complex panel Bj or, when
// FRB, from a real matrix (the compact copy of the factorised F block,
// leading dimension ldb).
// NTA: the A operand (the wave's own rows, read once per launch) is loaded
// non-temporally, so that it does not push the shared column panel out of L2.
template <int MODE, bool FRB, int NV, bool FRA = false, bool NTA = false>
__device__ __forceinline__ void wave_load(const void* __restrict__ Ai, int64_t lda, const void* __restrict__ Bj,
                                          int64_t ldb, int ks, WOpsT<NV>& o) {
  const int lane = threadIdx.x & 63;
  const int64_t offa = (int64_t)(4 * ks + (lane >> 4)) * lda + (lane & 15);
  typedef double ntd2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (FRA) o.a[v].x = reinterpret_cast<const double*>(Ai)[offa + 16 * v];
    else if (MODE == MM_RR)
      o.a[v].x = NTA ? __builtin_nontemporal_load(reinterpret_cast<const double*>(reinterpret_cast<const double2*>(Ai) + offa + 16 * v))
                     : reinterpret_cast<const double*>(reinterpret_cast<const double2*>(Ai) + offa + 16 * v)[0];
    else if (NTA) {
      const ntd2 t = __builtin_nontemporal_load(reinterpret_cast<const ntd2*>(reinterpret_cast<const double2*>(Ai) + offa + 16 * v));
      o.a[v] = make_double2(t.x, t.y);
    } else o.a[v] = reinterpret_cast<const double2*>(Ai)[offa + 16 * v];
  }
  const int64_t offb = (int64_t)(4 * ks + (lane >> 4)) * ldb + (lane & 15);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (FRB) o.b[u].x = reinterpret_cast<const double*>(Bj)[offb + 16 * u];
    else if (MODE == MM_CC) o.b[u] = reinterpret_cast<const double2*>(Bj)[offb + 16 * u];
    else o.b[u].x = reinterpret_cast<const double*>(reinterpret_cast<const double2*>(Bj) + offb + 16 * u)[0];
  }
}

// The column-panel (B) part of wave_load alone.
template <int MODE, bool FRB, int NV>
__device__ __forceinline__ void wave_load_b(const void* __restrict__ Bj, int64_t ldb, int ks, WOpsT<NV>& o) {
  const int lane = threadIdx.x & 63;
  const int64_t offb = (int64_t)(4 * ks + (lane >> 4)) * ldb + (lane & 15);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (FRB) o.b[u].x = reinterpret_cast<const double*>(Bj)[offb + 16 * u];
    else if (MODE == MM_CC) o.b[u] = reinterpret_cast<const double2*>(Bj)[offb + 16 * u];
    else o.b[u].x = reinterpret_cast<const double*>(reinterpret_cast<const double2*>(Bj) + offb + 16 * u)[0];
  }
}

// re -= br ar + bi ai,  im -= br ai - bi ar   (Q -= conj(b) a)
template <int MODE, int NV>
__device__ __forceinline__ void wave_step(const WOpsT<NV>& o, WAccT<NV>& q) {
  double nbr[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) nbr[u] = -o.b[u].x;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < NV; ++v) q.re[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(nbr[u], o.a[v].x, q.re[u][v], 0, 0, 0);
  if (MODE == MM_RR) return;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < NV; ++v) q.im[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(nbr[u], o.a[v].y, q.im[u][v], 0, 0, 0);
  if (MODE == MM_CR) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double nbi = -o.b[u].y;
#pragma unroll
    for (int v = 0; v < NV; ++v) q.re[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(nbi, o.a[v].y, q.re[u][v], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < NV; ++v) q.im[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.b[u].y, o.a[v].x, q.im[u][v], 0, 0, 0);
}

// The steady-state loop has no branch in its unrolled body (loads past the
// end re-read the last k-step), so the wait before each k-step leaves the
// younger prefetches in flight; the last nks % NB k-steps, already loaded,
// follow the loop.
// TWO: two-level summation.  The products of each run of 16 k-steps (64
// columns) are summed in accumulators of their own, started at zero, and each
// run's sum is then added to q; the rounding errors of a long sum (up to
// thousands of terms at p = 4) then grow with the runs' partial sums instead
// of the running total (measured in an emulation of the sweep: K_e and eta
// three to twenty times closer to the exact solve at p = 4, dp = 2).
// TAIL: the last 64 columns of A are the wave's previous tile of the same
// rows, still in registers (*tail, in the accumulator layout, which for
// k-step t of that tile is exactly the A operand: item t % 4 of block t / 4);
// only the column panel is loaded for them.  The products and their order
// are those of the loads from memory.
// TWO == 2: the running total of the two-level sum in the wave's LDS region
// `tot` (32 NV doubles per lane, item e of lane l at tot[64 e + l]) and the
// run summed in q itself, which frees one accumulator set of registers; the
// additions and their order are those of TWO == 1.
template <int MODE, bool FRB = false, int NV = 2, int TWO = 0, bool FRA = false, bool NTA = false,
          bool TAIL = false>
__device__ __forceinline__ void wave_gemm_t(const void* __restrict__ Ai, int64_t lda, const void* __restrict__ Bj,
                                            int64_t ldb, int K, WAccT<NV>& q, const WAccT<NV>* tail = nullptr,
                                            double* tot = nullptr) {
  constexpr int NB = WPipe<MODE, NV, TWO>::NB, KS = WPipe<MODE, NV, TWO>::KS;
  static_assert(!TWO || 16 % (NB * KS) == 0, "a run of 16 k-steps spans whole pipeline rounds");
  const int nks_all = K / (4 * KS);   // buffers' worth of k-steps (K is a multiple of 64)
  if (nks_all <= 0) return;
  const int nks = TAIL ? nks_all - 16 / KS : nks_all;   // buffers with A from memory
  const int nfull = nks - nks % NB;
  const int lane = threadIdx.x & 63;
  WAccT<NV> qb;                   // the current run's sum (TWO == 1)
  auto tot_at = [&](int part, int u, int v, int t) -> double& {
    return tot[64 * (((part * 4 + u) * NV + v) * 4 + t) + lane];
  };
  auto zero_run = [&]() {
    WAccT<NV>& z = TWO == 2 ? q : qb;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        z.re[u][v] = d4{0, 0, 0, 0};
        z.im[u][v] = d4{0, 0, 0, 0};
      }
  };
  auto fold_run = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (TWO == 2) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            tot_at(0, u, v, t) += q.re[u][v][t];
            if (MODE != MM_RR) tot_at(1, u, v, t) += q.im[u][v][t];
          }
        } else {
          q.re[u][v] += qb.re[u][v];
          if (MODE != MM_RR) q.im[u][v] += qb.im[u][v];
        }
      }
  };
  if (TWO == 2) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          tot_at(0, u, v, t) = q.re[u][v][t];
          if (MODE != MM_RR) tot_at(1, u, v, t) = q.im[u][v][t];
        }
  }
  if (TWO) zero_run();
  WAccT<NV>& acc = TWO == 1 ? qb : q;
  WOpsT<NV> o[NB][KS];
  if (nks > 0) {
#pragma unroll
  for (int s = 0; s < NB - 1; ++s)
#pragma unroll
    for (int u = 0; u < KS; ++u) wave_load<MODE, FRB, NV, FRA, NTA>(Ai, lda, Bj, ldb, min(s, nks - 1) * KS + u, o[s][u]);
  }
  for (int k0 = 0; k0 < nfull; k0 += NB) {
#pragma unroll
    for (int s = 0; s < NB; ++s) {
#pragma unroll
      for (int u = 0; u < KS; ++u)
        wave_load<MODE, FRB, NV, FRA, NTA>(Ai, lda, Bj, ldb, min(k0 + s + NB - 1, nks - 1) * KS + u,
                                      o[(s + NB - 1) % NB][u]);
      __builtin_amdgcn_sched_barrier(0);   // keep each prefetch in its slot (bounded live ranges)
#pragma unroll
      for (int u = 0; u < KS; ++u) wave_step<MODE, NV>(o[s][u], acc);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (TWO && (((k0 + NB) * KS) & 15) == 0) {
      fold_run();
      zero_run();
    }
  }
#pragma unroll
  for (int s = 0; s < NB - 1; ++s)
    if (s < nks - nfull) {
#pragma unroll
      for (int u = 0; u < KS; ++u) wave_step<MODE, NV>(o[s][u], acc);
    }
  if (TWO && ((nks * KS) & 15) != 0) fold_run();
  if (TAIL) {
    // the previous tile's 16 k-steps: one run of the two-level sum (nks KS is
    // a multiple of 16, so the run boundaries are those of the full loop)
    WOpsT<NV> ob[2];
    wave_load_b<MODE, FRB, NV>(Bj, ldb, nks * KS, ob[0]);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      if (t + 1 < 16) wave_load_b<MODE, FRB, NV>(Bj, ldb, nks * KS + t + 1, ob[(t + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        ob[t & 1].a[v] = make_double2(tail->re[t >> 2][v][t & 3], MODE == MM_RR ? 0.0 : tail->im[t >> 2][v][t & 3]);
      wave_step<MODE, NV>(ob[t & 1], acc);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (TWO) fold_run();
  }
  if (TWO == 2) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          q.re[u][v][t] = tot_at(0, u, v, t);
          q.im[u][v][t] = MODE != MM_RR ? tot_at(1, u, v, t) : 0.0;
        }
  }
}

// Rows [16 NV h, 16 NV (h + 1)) of the tile (i, j) of step j, one wave:
// X = A_ij - L_i,<j L_j,<j^H (the sum over columns from k0, the caller's bound
// below which the rows are zero), then L_ij = X L_jj^{-H} by block
// substitution over the four 16x16 blocks of the diagonal tile (chol_inv_tile's
// storage), computed transposed.  The waves of a tile are independent: row r
// of L_ij needs row r of X only.
// The tiles of the sweep run on waves of 16 RNV rows, 64 / (16 RNV) waves per
// tile and 4 / that tiles per workgroup.  Waves of 16 rows leave room for the
// run sums of the two-level summation next to the accumulators (with 32-row
// waves the accumulators alone fill half the registers); without it, 16- and
// 32-row waves were measured equally fast on the WR340 workload.
constexpr int RNV = 1;                    // 16-row blocks per wave of a regular tile
constexpr int RWPT = TB / (16 * RNV);   // waves per regular tile
static_assert(RWPT * 16 * RNV == TB, "the waves of a regular tile cover its rows");
constexpr int RTPW = 4 / RWPT;            // regular tiles per workgroup

// Use of the compact real copy of the F block by a tile: none, its operands
// (panel j and the stored diagonal tile j) from it, the tile's real output
// written to it too, or (a tile of the F block itself) every operand from it
// and the output to it only.
enum { FR_NONE = 0, FR_READ = 1, FR_WRITE = 2, FR_FB = 3 };

// keep (TAIL): in, the wave's tile (i, j - 1) as left by the previous call
// (used for the last 64 columns of the sum when j > 0); out, this tile.
template <int MODE, int FR = FR_NONE, int NV = 2, int TWO = 0, bool NTA = false, bool TAIL = false>
__device__ void wave_tile(const DevTables& T, const ChunkArgs& C, double2* __restrict__ Z, int64_t cell, int i, int j,
                          int h, unsigned char* slab, int k0 = 0, WAccT<NV>* keep = nullptr) {
  constexpr int RW = 16 * NV;   // rows of the wave: [RW h, RW h + RW) of the tile
  // ld and lane pass through empty asm so that, in a loop over tiles, the
  // compiler recomputes the lane addresses per tile instead of keeping them
  // all live across the loop (which spills)
  int64_t ld = T.ldz;
  __asm__ volatile("" : "+s"(ld));
  int lane = threadIdx.x & 63;
  __asm__ volatile("" : "+v"(lane));
  double2* tile = Z + (int64_t)(j * TB) * ld + i * TB + RW * h;   // rows of A_ij in, of L_ij out
  // panel j and the diagonal tile j: from Z, or from the real copy of the F block
  constexpr bool FRB = FR == FR_READ || FR == FR_FB;
  const int64_t ldf = fr_ld(T);
  double* Fr = FR != FR_NONE ? C.fr + cell * fr_stride(T) : nullptr;
  // the accumulators start as A_ij^T, so that they end as X^T (a tile of the
  // F block starts from the real copy, where its Gram block is)
  WAccT<NV> q;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = 16 * v + (lane & 15), c = 16 * u + 4 * t + (lane >> 4);
        if (FR == FR_FB) {
          q.re[u][v][t] = Fr[(int64_t)(j * TB + c) * ldf + i * TB + RW * h + r];
          q.im[u][v][t] = 0.0;
        } else {
          const double2 a = tile[(int64_t)c * ld + r];
          q.re[u][v][t] = a.x;
          q.im[u][v][t] = MODE == MM_RR ? 0.0 : a.y;
        }
      }
  __builtin_amdgcn_sched_barrier(0);
  if (FR == FR_FB)
    wave_gemm_t<MODE, true, NV, TWO, true>(Fr + (int64_t)k0 * ldf + i * TB + RW * h, ldf,
                                           Fr + (int64_t)k0 * ldf + j * TB, ldf, j * TB - k0, q);
  else if (FRB && TAIL)
    wave_gemm_t<MODE, true, NV, TWO, false, false, true>(Z + (int64_t)k0 * ld + i * TB + RW * h, ld,
                                                         Fr + (int64_t)k0 * ldf + j * TB, ldf, j * TB - k0, q, keep,
                                                         TWO == 2 ? reinterpret_cast<double*>(slab) : nullptr);
  else if (FRB)
    wave_gemm_t<MODE, true, NV, TWO>(Z + (int64_t)k0 * ld + i * TB + RW * h, ld, Fr + (int64_t)k0 * ldf + j * TB,
                                     ldf, j * TB - k0, q);
  else
    wave_gemm_t<MODE, false, NV, TWO, false, NTA>(Z + (int64_t)k0 * ld + i * TB + RW * h, ld,
                                                  Z + (int64_t)k0 * ld + j * TB, ld, j * TB - k0, q);
  __builtin_amdgcn_sched_barrier(0);
  if (TAIL) {
    // the previous tile of these rows came from registers (keep); its stores,
    // read from memory by the tile after this one, are made visible here,
    // long after they were issued, instead of right after them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  const double2* tL = Z + (int64_t)(j * TB) * ld + j * TB;   // diagonal tile j (chol_inv_tile's storage)
  const double* tLr = FRB ? Fr + (int64_t)(j * TB) * ldf + j * TB : nullptr;
  const int nvb = T.nvp / TB;
  const bool wsplit = C.split && i >= nvb;
  const bool last_w = j + 1 == nvb;
  uint16_t* wp = wsplit ? C.wsplit + cell * split_elems(T) : nullptr;
  const int nkc = T.nvp / 32;
  // Block forward substitution conj(L_jj) Y = Q over the four 16-row blocks
  // (Y = L_ij^T, Q = X^T; chol_inv_tile's storage: L_jj below the block
  // diagonal, the inverses Dinv of its diagonal blocks on it):
  //   Q[mb] -= sum_{kb < mb} conj(L_jj[mb][kb]) Y[kb],  Y[mb] = conj(Dinv[mb]) Q[mb],
  // where Y[mb] replaces Q[mb] in the accumulators (it is the B operand of the
  // later updates, item t of lane l being row 16 mb + 4 t + (l >> 4)).
  // A operand of block (m, k) at k-step t: element [16 m + (l & 15)][16 k + 4 t + (l >> 4)].
#define DPG_DIAG_OP(m, k, t)                                                                              \
  (FRB ? make_double2(tLr[(int64_t)(16 * (k) + 4 * (t) + (lane >> 4)) * ldf + 16 * (m) + (lane & 15)], 0.0)  \
       : tL[(int64_t)(16 * (k) + 4 * (t) + (lane >> 4)) * ld + 16 * (m) + (lane & 15)])
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    __builtin_amdgcn_sched_barrier(0);   // one block at a time (bounded live ranges)
    // Q[mb] -= sum_{kb < mb} conj(L_jj[mb][kb]) Y[kb]
#pragma unroll
    for (int kb = 0; kb < mb; ++kb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 L = DPG_DIAG_OP(mb, kb, t);
#pragma unroll
        for (int nb = 0; nb < NV; ++nb) {
          q.re[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-L.x, q.re[kb][nb][t], q.re[mb][nb], 0, 0, 0);
          if (MODE != MM_RR)
            q.im[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-L.x, q.im[kb][nb][t], q.im[mb][nb], 0, 0, 0);
          if (MODE == MM_CC) {
            q.re[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-L.y, q.im[kb][nb][t], q.re[mb][nb], 0, 0, 0);
            q.im[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(L.y, q.re[kb][nb][t], q.im[mb][nb], 0, 0, 0);
          }
        }
      }
    // Y[mb] = conj(Dinv[mb]) Q[mb]
    d4 yr[NV], yi[NV];
#pragma unroll
    for (int nb = 0; nb < NV; ++nb) {
      yr[nb] = d4{0, 0, 0, 0};
      yi[nb] = d4{0, 0, 0, 0};
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double2 L = DPG_DIAG_OP(mb, mb, t);
#pragma unroll
      for (int nb = 0; nb < NV; ++nb) {
        yr[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(L.x, q.re[mb][nb][t], yr[nb], 0, 0, 0);
        if (MODE != MM_RR) yi[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(L.x, q.im[mb][nb][t], yi[nb], 0, 0, 0);
        if (MODE == MM_CC) {
          yr[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(L.y, q.im[mb][nb][t], yr[nb], 0, 0, 0);
          yi[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-L.y, q.re[mb][nb][t], yi[nb], 0, 0, 0);
        }
      }
    }
    // Y[mb] replaces Q[mb]: the B operand of the later blocks' updates
#pragma unroll
    for (int nb = 0; nb < NV; ++nb) {
      q.re[mb][nb] = yr[nb];
      if (MODE != MM_RR) q.im[mb][nb] = yi[nb];
    }
  }
  // The stores of L_ij (and of its bf16 planes) follow the substitution: on
  // this hardware a wait for a load also waits for the stores issued before
  // it, so stores between the blocks would hold up the loads of the next
  // block's diagonal-tile operands.
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    __builtin_amdgcn_sched_barrier(0);
    // item t of block (mb, nb): L_ij[row RW h + 16 nb + (l & 15)][column 16 mb + 4 t + (l >> 4)]
#pragma unroll
    for (int nb = 0; nb < NV; ++nb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = 16 * nb + (lane & 15), c = 16 * mb + 4 * t + (lane >> 4);
        const double vr = q.re[mb][nb][t], vi = MODE == MM_RR ? 0.0 : q.im[mb][nb][t];
        // in the split path the last column block of W^H is read only through its
        // bf16 planes, except the residual row (eta is formed from it in FP64)
        const bool store_l = !(wsplit && last_w) || i * TB + RW * h + r == T.nvp + T.k + 1;
        if (store_l && FR != FR_FB) tile[(int64_t)c * ld + r] = make_double2(vr, vi);
        if (FR == FR_WRITE || FR == FR_FB) Fr[(int64_t)(j * TB + c) * ldf + i * TB + RW * h + r] = vr;
        if (wsplit) {
          // three-term bf16 splits of re and im into the wave's LDS slab
          // [RW rows][6 planes][16 columns] (row pitch WSP_PITCH bytes)
          uint16_t* sl = reinterpret_cast<uint16_t*>(slab + r * WSP_PITCH) + 4 * t + (lane >> 4);
          uint32_t hp[3];
          split3_bf16_pair(vr, vi, hp);
          sl[0] = (uint16_t)hp[0];
          sl[16] = (uint16_t)hp[1];
          sl[32] = (uint16_t)hp[2];
          sl[48] = (uint16_t)(hp[0] >> 16);
          sl[64] = (uint16_t)(hp[1] >> 16);
          sl[80] = (uint16_t)(hp[2] >> 16);
        }
      }
    if (wsplit) {
      // W^H block (i, j) in the split layout [row][k / 32][plane][k % 32]
      // (planes re0, re1, re2, im0, im1, im2): each lane stores 16-byte runs
      // of 8 columns, gathered from the slab written above by the same wave.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int e = 0; e < 3 * NV; ++e) {
        const int id = e * 64 + lane;            // (row, plane, half) of RW x 6 x 2
        const int r = id / 12, pl = (id % 12) >> 1, hf = id & 1;
        const uint4 v = *reinterpret_cast<const uint4*>(slab + r * WSP_PITCH + pl * 32 + hf * 16);
        const int kk = j * TB + 16 * mb + 8 * hf;
        const int64_t o = ((int64_t)((i - nvb) * TB + RW * h + r) * nkc + kk / 32) * 192 + pl * 32 + (kk % 32);
        *reinterpret_cast<uint4*>(wp + o) = v;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if (TAIL) *keep = q;
}

// Rows [RW h, RW h + RW) (RW = 16 NV) of a diagonal block update, one wave:
//   S = S0 - P_h P^H ,  P the 64-row panel (columns [0, K) at P), P_h its rows [RW h, RW h + RW),
// with S0 the column-major tile S0g (FROM_TILE) or the LDS block
// Sr/Si[r*65 + c] itself; the whole RW x 64 result is written to
// Sr/Si[r*65 + c] (only its lower part is meaningful).  TWO: two-level
// summation (wave_gemm_t).  PREAL: P is a real matrix (the compact copy of
// the F block) with leading dimension ldp; S0REAL: so is S0g (the real tile
// at S0g, leading dimension ldp).
template <int MODE, bool FROM_TILE, int NV = 2, bool TWO = false, bool PREAL = false, bool S0REAL = false>
__device__ __forceinline__ void diag_update(const double2* __restrict__ S0g, const void* __restrict__ P, int64_t ld,
                                            int K, int h, double* Sr, double* Si, int64_t ldp = 0) {
  constexpr int RW = 16 * NV;
  int lane = threadIdx.x & 63;
  __asm__ volatile("" : "+v"(lane));   // not hoisted out of a caller's loop (as in wave_tile)
  __asm__ volatile("" : "+s"(ld));
  WAccT<NV> q;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = RW * h + 16 * v + (lane & 15), c = 16 * u + 4 * t + (lane >> 4);
        if (FROM_TILE && S0REAL) {
          q.re[u][v][t] = reinterpret_cast<const double*>(S0g)[(int64_t)c * ldp + r];
          q.im[u][v][t] = 0.0;
        } else if (FROM_TILE) {
          const double2 a = S0g[(int64_t)c * ld + r];
          q.re[u][v][t] = a.x;
          q.im[u][v][t] = MODE == MM_RR ? 0.0 : a.y;
        } else {
          q.re[u][v][t] = Sr[r * 65 + c];
          q.im[u][v][t] = MODE == MM_RR ? 0.0 : Si[r * 65 + c];
        }
      }
  if (PREAL)
    wave_gemm_t<MODE, true, NV, TWO, true>(reinterpret_cast<const double*>(P) + RW * h, ldp, P, ldp, K, q);
  else
    wave_gemm_t<MODE, false, NV, TWO>(reinterpret_cast<const double2*>(P) + RW * h, ld, P, ld, K, q);
  // item t of block (u, v): S[row RW h + 16v + (l & 15)][column 16u + 4t + (l >> 4)]
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = RW * h + 16 * v + (lane & 15), c = 16 * u + 4 * t + (lane >> 4);
        Sr[r * 65 + c] = q.re[u][v][t];
        if (MODE != MM_RR) Si[r * 65 + c] = q.im[u][v][t];   // a real block has no Si
      }
}

// Step j of the left-looking factorisation over the row tiles i > j:
//   L_ij = (A_ij - sum_{m<j} L_im L_jm^H) L_jj^{-H} ,
// for the columns after the real F block (all of them when there is none),
// where every tile is complex.  Tile i = j+1 (while it is a test tile) is
// the lookahead tile: its workgroup also forms A_ii - sum_{m<=j} L_im L_im^H
// and factorises it (chol_inv_tile) for step j+1, so no separate launch
// factors diagonal blocks.  Every tile is four 16-row waves (wave_tile), one
// tile per workgroup; every long sum is two-level.
__global__ __launch_bounds__(NT, 2) void k_chol_step(DevTables T, ChunkArgs C, int j) {
  const int nrb = T.nrows / TB, nvb = T.nvp / TB;
  const bool la = j + 1 < nvb;
  const int nreg = nrb - j - 1 - (la ? 1 : 0);   // regular tiles
  // Workgroup ids [0, n8) carry the lookahead tile of every cell and are
  // dispatched first, spread over all CUs (cell c on XCD c % 8).  The regular
  // tiles follow: per XCD x the (cell, tile) pairs of its cells c = 8 m + x
  // form one list in (m, tile) order, RTPW per workgroup.
  const int64_t n8 = la ? (C.n + 7) / 8 * 8 : 0;
  if ((int64_t)blockIdx.x >= n8) {
    const int64_t w = (int64_t)blockIdx.x - n8;
    const int wave = (int)(threadIdx.x >> 6);
    const int64_t item = (w >> 3) * RTPW + wave / RWPT;
    const int h = wave % RWPT;
    const int64_t m = item / nreg;
    const int t = (int)(item - m * nreg);
    const int64_t cell = m * 8 + (w & 7);
    if (cell >= C.n) return;   // whole waves: no barrier follows on this path
    const int i = j + 1 + (la ? 1 : 0) + t;
    double2* Z = C.Z + cell * T.zstride;
    extern __shared__ double smem[];
    unsigned char* slab = reinterpret_cast<unsigned char*>(smem) + wave * WSP_BYTES;
    // rows that are zero in the F columns stay zero there (k_chol_fpanel leaves them), so their sum starts after
    const int r0 = i * TB + 16 * RNV * h;
    const int k0 = frows_class(T, r0, 16 * RNV) == FROWS_ZERO ? (T.Np / TB) * TB : 0;
    wave_tile<MM_CC, FR_NONE, RNV, true, true>(T, C, Z, cell, i, j, h, slab, k0);
    return;
  }
  // ---- lookahead workgroup: tile (i, j), i = j + 1, on the four waves (16
  // rows each); then the four waves form A_ii - sum_{m<=j} L_im L_im^H in LDS
  // (16 rows each) and factorise it (Cholesky + diagonal-block inverses).
  // Both long sums are two-level.
  const int64_t cell = blockIdx.x;
  if (cell >= C.n) return;
  const int i = j + 1;
  const int64_t ld = T.ldz;
  const int wave = (int)(threadIdx.x >> 6);
  double2* Z = C.Z + cell * T.zstride;
  extern __shared__ double smem[];
  double* Cr = smem;
  double* Ci = Cr + 64 * 65;
  double2* tileD = Z + (int64_t)(i * TB) * ld + i * TB;
  wave_tile<MM_CC, FR_NONE, 1, true>(T, C, Z, cell, i, j, wave, nullptr);
  __syncthreads();   // L_ij stored (workgroup scope)
  diag_update<MM_CC, true, 1, true>(tileD, Z + i * TB, ld, (j + 1) * TB, wave, Cr, Ci);
  __syncthreads();
  const int fail = chol_inv_tile<false>(Cr, Ci, tileD, ld);
  const int64_t gc = C.cell_ids[cell];
  if (threadIdx.x == 0 && fail && C.info[gc - C.cell_base] == 0) C.info[gc - C.cell_base] = i * TB + fail;
}

// Factorisation of the real F block (row and column tiles < nF) of every
// cell in one launch, one workgroup per cell:
//   L_00 = chol(A_00);  for j = 0 .. nF-2:
//     L_ij = (A_ij - sum_{m<j} L_im L_jm^T) L_jj^{-T}   for j < i < nF
//            (one tile at a time on the four 16-row waves),
//     L_{j+1,j+1} = chol(A_{j+1,j+1} - sum_{m<=j} L_{j+1,m} L_{j+1,m}^T)
// (diagonal tiles in chol_inv_tile's storage; two-level sums).
// The block is small, so its cost is the latency of the chain, which one
// workgroup walks without a launch (and a pass over all cells) per step.
__global__ __launch_bounds__(NT, 3) void k_chol_fblock(DevTables T, ChunkArgs C, int nF) {
  const int64_t cell = blockIdx.x;
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  const int64_t ld = T.ldz;
  const int wave = (int)(threadIdx.x >> 6);
  double2* Z = C.Z + cell * T.zstride;
  extern __shared__ double smem[];
  double* Cr = smem;
  double* Ci = Cr + 64 * 65;
  // the block lives only in its compact real copy: the formation writes the
  // Gram block there, and the factorisation overwrites it in place (L_ij below
  // the diagonal, the diagonal tiles as stored), the operands of its own later
  // tiles and of the F-column launch.
  double* fr = C.fr + cell * fr_stride(T);
  const int64_t ldf = fr_ld(T);
  int fail = 0;
  for (int j = 0;; ++j) {
    // diagonal block j, updated by the columns before it, into LDS
    const double* tileD = fr + (int64_t)(j * TB) * ldf + j * TB;
    if (j == 0) {
      for (int e = threadIdx.x; e < 64 * 64; e += NT) {
        const int q = e >> 6, r = e & 63;
        if (q <= r) Cr[r * 65 + q] = tileD[(int64_t)q * ldf + r];
      }
    } else {
      diag_update<MM_RR, true, 1, true, true, true>(reinterpret_cast<const double2*>(tileD), fr + j * TB, ld, j * TB,
                                                    wave, Cr, Ci, ldf);
    }
    __syncthreads();
    const int f = chol_inv_tile<true>(Cr, Ci, nullptr, 0, fr + (int64_t)(j * TB) * ldf + j * TB, ldf);
    if (f && !fail) fail = j * TB + f;
    if (j + 1 == nF) break;
    __syncthreads();   // diagonal tile j stored (workgroup scope); LDS free
    for (int i = j + 1; i < nF; ++i) wave_tile<MM_RR, FR_FB, 1, true>(T, C, Z, cell, i, j, wave, nullptr);
    __syncthreads();   // column block j stored
  }

  if (threadIdx.x == 0 && fail && C.info[gc - C.cell_base] == 0) C.info[gc - C.cell_base] = fail;
}

// The real F columns of all remaining rows in one launch.  Once the F block
// (row and column tiles < nF, all real) is factorised, the rows i >= nF need
// nothing else for their F columns: each 16-row wave walks its rows through
// j = 0 .. nF-1,
//   L_ij = (A_ij - sum_{m<j} L_im L_jm^T) L_jj^{-T} ,
// reading back the row panel L_i,<j it has written at the earlier j (the
// last of its tiles, L_i,j-1, straight from its registers), instead of every
// step re-reading it in a launch of its own.  Row tile nF has a workgroup of
// its own per cell: its four waves walk it, then form A_ii - sum_{m<nF}
// L_im L_im^H in LDS and factorise it for the step nF.  Per XCD the cells
// come in order, each as that workgroup followed by those of its other row
// tiles, so that the long row-nF workgroups run beside the others instead
// of all at the start.  Every sum is two-level (the running totals of the
// other row tiles in LDS, which frees the registers of the kept tile).
__global__ __launch_bounds__(NT, 2) void k_chol_fpanel(DevTables T, ChunkArgs C, int nF) {
  const int nrb = T.nrows / TB;
  const int nreg = nrb - nF - 1;   // row tiles after nF, RTPW per workgroup
  const int64_t n8 = (C.n + 7) / 8 * 8;
  const int wave = (int)(threadIdx.x >> 6);
  extern __shared__ double smem[];
  static_assert(RTPW == 1, "one row tile per workgroup");
  // per XCD x its cells c = 8 m + x in order, each as its row-nF workgroup
  // followed by its regular row tiles
  const int64_t w = blockIdx.x;
  const int64_t slot = w >> 3;
  const int64_t m = slot / (1 + nreg);
  const int tt = (int)(slot - m * (1 + nreg));
  if (tt > 0) {
    const int h = wave % RWPT;
    const int t = tt - 1;
    const int64_t cell = m * 8 + (w & 7);
    if (cell >= C.n) return;   // whole waves: no barrier on this path
    const int i = nF + 1 + t;
    constexpr int RW = 16 * RNV;
    double2* Z = C.Z + cell * T.zstride;
    unsigned char* slab = reinterpret_cast<unsigned char*>(smem) + wave * WLDS_BYTES;
    const int cls = frows_class(T, i * TB + RW * h, RW);
    if (cls == FROWS_ZERO) {
      // L_i,F = 0 (A_i,F = 0, already so in the workspace); only the bf16
      // planes of these W rows need their zeros for the F columns, and only
      // if the HERK reads them (it skips the F columns of a block of W that
      // is zero there)
      const int wblk = i - T.nvp / TB;
      if (C.split && herk_k0(T, wblk, wblk) == 0) {
        const int nkc = T.nvp / 32;
        uint16_t* wp = C.wsplit + cell * split_elems(T) + (int64_t)((i - T.nvp / TB) * TB + RW * h) * nkc * 192;
        const int per_row = 2 * nF * 192 / 8;   // 16-byte runs of the F columns in one row
        for (int e = (int)(threadIdx.x & 63); e < RW * per_row; e += 64) {
          const int rr = e / per_row, o = e - rr * per_row;
          *reinterpret_cast<uint4*>(wp + (int64_t)rr * nkc * 192 + 8 * o) = make_uint4(0u, 0u, 0u, 0u);
        }
      }
      return;
    }
    WAccT<RNV> prev;   // this wave's tile (i, j - 1): the last 64 columns of the next sum
    for (int j = 0; j < nF; ++j) {
      // L_ij (stored by all lanes) feeds the loads of step j + 2 (step j + 1
      // takes it from registers): wave_tile makes it visible after the k-loop
      // of step j + 1
      if (cls == FROWS_REAL) wave_tile<MM_RR, FR_READ, RNV, 2, false, true>(T, C, Z, cell, i, j, h, slab, 0, &prev);
      else wave_tile<MM_CR, FR_READ, RNV, 2, false, true>(T, C, Z, cell, i, j, h, slab, 0, &prev);
    }
    return;
  }
  const int64_t cell = m * 8 + (w & 7);
  if (cell >= C.n) return;   // the whole workgroup
  const int i = nF;
  const int64_t ld = T.ldz;
  double2* Z = C.Z + cell * T.zstride;
  double* Cr = smem;
  double* Ci = Cr + 64 * 65;
  double2* tileD = Z + (int64_t)(i * TB) * ld + i * TB;
  for (int j = 0; j < nF; ++j) {
    wave_tile<MM_CR, FR_READ, 1, true>(T, C, Z, cell, i, j, wave, nullptr);
    // L_ij (the wave's own rows) feeds the loads of step j + 1
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  __syncthreads();   // row tile nF stored (workgroup scope)
  diag_update<MM_CC, true, 1, true>(tileD, Z + i * TB, ld, nF * TB, wave, Cr, Ci);
  __syncthreads();
  const int fail = chol_inv_tile<false>(Cr, Ci, tileD, ld);
  const int64_t gc = C.cell_ids[cell];
  if (threadIdx.x == 0 && fail && C.info[gc - C.cell_base] == 0) C.info[gc - C.cell_base] = i * TB + fail;
}

// ================================================================ K_aug = W^H W
__global__ __launch_bounds__(NT, 2) void k_herk(DevTables T, ChunkArgs C) {
  const int kb = T.kp / TB;
  const int ntiles = kb * (kb + 1) / 2;
  int64_t cell;
  int tile;
  if (!decode_cell_tile(C.n, ntiles, cell, tile)) return;
  int a = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= tile) ++a;
  while (a * (a + 1) / 2 > tile) --a;
  const int b = tile - a * (a + 1) / 2;
  const int64_t gc = C.cell_ids[cell];
  extern __shared__ double smem[];
  Stage* st = reinterpret_cast<Stage*>(smem);
  const int64_t ld = T.ldz;
  const double2* Z = C.Z + cell * T.zstride;
  Acc acc;
  acc_zero(acc);
  const int k0 = herk_k0(T, a, b);
  gemm_abh(Z + (int64_t)k0 * ld + T.nvp + a * TB, Z + (int64_t)k0 * ld + T.nvp + b * TB, ld, T.nvp - k0, st, acc);
  const int k = T.k;
  double2* K = C.K + (C.K_off[gc] - C.K_base);
  double2* L = C.l + (C.v_off[gc] - C.v_base);
  acc_for_each(acc, [&](int r, int c, double vr, double vi) {
    const int al = a * TB + r, be = b * TB + c;
    if (al < k && be < k) {
      if (a == b && be > al) return;
      K[(int64_t)be * k + al] = make_double2(vr, vi);
      if (al != be) K[(int64_t)al * k + be] = make_double2(vr, -vi);
    } else if (al == k && be < k) {
      L[be] = make_double2(vr, -vi);
    } else if (al == k + 1 && be == k + 1) {
      C.eta[gc - C.cell_base] = sqrt(fmax(vr, 0.0));
    }
  });
}

// ================================================================ split-precision K_aug
// K_aug = W^H W from the three-term bf16 splits of W^H on bf16 MFMA
// (v_mfma_f32_16x16x32_bf16): for each real product X Y^T the terms
// X_s Y_t with s + t <= 2 are kept (six products, ~24-bit operands); the
// FP32 accumulators are folded into FP64 after every 32 columns.  eta is not
// taken from here (FP64 reduction in k_eta).
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int SKC = 32;              // k per stage

// Staged planes: per row the four 16-byte chunks of its 32 k, chunk c at
// position c ^ swz(row).  Reads (one chunk of 16 consecutive rows per lane
// group) and stores (the four chunks of consecutive rows) then touch distinct
// banks in every cycle with 32 as with 64 four-byte LDS banks, as 128-bit
// accesses.
struct SplitStage {
  uint4 A[6][64 * 4];
  uint4 B[6][64 * 4];
};
__device__ __forceinline__ int swz(int row) { return ((row >> 1) ^ (row >> 3)) & 3; }

__device__ inline bf8 lds_frag(const uint4* plane, int row, int kq) {
  return __builtin_bit_cast(bf8, plane[row * 4 + (kq ^ swz(row))]);
}

__device__ inline bf8 neg_frag(bf8 a) {
  uint4 v = __builtin_bit_cast(uint4, a);
  v.x ^= 0x80008000u;
  v.y ^= 0x80008000u;
  v.z ^= 0x80008000u;
  v.w ^= 0x80008000u;
  return __builtin_bit_cast(bf8, v);
}

__global__ __launch_bounds__(NT, 2) void k_herk_split(DevTables T, ChunkArgs C) {
  const int kb = T.kp / TB;
  const int ntiles = kb * (kb + 1) / 2;
  int64_t cell;
  int tile;
  if (!decode_cell_tile(C.n, ntiles, cell, tile)) return;
  int a = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= tile) ++a;
  while (a * (a + 1) / 2 > tile) --a;
  const int b = tile - a * (a + 1) / 2;
  const int64_t gc = C.cell_ids[cell];
  extern __shared__ double smem[];
  SplitStage* ss = reinterpret_cast<SplitStage*>(smem);
  const uint16_t* wp = C.wsplit + cell * split_elems(T);
  const int nkc = T.nvp / 32;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w & 1, wc = w >> 1;
  // staging map: thread -> (row, 8-column chunk)
  const int srow = threadIdx.x >> 2, skq = threadIdx.x & 3;
  const uint16_t* pa = wp + (int64_t)(a * TB + srow) * nkc * 192 + skq * 8;
  const uint16_t* pb = wp + (int64_t)(b * TB + srow) * nkc * 192 + skq * 8;
  // prefetch registers (named individually: arrays of these were kept in scratch)
  uint4 ra0, ra1, ra2, ra3, ra4, ra5, rb0, rb1, rb2, rb3, rb4, rb5;
#define DPG_SPLIT_GLOAD(k0)                                                      \
  do {                                                                           \
    ra0 = *reinterpret_cast<const uint4*>(pa + (k0) * 6 + 0);                \
    ra1 = *reinterpret_cast<const uint4*>(pa + (k0) * 6 + 32);                \
    ra2 = *reinterpret_cast<const uint4*>(pa + (k0) * 6 + 64);                \
    ra3 = *reinterpret_cast<const uint4*>(pa + (k0) * 6 + 96);                \
    ra4 = *reinterpret_cast<const uint4*>(pa + (k0) * 6 + 128);                \
    ra5 = *reinterpret_cast<const uint4*>(pa + (k0) * 6 + 160);                \
    rb0 = *reinterpret_cast<const uint4*>(pb + (k0) * 6 + 0);                \
    rb1 = *reinterpret_cast<const uint4*>(pb + (k0) * 6 + 32);                \
    rb2 = *reinterpret_cast<const uint4*>(pb + (k0) * 6 + 64);                \
    rb3 = *reinterpret_cast<const uint4*>(pb + (k0) * 6 + 96);                \
    rb4 = *reinterpret_cast<const uint4*>(pb + (k0) * 6 + 128);                \
    rb5 = *reinterpret_cast<const uint4*>(pb + (k0) * 6 + 160);                \
  } while (0)
#define DPG_SPLIT_LSTORE()                                                       \
  do {                                                                           \
    const int o_ = srow * 4 + (skq ^ swz(srow));                                 \
    ss->A[0][o_] = ra0;                                                          \
    ss->A[1][o_] = ra1;                                                          \
    ss->A[2][o_] = ra2;                                                          \
    ss->A[3][o_] = ra3;                                                          \
    ss->A[4][o_] = ra4;                                                          \
    ss->A[5][o_] = ra5;                                                          \
    ss->B[0][o_] = rb0;                                                          \
    ss->B[1][o_] = rb1;                                                          \
    ss->B[2][o_] = rb2;                                                          \
    ss->B[3][o_] = rb3;                                                          \
    ss->B[4][o_] = rb4;                                                          \
    ss->B[5][o_] = rb5;                                                          \
  } while (0)
  f4 fr[2][2], fi[2][2];
  double dr[2][2][4], di[2][2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      fr[u][v] = f4{0, 0, 0, 0};
      fi[u][v] = f4{0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < 4; ++e) dr[u][v][e] = di[u][v][e] = 0.0;
    }
  const int nst = T.nvp / SKC;
  const int s0 = herk_k0(T, a, b) / SKC;   // stages of the F columns skipped where they contribute nothing
  DPG_SPLIT_GLOAD(s0 * SKC);
  for (int sidx = s0; sidx < nst; ++sidx) {
    __syncthreads();
    DPG_SPLIT_LSTORE();
    __syncthreads();
    if (sidx + 1 < nst) DPG_SPLIT_GLOAD((sidx + 1) * SKC);
    const int kq = lane >> 4;
    // B fragments of both column blocks once per stage; A per row block; the
    // four accumulators of a row block alternate so that no MFMA waits on the
    // previous one's result.
    bf8 Br[2][3], Bi[2][3];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int brow = wc * 32 + v * 16 + (lane & 15);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        Br[v][t] = lds_frag(ss->B[t], brow, kq);
        Bi[v][t] = lds_frag(ss->B[3 + t], brow, kq);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int arow = wr * 32 + u * 16 + (lane & 15);
      bf8 Ar[3], Ai[3], nAr[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        Ar[t] = lds_frag(ss->A[t], arow, kq);
        Ai[t] = lds_frag(ss->A[3 + t], arow, kq);
        nAr[t] = neg_frag(Ar[t]);
      }
      // re += Ar Br^T + Ai Bi^T ; im += Ai Br^T - Ar Bi^T   (terms with s + t <= 2).
      // The accumulators start each stage at zero and take the small terms
      // first and the two leading (s = t = 0) products last, so that only
      // those two roundings happen at the size of the stage's sum.
#pragma unroll
      for (int o = 0; o < 6; ++o) {
        // (s, t) = (2,0) (1,1) (0,2) (1,0) (0,1) (0,0)
        const int s2 = o < 3 ? 2 - o : (o < 5 ? 4 - o : 0);
        const int t2 = o < 3 ? o : (o < 5 ? o - 3 : 0);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          fr[u][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar[s2], Br[v][t2], fr[u][v], 0, 0, 0);
          fi[u][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ai[s2], Br[v][t2], fi[u][v], 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          fr[u][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ai[s2], Bi[v][t2], fr[u][v], 0, 0, 0);
          fi[u][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nAr[s2], Bi[v][t2], fi[u][v], 0, 0, 0);
        }
      }
    }
    {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            dr[u][v][e] += (double)fr[u][v][e];
            di[u][v][e] += (double)fi[u][v][e];
          }
          fr[u][v] = f4{0, 0, 0, 0};
          fi[u][v] = f4{0, 0, 0, 0};
        }
    }
  }
  // The tile leaves through LDS, 32 columns at a time, so that both its
  // stores (column runs of K) and those of its conjugate mirror (row runs)
  // are coalesced.
  const int k = T.k;
  double2* K = C.K + (C.K_off[gc] - C.K_base);
  double2* L = C.l + (C.v_off[gc] - C.v_base);
  constexpr int OP = 33;   // double2 pitch of the staged [64][32] half tile
  static_assert(64 * OP * sizeof(double2) <= sizeof(SplitStage), "staged half tile fits the stage buffer");
  double2* so = reinterpret_cast<double2*>(smem);
#pragma unroll
  for (int hc = 0; hc < 2; ++hc) {
    __syncthreads();   // stage buffer free
    if (wc == hc) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            // f32 16x16 accumulator layout: item e of lane l -> row 4(l>>4) + e, column l & 15
            const int r = wr * 32 + u * 16 + 4 * (lane >> 4) + e, cl = v * 16 + (lane & 15);
            so[r * OP + cl] = make_double2(dr[u][v][e], di[u][v][e]);
          }
    }
    __syncthreads();
    // element (al, be) of the tile: al = a TB + row, be = b TB + 32 hc + column
    for (int e = threadIdx.x; e < 64 * 32; e += NT) {
      const int cl = e >> 6, rl = e & 63;
      const int al = a * TB + rl, be = b * TB + 32 * hc + cl;
      const double2 v = so[rl * OP + cl];
      if (al < k && be < k) {
        if (!(a == b && be > al)) K[(int64_t)be * k + al] = v;
      } else if (al == k && be < k) {
        L[be] = make_double2(v.x, -v.y);
      }
    }
    for (int e = threadIdx.x; e < 64 * 32; e += NT) {
      const int rl = e >> 5, cl = e & 31;
      const int al = a * TB + rl, be = b * TB + 32 * hc + cl;
      if (al < k && be < k && al != be && !(a == b && be > al)) {
        const double2 v = so[rl * OP + cl];
        K[(int64_t)al * k + be] = make_double2(v.x, -v.y);
      }
    }
  }
}

#undef DPG_SPLIT_GLOAD
#undef DPG_SPLIT_LSTORE

// eta = ||L^{-1} D r|| in FP64: the residual row of W^H, reduced in a fixed order.
__global__ __launch_bounds__(NT) void k_eta(DevTables T, ChunkArgs C) {
  const int64_t cell = blockIdx.x;
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  const double2* z = C.Z + cell * T.zstride + T.nvp + T.k + 1;
  __shared__ double part[NT];
  double s = 0.0;
  for (int m = threadIdx.x; m < T.nvp; m += NT) {
    const double2 v = z[(int64_t)m * T.ldz];
    s += v.x * v.x + v.y * v.y;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) C.eta[gc - C.cell_base] = sqrt(part[0]);
}

// ================================================================ parity extraction
// G (full Hermitian, from the lower triangle), B_f and l of each chunk cell
// from the workspace (before factorisation).  SCALED = false: the unscaled
// forms (each entry divided by its Jacobi factors).  SCALED = true: the
// Jacobi-scaled system exactly as the factorisation reads it, D G D, D B_f,
// D l and D r (r = B_f x - l, zero without x), plus d = diag(G)^{-1/2}.
template <bool SCALED>
__global__ __launch_bounds__(NT) void k_extract(DevTables T, ChunkArgs C, double2* G, double2* Bf, double2* lv,
                                                double2* rv, double* dv) {
  const int64_t cell = blockIdx.y;
  if (cell >= C.n) return;
  const int nv = 2 * T.N;
  const double* d = C.dscale + cell * (int64_t)T.nvp;
  const double2* Z = C.Z + cell * T.zstride;
  const int64_t ld = T.ldz;
  auto zrow = [&](int i) { return i < T.N ? i : T.Np + (i - T.N); };
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t nG = (int64_t)nv * nv, nB = (int64_t)nv * T.k;
  if (e < nG) {
    const int i = (int)(e % nv), jj = (int)(e / nv);
    const int zi = zrow(i), zj = zrow(jj);
    const int nfb = (T.Np / TB) * TB;   // the real F block is in its compact copy
    double2 v;
    if (zi < nfb && zj < nfb)
      v = make_double2(C.fr[cell * fr_stride(T) + (int64_t)min(zi, zj) * fr_ld(T) + max(zi, zj)], 0.0);
    else
      v = (zi >= zj) ? Z[(int64_t)zj * ld + zi] : cconj(Z[(int64_t)zi * ld + zj]);
    const double s = SCALED ? 1.0 : 1.0 / (d[zi] * d[zj]);
    G[cell * nG + e] = make_double2(v.x * s, v.y * s);
  } else if (e < nG + nB) {
    const int64_t f = e - nG;
    const int i = (int)(f % nv), a = (int)(f / nv);
    const int zi = zrow(i);
    const double2 v =
        trace_unwritten(T, T.nvp + a, zi) ? make_double2(0.0, 0.0) : cconj(Z[(int64_t)zi * ld + T.nvp + a]);
    Bf[cell * nB + f] = SCALED ? v : make_double2(v.x / d[zi], v.y / d[zi]);
  } else if (e < nG + nB + nv) {
    const int i = (int)(e - nG - nB);
    const int zi = zrow(i);
    const double2 v = cconj(Z[(int64_t)zi * ld + T.nvp + T.k]);
    lv[cell * nv + i] = SCALED ? v : make_double2(v.x / d[zi], v.y / d[zi]);
    if (SCALED) {
      rv[cell * nv + i] = cconj(Z[(int64_t)zi * ld + T.nvp + T.k + 1]);
      dv[cell * nv + i] = d[zi];
    }
  }
}

}  // namespace

// ================================================================ launchers
static size_t scale_smem(const DevTables& t) { return sizeof(double) * (12 * (size_t)t.nq + 36 * (size_t)t.nfq); }

// Kernel class ids (match the DPG_K_* enum of the public header).
enum { KC_SCALE, KC_FORM_SM, KC_FORM_IF, KC_FORM_PAD, KC_FORM_B, KC_FORM_LOAD, KC_RESID, KC_CHOL_DIAG, KC_CHOL_PANEL,
       KC_HERK };

#define DPG_LAUNCH(cls, prof, st, ...)       \
  do {                                       \
    if (prof) (prof)->begin((cls), (st));    \
    hipLaunchKernelGGL(__VA_ARGS__);         \
    if (prof) (prof)->end((st));             \
  } while (0)

hipError_t launch_formation(const DevTables& t, const ProbArgs& pa, const ChunkArgs& ca, hipStream_t st,
                            Prof* prof) {
  if (ca.n <= 0) return hipSuccess;
  const size_t sm = scale_smem(t);
  DPG_LAUNCH(KC_SCALE, prof, st, k_cell_scale, dim3((unsigned)ca.n), dim3(NT), sm, st, t, pa, ca);
  const dim3 gsm(grid_cells_tiles(ca.n, 6));
  if (t.sf_cap != 4 && t.sf_cap != 8) return hipErrorInvalidValue;
  switch (t.n1 * 16 + t.sf_cap) {
#define DPG_SM_CASE(Q, CP)                                                                                    \
  case Q * 16 + CP:                                                                                           \
    DPG_LAUNCH(KC_FORM_SM, prof, st, (k_form_SM<Q, CP>), gsm, dim3(NT), (sizeof(double) * SfShape<Q, CP>::total), \
               st, t, pa, ca);                                                                                \
    break;
    DPG_SM_CASE(4, 4)
    DPG_SM_CASE(4, 8)
    DPG_SM_CASE(5, 4)
    DPG_SM_CASE(5, 8)
    DPG_SM_CASE(6, 4)
    DPG_SM_CASE(6, 8)
    DPG_SM_CASE(7, 4)
    DPG_SM_CASE(7, 8)
    DPG_SM_CASE(8, 4)
    DPG_SM_CASE(8, 8)
#undef DPG_SM_CASE
    default:
      return hipErrorInvalidValue;
  }
  const int nt = (t.Np + 63) / 64;
  DPG_LAUNCH(KC_FORM_IF, prof, st, k_form_IF, dim3(grid_cells_tiles(ca.n, nt * nt)), dim3(NT), 0, st, t, pa, ca);
  DPG_LAUNCH(KC_FORM_PAD, prof, st, k_form_pad, dim3((unsigned)ca.n), dim3(NT), 0, st, t, ca);
  // B_f^H: volume D and R (sum factorised), the volume part of the residual
  // row (matrix free), the Robin-face part, then the trace rows and padding
  const dim3 gb(grid_cells_tiles(ca.n, 9));
  switch ((t.n1 * 16 + t.p + 1) * 16 + t.sf_cap) {
#define DPG_B_CASE(Q, PP)                                                                                          \
  case (Q * 16 + PP) * 16 + 4:                                                                                     \
    DPG_LAUNCH(KC_FORM_B, prof, st, (k_form_Bsf<Q, PP, 4>), gb, dim3(NT), (sizeof(double) * SfbShape<Q, PP, 4>::total), \
               st, t, pa, ca);                                                                                     \
    if (ca.x)                                                                                                      \
      DPG_LAUNCH(KC_FORM_B, prof, st, (k_form_resid<Q, PP>), dim3((unsigned)ca.n), dim3(NT),                       \
                 (sizeof(double) * SfrShape<Q, PP>::total), st, t, pa, ca);                                        \
    break;                                                                                                         \
  case (Q * 16 + PP) * 16 + 8:                                                                                     \
    DPG_LAUNCH(KC_FORM_B, prof, st, (k_form_Bsf<Q, PP, 8>), gb, dim3(NT), (sizeof(double) * SfbShape<Q, PP, 8>::total), \
               st, t, pa, ca);                                                                                     \
    if (ca.x)                                                                                                        \
      DPG_LAUNCH(KC_FORM_B, prof, st, (k_form_resid<Q, PP>), dim3((unsigned)ca.n), dim3(NT),                         \
                 (sizeof(double) * SfrShape<Q, PP>::total), st, t, pa, ca);                                          \
    break;
    DPG_B_CASE(4, 2)
    DPG_B_CASE(5, 2)
    DPG_B_CASE(5, 3)
    DPG_B_CASE(6, 3)
    DPG_B_CASE(6, 4)
    DPG_B_CASE(7, 4)
    DPG_B_CASE(7, 5)
    DPG_B_CASE(8, 5)
#undef DPG_B_CASE
    default:
      return hipErrorInvalidValue;
  }
  DPG_LAUNCH(KC_FORM_B, prof, st, k_form_Bt, dim3(grid_cells_tiles(ca.n, nt)), dim3(NT), sizeof(double) * BQC * t.m1,
             st, t, pa, ca);
  switch ((t.nt1 + 63) / 64) {   // nt1 = 12 (p + 1)^2: 48, 108, 192, 300
#define DPG_T_CASE(M) \
  case M:             \
    DPG_LAUNCH(KC_FORM_B, prof, st, k_form_T<M>, dim3(grid_cells_tiles(ca.n, nt)), dim3(NT), 0, st, t, pa, ca); break;
    DPG_T_CASE(1)
    DPG_T_CASE(2)
    DPG_T_CASE(3)
    DPG_T_CASE(5)
#undef DPG_T_CASE
    default:
      return hipErrorInvalidValue;
  }
  DPG_LAUNCH(KC_FORM_LOAD, prof, st, k_form_load, dim3(grid_cells_tiles(ca.n, nt)), dim3(NT),
             sizeof(double2) * 3 * t.nfq, st, t, pa, ca);
  return hipGetLastError();
}

hipError_t launch_factor(const DevTables& t, const ChunkArgs& ca, hipStream_t st, Prof* prof) {
  if (ca.n <= 0) return hipSuccess;
  const int nvb = t.nvp / TB, nrb = t.nrows / TB;
  const int64_t n8 = (ca.n + 7) / 8 * 8;
  // the lookahead (or row-nF) workgroup of every cell + one row tile per
  // workgroup (the step kernel puts all lookahead workgroups first, the
  // F-column kernel each cell's row-nF workgroup before its row tiles)
  auto grid_of = [&](bool la, int nreg) {
    return (unsigned)((la ? n8 : 0) + 8 * ((n8 / 8 * nreg + RTPW - 1) / RTPW));
  };
  int j0 = 0;
  const int nF = t.Np / TB;   // leading column tiles that are real
  if (nF >= 1) {
    // F block first (one workgroup per cell), then the F columns of every other row in one launch
    DPG_LAUNCH(KC_CHOL_DIAG, prof, st, k_chol_fblock, dim3((unsigned)ca.n), dim3(NT), kFblockSmem, st, t, ca, nF);
    DPG_LAUNCH(KC_CHOL_PANEL, prof, st, k_chol_fpanel, dim3(grid_of(true, nrb - nF - 1)), dim3(NT), kFactorSmem, st,
               t, ca, nF);
    j0 = nF;
  } else {
    DPG_LAUNCH(KC_CHOL_DIAG, prof, st, k_chol_diag0, dim3((unsigned)ca.n), dim3(NT), kFactorSmem, st, t, ca);
  }
  for (int j = j0; j < nvb; ++j) {
    const bool la = j + 1 < nvb;
    const int nreg = nrb - j - 1 - (la ? 1 : 0);
    DPG_LAUNCH(KC_CHOL_PANEL, prof, st, k_chol_step, dim3(grid_of(la, nreg)), dim3(NT), kFactorSmem, st, t, ca, j);
  }
  return hipGetLastError();
}

hipError_t launch_herk(const DevTables& t, const ChunkArgs& ca, hipStream_t st, Prof* prof) {
  if (ca.n <= 0) return hipSuccess;
  const int kb = t.kp / TB;
  if (ca.split) {
    DPG_LAUNCH(KC_HERK, prof, st, k_herk_split, dim3(grid_cells_tiles(ca.n, kb * (kb + 1) / 2)), dim3(NT),
               sizeof(SplitStage), st, t, ca);
    DPG_LAUNCH(KC_RESID, prof, st, k_eta, dim3((unsigned)ca.n), dim3(NT), 0, st, t, ca);
  } else {
    DPG_LAUNCH(KC_HERK, prof, st, k_herk, dim3(grid_cells_tiles(ca.n, kb * (kb + 1) / 2)), dim3(NT),
               2 * sizeof(Stage), st, t, ca);
  }
  return hipGetLastError();
}

hipError_t launch_extract(const DevTables& t, const ChunkArgs& ca, double2* G, double2* Bf, double2* lvec,
                          hipStream_t st, double2* rvec, double* dvec) {
  if (ca.n <= 0) return hipSuccess;
  const int64_t nv = 2 * t.N;
  const int64_t tot = nv * nv + nv * t.k + nv;
  const dim3 grid((unsigned)((tot + NT - 1) / NT), (unsigned)ca.n);
  if (rvec && dvec)
    hipLaunchKernelGGL(k_extract<true>, grid, dim3(NT), 0, st, t, ca, G, Bf, lvec, rvec, dvec);
  else
    hipLaunchKernelGGL(k_extract<false>, grid, dim3(NT), 0, st, t, ca, G, Bf, lvec, rvec, dvec);
  return hipGetLastError();
}

// Kernels that need more than 64 KB of dynamic LDS must opt in once.
hipError_t configure_kernels() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int optin = 0;
  e = hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev);
  if (e != hipSuccess) return e;
  const void* fns[] = {reinterpret_cast<const void*>(&k_chol_diag0), reinterpret_cast<const void*>(&k_chol_step),
                       reinterpret_cast<const void*>(&k_chol_fpanel), reinterpret_cast<const void*>(&k_chol_fblock),
                       reinterpret_cast<const void*>(&k_cell_scale),
                       reinterpret_cast<const void*>(&k_form_Bt), reinterpret_cast<const void*>(&k_herk),
                       reinterpret_cast<const void*>(&k_herk_split),
#define DPG_FORM_FNS(Q, PP)                                                                                      \
  reinterpret_cast<const void*>(&k_form_Bsf<Q, PP, 4>), reinterpret_cast<const void*>(&k_form_Bsf<Q, PP, 8>),     \
      reinterpret_cast<const void*>(&k_form_resid<Q, PP>),
                       DPG_FORM_FNS(4, 2) DPG_FORM_FNS(5, 2) DPG_FORM_FNS(5, 3) DPG_FORM_FNS(6, 3) DPG_FORM_FNS(6, 4)
                       DPG_FORM_FNS(7, 4) DPG_FORM_FNS(7, 5) DPG_FORM_FNS(8, 5)
#undef DPG_FORM_FNS
#define DPG_SM_FNS(Q) reinterpret_cast<const void*>(&k_form_SM<Q, 4>), reinterpret_cast<const void*>(&k_form_SM<Q, 8>),
                       DPG_SM_FNS(4) DPG_SM_FNS(5) DPG_SM_FNS(6) DPG_SM_FNS(7) DPG_SM_FNS(8)
#undef DPG_SM_FNS
                       nullptr};
  for (const void* f : fns) {
    if (!f) continue;
    hipFuncAttributes fa;
    e = hipFuncGetAttributes(&fa, f);
    if (e != hipSuccess) return e;
    // the dynamic allowance is what the per-block limit leaves after static LDS
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, optin - (int)fa.sharedSizeBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dpg
