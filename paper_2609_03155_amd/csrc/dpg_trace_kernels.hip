// HIP kernels of the condensed trace system (paper §2.3: static condensation
// of the interior unknowns, A_K = M3 - M2^H M1^{-1} M2, b_K = l_t - M2^H M1^{-1} l_u,
// and the global system solved by CG).
//
// The condensation reuses the blocked Cholesky/TRSM/HERK kernels of the local
// solve on a second augmented matrix per cell, built from K_e and l_e:
//   rows [0, nvp')          D M1 D (lower; identity padding to a multiple of 64)
//   rows [nvp', nvp'+n_t)   (D M2)^H
//   row  nvp'+n_t           (D l_u)^H
// with D = diag(M1)^{-1/2}.  After the factorisation the HERK of the lower
// rows yields M2^H M1^{-1} M2 and M2^H M1^{-1} l_u, which k_cond_finish
// subtracts from M3 and l_t.  Assembly gathers every nonzero of the global
// CSR matrix from its cell contributions (fixed order: deterministic, no
// atomics); the matvec is the complex CSR product of the CG iteration.
//
// The global system is solved by CG without a preconditioner (the system is
// Hermitian positive definite); its scalars stay on the device and every
// reduction runs in a fixed order, so a solve is bitwise reproducible.  The
// interior unknowns are then recovered per cell, u = M1^{-1} (l_u - M2 t_K):
// the same factorisation kernels on D M1 D with the single row (D r)^H,
// r = l_u - M2 t_K, appended, leave y = L^{-1} D r in that row; a backward
// substitution through the stored factor gives u = D L^{-H} y.
#include "dpg_kernels.h"

#include <algorithm>

namespace dpg {

namespace {

constexpr int NT = 256;
constexpr int TB = 64;   // tile of the blocked factorisation

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One workgroup per (cell, column a) of the condensation matrix.
__global__ __launch_bounds__(NT) void k_cond_load(DevTables T, ChunkArgs C, CondArgs A) {
  const int64_t cell = (int64_t)blockIdx.x / T.nvp;
  const int a = (int)((int64_t)blockIdx.x - cell * T.nvp);
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  const double2* K = A.Ke + (A.Ke_off[gc] - A.Ke_base);
  const double2* le = A.le + (A.le_off[gc] - A.le_base);
  const int nu = A.nu, kf = A.kfull;
  double2* Z = C.Z + cell * T.zstride + (int64_t)a * T.ldz;
  const bool real_col = a < nu;
  const double da = real_col ? rsqrt(K[(int64_t)a * kf + a].x) : 1.0;
  if (a == 0 && threadIdx.x == 0) C.info[gc - C.cell_base] = 0;   // the factorisation reports pivots
  for (int i = threadIdx.x; i < T.nrows; i += NT) {
    double2 v = make_double2(0.0, 0.0);
    if (i < T.nvp) {
      if (real_col && i < nu && i >= a) {
        const double di = rsqrt(K[(int64_t)i * kf + i].x);
        const double2 m = K[(int64_t)a * kf + i];
        v = make_double2(di * da * m.x, di * da * m.y);
      } else if (i == a && !real_col) {
        v = make_double2(1.0, 0.0);
      }
    } else if (real_col) {
      const int t = i - T.nvp;
      if (t < T.k) {
        const double2 m = K[(int64_t)a * kf + nu + t];   // (M2^H)(t, a) = K_e(nu + t, a)
        v = make_double2(da * m.x, da * m.y);
      } else if (t == T.k) {
        v = make_double2(da * le[a].x, -da * le[a].y);   // conj(d l_u)
      }
    }
    Z[i] = v;
  }
}

// A_K = M3 - A', b_K = l_t - b' in place (A', b' written by the HERK); one
// workgroup per (cell, column s).
__global__ __launch_bounds__(NT) void k_cond_finish(DevTables T, ChunkArgs C, CondArgs A) {
  const int nt = T.k;
  const int64_t cell = (int64_t)blockIdx.x / nt;
  const int s = (int)((int64_t)blockIdx.x - cell * nt);
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  const double2* K = A.Ke + (A.Ke_off[gc] - A.Ke_base);
  const double2* le = A.le + (A.le_off[gc] - A.le_base);
  const int nu = A.nu, kf = A.kfull;
  double2* Ak = C.K + (C.K_off[gc] - C.K_base) + (int64_t)s * nt;
  const double2* M3 = K + (int64_t)(nu + s) * kf + nu;
  for (int t = threadIdx.x; t < nt; t += NT) {
    const double2 m = M3[t], p = Ak[t];
    Ak[t] = make_double2(m.x - p.x, m.y - p.y);
  }
  if (s == 0) {
    double2* bk = C.l + (C.v_off[gc] - C.v_base);
    for (int t = threadIdx.x; t < nt; t += NT) {
      const double2 m = le[nu + t], p = bk[t];
      bk[t] = make_double2(m.x - p.x, m.y - p.y);
    }
  }
}

// vals[z] = sum of the cell contributions of nonzero z, in list order.
__global__ __launch_bounds__(NT) void k_gather(int64_t n, const int64_t* __restrict__ ptr,
                                               const int64_t* __restrict__ src, const double2* __restrict__ from,
                                               double2* __restrict__ to) {
  const int64_t z = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (z >= n) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t k = ptr[z]; k < ptr[z + 1]; ++k) {
    const double2 v = from[src[k]];
    acc.x += v.x;
    acc.y += v.y;
  }
  to[z] = acc;
}

// y = A x, complex CSR; one wave per row, lanes strided over the row, then
// a fixed-order butterfly reduction (deterministic).
__global__ __launch_bounds__(NT) void k_csr_matvec(int64_t n_rows, const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col, const double2* __restrict__ val,
                                                   const double2* __restrict__ x, double2* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_rows) return;
  double re = 0.0, im = 0.0;
  for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += 64) {
    const double2 p = cmul(val[k], x[col[k]]);
    re += p.x;
    im += p.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) y[row] = make_double2(re, im);
}

// ---------------------------------------------------------------- CG
// Iteration scalars (device doubles): rr = r^H r, alpha, beta, ||b||^2, the
// convergence flag, the iteration count, tol^2.  Every kernel of an
// iteration returns at once when the flag is set, so iterations launched
// past convergence change nothing.
__device__ __forceinline__ bool cg_done(const double* sc) { return sc[CG_DONE] != 0.0; }

// Fixed-order sum of one double per thread of the block (a power of two).
template <int NTH>
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int off = NTH / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  return red[0];
}

// q = A p (one wave per row, as k_csr_matvec) and, per workgroup, the partial
// sum of Re(conj(p_i) q_i) over its rows.
__global__ __launch_bounds__(NT) void k_cg_matvec_dot(int64_t n, const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, const double2* __restrict__ val,
                                                      const double2* __restrict__ p, double2* __restrict__ q,
                                                      double* __restrict__ part, const double* __restrict__ sc) {
  __shared__ double red[NT / 64];
  if (cg_done(sc)) return;
  const int64_t row = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double re = 0.0, im = 0.0;
  if (row < n) {
    for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += 64) {
      const double2 v = cmul(val[k], p[col[k]]);
      re += v.x;
      im += v.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
  }
  if (lane == 0) {
    double d = 0.0;
    if (row < n) {
      q[row] = make_double2(re, im);
      const double2 pr = p[row];
      d = pr.x * re + pr.y * im;
    }
    red[threadIdx.x >> 6] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Thread t's share of a fixed-order sum: part[t], part[t + RNT], ... added in
// that order, the loads issued eight at a time (the partial sums of the
// matvec are n / 4 doubles, which one workgroup reads).
constexpr int RNT = 1024;
__device__ __forceinline__ double strided_sum(const double* __restrict__ part, int64_t m) {
  double v = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 7 * (int64_t)RNT < m; i += 8 * (int64_t)RNT) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = part[i + (int64_t)u * RNT];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  for (; i < m; i += RNT) v += part[i];
  return v;
}

// One workgroup: s = sum of part[0, m) in a fixed order, then
//   MODE 0 (alpha):  alpha = rr / s  (0 if s <= 0: no further progress);
//   MODE 1 (beta):   rr_new = s, beta = rr_new / rr, rr = rr_new, count the
//                    iteration and set the flag once rr <= tol^2 ||b||^2;
//   MODE 2 (start):  rr = s, ||b||^2 = part[m, 2m) summed likewise, flag set if
//                    the start already satisfies the test.
template <int MODE>
__global__ __launch_bounds__(RNT) void k_cg_scalar(const double* __restrict__ part, int64_t m, double* __restrict__ sc) {
  __shared__ double red[RNT];
  if (cg_done(sc)) return;
  const double s = block_sum<RNT>(strided_sum(part, m), red);
  double sb = 0.0;
  if (MODE == 2) {
    __syncthreads();
    sb = block_sum<RNT>(strided_sum(part + m, m), red);
  }
  if (threadIdx.x != 0) return;
  if (MODE == 0) {
    sc[CG_ALPHA] = (s > 0.0 && sc[CG_RR] > 0.0) ? sc[CG_RR] / s : 0.0;
  } else if (MODE == 1) {
    const double rr = sc[CG_RR];
    sc[CG_BETA] = rr > 0.0 ? s / rr : 0.0;
    sc[CG_RR] = s;
    sc[CG_ITERS] += 1.0;
    if (!(s > sc[CG_TOL2] * sc[CG_BN2])) sc[CG_DONE] = 1.0;
  } else {
    sc[CG_RR] = s;
    sc[CG_BN2] = sb;
    sc[CG_ITERS] = 0.0;
    sc[CG_DONE] = (sb == 0.0 || !(s > sc[CG_TOL2] * sb)) ? 1.0 : 0.0;
  }
}

// Elements per workgroup of the vector kernels (each thread a fixed run).
constexpr int VPT = 8;
constexpr int64_t VCHUNK = (int64_t)NT * VPT;

// x += alpha p, r -= alpha q, and the partial sums of |r_i|^2.
__global__ __launch_bounds__(NT) void k_cg_update(int64_t n, double2* __restrict__ x, double2* __restrict__ r,
                                                  const double2* __restrict__ p, const double2* __restrict__ q,
                                                  double* __restrict__ part, const double* __restrict__ sc) {
  __shared__ double red[NT];
  if (cg_done(sc)) return;
  const double alpha = sc[CG_ALPHA];
  double acc = 0.0;
  const int64_t base = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int64_t i = base + (int64_t)u * NT;
    if (i < n) {
      const double2 pi = p[i], qi = q[i];
      double2 xi = x[i], ri = r[i];
      xi.x = fma(alpha, pi.x, xi.x);
      xi.y = fma(alpha, pi.y, xi.y);
      ri.x = fma(-alpha, qi.x, ri.x);
      ri.y = fma(-alpha, qi.y, ri.y);
      x[i] = xi;
      r[i] = ri;
      acc += ri.x * ri.x + ri.y * ri.y;
    }
  }
  const double s = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = r + beta p.
__global__ __launch_bounds__(NT) void k_cg_direction(int64_t n, const double2* __restrict__ r, double2* __restrict__ p,
                                                     const double* __restrict__ sc) {
  if (cg_done(sc)) return;
  const double beta = sc[CG_BETA];
  const int64_t base = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int64_t i = base + (int64_t)u * NT;
    if (i < n) {
      const double2 ri = r[i], pi = p[i];
      p[i] = make_double2(fma(beta, pi.x, ri.x), fma(beta, pi.y, ri.y));
    }
  }
}

// Start: r = b - q (q = A x0), p = r; partial sums of |r_i|^2 into part[blk]
// and of |b_i|^2 into part[nblk + blk].
__global__ __launch_bounds__(NT) void k_cg_start(int64_t n, const double2* __restrict__ b, const double2* __restrict__ q,
                                                 double2* __restrict__ r, double2* __restrict__ p,
                                                 double* __restrict__ part) {
  __shared__ double red[NT];
  double ar = 0.0, ab = 0.0;
  const int64_t base = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int64_t i = base + (int64_t)u * NT;
    if (i < n) {
      const double2 bi = b[i], qi = q[i];
      const double2 ri = make_double2(bi.x - qi.x, bi.y - qi.y);
      r[i] = ri;
      p[i] = ri;
      ar += ri.x * ri.x + ri.y * ri.y;
      ab += bi.x * bi.x + bi.y * bi.y;
    }
  }
  const double sr = block_sum<NT>(ar, red);
  __syncthreads();
  const double sb = block_sum<NT>(ab, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sr;
    part[gridDim.x + blockIdx.x] = sb;
  }
}

// ---------------------------------------------------------------- trace scatter
// out[i] = t[glob[i]], or 0 where glob[i] < 0 (removed or constrained).
__global__ __launch_bounds__(NT) void k_scatter(int64_t n, const int64_t* __restrict__ glob,
                                                const double2* __restrict__ t, double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int64_t g = glob[i];
  out[i] = g >= 0 ? t[g] : make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------- reconstruction
// Column a of the reconstruction matrix (one workgroup per (cell, a)):
//   rows [0, nvp)   column a of D M1 D (lower part; identity on the padding),
//   row  nvp        conj(d_a r_a),  r_a = l_u[a] - sum_t M2(a, t) t_K[t],
//   rows after      zero.
// M2(a, t) = conj(K_e(nu + t, a)), read down column a of K_e.
__global__ __launch_bounds__(NT) void k_recon_load(DevTables T, ChunkArgs C, CondArgs A) {
  __shared__ double red[2][NT];
  const int64_t cell = (int64_t)blockIdx.x / T.nvp;
  const int a = (int)((int64_t)blockIdx.x - cell * T.nvp);
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  const double2* K = A.Ke + (A.Ke_off[gc] - A.Ke_base);
  const double2* le = A.le + (A.le_off[gc] - A.le_base);
  const double2* tk = A.tk + A.tk_off[gc];
  const int nu = A.nu, kf = A.kfull, nt = kf - nu;
  double2* Z = C.Z + cell * T.zstride + (int64_t)a * T.ldz;
  const bool real_col = a < nu;
  const double da = real_col ? rsqrt(K[(int64_t)a * kf + a].x) : 1.0;
  if (a == 0 && threadIdx.x == 0) C.info[gc - C.cell_base] = 0;   // the factorisation reports pivots
  // r_a (workgroup reduction in a fixed order)
  double sr = 0.0, si = 0.0;
  if (real_col) {
    for (int t = threadIdx.x; t < nt; t += NT) {
      const double2 m = K[(int64_t)a * kf + nu + t];   // K_e(nu + t, a) = conj(M2(a, t))
      const double2 v = tk[t];
      sr += m.x * v.x + m.y * v.y;                     // Re(conj(m) v)
      si += m.x * v.y - m.y * v.x;                     // Im(conj(m) v)
    }
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = si;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < T.nrows; i += NT) {
    double2 v = make_double2(0.0, 0.0);
    if (i < T.nvp) {
      if (real_col && i < nu && i >= a) {
        const double di = rsqrt(K[(int64_t)i * kf + i].x);
        const double2 m = K[(int64_t)a * kf + i];
        v = make_double2(di * da * m.x, di * da * m.y);
      } else if (i == a && !real_col) {
        v = make_double2(1.0, 0.0);
      }
    } else if (i == T.nvp && real_col) {
      const double rr = le[a].x - red[0][0], ri = le[a].y - red[1][0];
      v = make_double2(da * rr, -da * ri);   // conj(d_a r_a)
    }
    Z[i] = v;
  }
}

// Backward substitution per cell (one workgroup): z = L^{-H} y with y the
// conjugate of row nvp and L stored by the factorisation (L_ij below the
// diagonal tiles; on them L_jj below the 16x16 block diagonal and the
// inverses of its diagonal blocks); for column blocks J = nvb-1 .. 0
//   s_J = y_J - sum_{I > J} L_IJ^H z_I,   L_JJ^H z_J = s_J ;
// then x_e = [D z (first nu) ; t_K].  For s_J each wave takes 16 columns of
// block J, its lanes run down a column (contiguous), and one butterfly per
// column sums the lanes (fixed order); the tile's own substitution is small
// and runs on one wave.
__global__ __launch_bounds__(NT) void k_recon_back(DevTables T, ChunkArgs C, CondArgs A) {
  extern __shared__ double2 zs[];   // [nvp] z, then [64] s and [64] t of the current block
  const int64_t cell = blockIdx.x;
  if (cell >= C.n) return;
  const int64_t gc = C.cell_ids[cell];
  const int64_t ld = T.ldz;
  const double2* Z = C.Z + cell * T.zstride;
  const int nvb = T.nvp / TB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double2* sb = zs + T.nvp;
  for (int J = nvb - 1; J >= 0; --J) {
    for (int cc = 0; cc < 16; ++cc) {
      const int c = wave * 16 + cc;
      const double2* colp = Z + (int64_t)(J * TB + c) * ld;
      double re = 0.0, im = 0.0;
      for (int rr = (J + 1) * TB + lane; rr < T.nvp; rr += 64) {
        const double2 l = colp[rr], z = zs[rr];
        re += l.x * z.x + l.y * z.y;   // conj(l) z
        im += l.x * z.y - l.y * z.x;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
      }
      if (lane == 0) {
        const double2 yrow = colp[T.nvp];   // conj(y_c)
        sb[c] = make_double2(yrow.x - re, -yrow.y - im);
      }
    }
    __syncthreads();
    // L_JJ^H z_J = s_J by backward substitution over the tile's four 16-row
    // blocks m (the factorisation stores L_JJ below the block diagonal and the
    // inverses Dinv of its diagonal blocks on it):
    //   t = s[m] - sum_{m2 > m} L_JJ[m2][m]^H z[m2],  z[m] = Dinv[m]^H t.
    // All 64 lanes of wave 0: lane (ro, cg) = (l & 15, l >> 4) takes rows
    // ro + 16 k of columns c = 16 m + cg + 4 q (q = 0..3), so that the 16
    // lanes of a column read consecutive rows; the sums over ro close with a
    // butterfly in a fixed order.
    if (wave == 0) {
      const double2* tile = Z + (int64_t)(J * TB) * ld + J * TB;   // column c at tile + c ld
      double2* tb = sb + TB;                                        // [64] t of the current block
      const int ro = lane & 15, cg = lane >> 4;
      auto butterfly = [&](double2* acc) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int off = 8; off > 0; off >>= 1) {
            acc[q].x += __shfl_xor(acc[q].x, off, 64);
            acc[q].y += __shfl_xor(acc[q].y, off, 64);
          }
      };
      for (int m = 3; m >= 0; --m) {
        double2 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
        for (int r = 16 * (m + 1) + ro; r < TB; r += 16) {
          const double2 z = zs[J * TB + r];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double2 l = tile[(int64_t)(16 * m + cg + 4 * q) * ld + r];
            acc[q].x += l.x * z.x + l.y * z.y;   // conj(l) z
            acc[q].y += l.x * z.y - l.y * z.x;
          }
        }
        butterfly(acc);
        if (ro == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int c = 16 * m + cg + 4 * q;
            tb[c] = make_double2(sb[c].x - acc[q].x, sb[c].y - acc[q].y);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // z[c] = sum_{r >= c in block m} conj(Dinv[r][c]) t[r]
        {
          const int r = 16 * m + ro;
          const double2 t = tb[r];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int c = 16 * m + cg + 4 * q;
            double2 v = make_double2(0.0, 0.0);
            if (r >= c) {
              const double2 l = tile[(int64_t)c * ld + r];
              v = make_double2(l.x * t.x + l.y * t.y, l.x * t.y - l.y * t.x);
            }
            acc[q] = v;
          }
        }
        butterfly(acc);
        if (ro == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q) zs[J * TB + 16 * m + cg + 4 * q] = acc[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
    }
    __syncthreads();
  }
  const double2* K = A.Ke + (A.Ke_off[gc] - A.Ke_base);
  const double2* tk = A.tk + A.tk_off[gc];
  double2* x = A.xout + (A.le_off[gc] - A.le_base);
  const int nu = A.nu, kf = A.kfull;
  for (int i = threadIdx.x; i < kf; i += NT) {
    if (i < nu) {
      const double d = rsqrt(K[(int64_t)i * kf + i].x);
      const double2 z = zs[i];
      x[i] = make_double2(d * z.x, d * z.y);
    } else {
      x[i] = tk[i - nu];
    }
  }
}

// ---------------------------------------------------------------- power dissipation
// Per cell of a degree group (one workgroup): with E, H the DG fields of the
// cell's coefficients x = [E_x, E_y, E_z, H_x, H_y, H_z] (Lagrange-GLL
// functions, the table's trial basis at the volume Gauss points), the
// integrals over the cell of |E|^2 and |H|^2 and of the dissipated power
// density omega (eps_im |E|^2 + mu_im |H|^2) / 2, in the non-dimensional
// variables (lengths in units of L):  out[cell] = {power, |E|^2, |H|^2}.
__global__ __launch_bounds__(NT) void k_power(DevTables T, ProbArgs P, const int64_t* __restrict__ cell_ids, int64_t n,
                                              const double2* __restrict__ x, const int64_t* __restrict__ v_off,
                                              double* __restrict__ out) {
  extern __shared__ double2 xs[];   // [6 m1] the cell's field coefficients
  __shared__ double red[2][NT];
  const int64_t cell = blockIdx.x;
  if (cell >= n) return;
  const int64_t gc = cell_ids[cell];
  const int m1 = T.m1;
  const double2* xc = x + v_off[gc];
  for (int i = threadIdx.x; i < 6 * m1; i += NT) xs[i] = xc[i];
  double X[8][3];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int64_t id = P.cells[8 * gc + v];
#pragma unroll
    for (int d = 0; d < 3; ++d) X[v][d] = P.vertices[3 * id + d] * P.inv_len;
  }
  __syncthreads();
  double se = 0.0, sh = 0.0;
  for (int q = threadIdx.x; q < T.nq; q += NT) {
    const double* xi = T.vol_pts + 3 * q;
    // J_ab = dx_a / dxi_b of the trilinear map (vertex v(i,j,k) at 4k + 2j + i)
    double J[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int i = v & 1, j = (v >> 1) & 1, k = v >> 2;
      const double fx = i ? xi[0] : 1.0 - xi[0], fy = j ? xi[1] : 1.0 - xi[1], fz = k ? xi[2] : 1.0 - xi[2];
      const double gx = i ? 1.0 : -1.0, gy = j ? 1.0 : -1.0, gz = k ? 1.0 : -1.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        J[a][0] += gx * fy * fz * X[v][a];
        J[a][1] += fx * gy * fz * X[v][a];
        J[a][2] += fx * fy * gz * X[v][a];
      }
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double wq = T.vol_w[q] * fabs(det);
    double fr[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, fi[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double* ph = T.vol_phi + (int64_t)q * m1;
    for (int a = 0; a < m1; ++a) {
      const double f = ph[a];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double2 u = xs[c * m1 + a];
        fr[c] = fma(f, u.x, fr[c]);
        fi[c] = fma(f, u.y, fi[c]);
      }
    }
    double e2 = 0.0, h2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e2 += fr[c] * fr[c] + fi[c] * fi[c];
      h2 += fr[3 + c] * fr[3 + c] + fi[3 + c] * fi[3 + c];
    }
    se = fma(wq, e2, se);
    sh = fma(wq, h2, sh);
  }
  red[0][threadIdx.x] = se;
  red[1][threadIdx.x] = sh;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double IE = red[0][0], IH = red[1][0];
    out[3 * gc + 0] = 0.5 * P.omega * (P.eps[2 * gc + 1] * IE + P.mu[2 * gc + 1] * IH);
    out[3 * gc + 1] = IE;
    out[3 * gc + 2] = IH;
  }
}

}  // namespace

hipError_t launch_power(const DevTables& t, const ProbArgs& pa, const int64_t* cell_ids, int64_t n, const double2* x,
                        const int64_t* v_off, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_power, dim3((unsigned)n), dim3(NT), sizeof(double2) * 6 * t.m1, st, t, pa, cell_ids, n, x, v_off,
                     out);
  return hipGetLastError();
}

hipError_t launch_cond_load(const DevTables& t, const ChunkArgs& ca, const CondArgs& a, hipStream_t st) {
  if (ca.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cond_load, dim3((unsigned)(ca.n * t.nvp)), dim3(NT), 0, st, t, ca, a);
  return hipGetLastError();
}

hipError_t launch_cond_finish(const DevTables& t, const ChunkArgs& ca, const CondArgs& a, hipStream_t st) {
  if (ca.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cond_finish, dim3((unsigned)(ca.n * t.k)), dim3(NT), 0, st, t, ca, a);
  return hipGetLastError();
}

hipError_t launch_gather(int64_t n, const int64_t* ptr, const int64_t* src, const double2* from, double2* to,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, ptr, src, from, to);
  return hipGetLastError();
}

hipError_t launch_csr_matvec(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const double2* val,
                             const double2* x, double2* y, hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  const int64_t rows_per_block = NT / 64;
  hipLaunchKernelGGL(k_csr_matvec, dim3((unsigned)((n_rows + rows_per_block - 1) / rows_per_block)), dim3(NT), 0,
                     st, n_rows, row_ptr, col, val, x, y);
  return hipGetLastError();
}

}  // namespace dpg

namespace dpg {

hipError_t launch_recon_load(const DevTables& t, const ChunkArgs& ca, const CondArgs& a, hipStream_t st) {
  if (ca.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_recon_load, dim3((unsigned)(ca.n * t.nvp)), dim3(NT), 0, st, t, ca, a);
  return hipGetLastError();
}

hipError_t launch_recon_back(const DevTables& t, const ChunkArgs& ca, const CondArgs& a, hipStream_t st) {
  if (ca.n <= 0) return hipSuccess;
  const size_t smem = sizeof(double2) * ((size_t)t.nvp + 2 * TB);
  hipLaunchKernelGGL(k_recon_back, dim3((unsigned)ca.n), dim3(NT), smem, st, t, ca, a);
  return hipGetLastError();
}

hipError_t launch_scatter(int64_t n, const int64_t* glob, const double2* t, double2* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, glob, t, out);
  return hipGetLastError();
}

int64_t cg_mv_blocks(int64_t n) { return (n + NT / 64 - 1) / (NT / 64); }

int64_t cg_part_len(int64_t n) {
  const int64_t nmv = cg_mv_blocks(n), nv = (n + VCHUNK - 1) / VCHUNK;
  return std::max<int64_t>(nmv, 2 * nv) + 1;
}

hipError_t launch_cg_start(const CgArgs& g, hipStream_t st) {
  const int64_t n = g.n;
  const unsigned nmv = (unsigned)((n + NT / 64 - 1) / (NT / 64)), nv = (unsigned)((n + VCHUNK - 1) / VCHUNK);
  hipLaunchKernelGGL(k_csr_matvec, dim3(nmv), dim3(NT), 0, st, n, g.row_ptr, g.col, g.val, g.x, g.q);
  hipLaunchKernelGGL(k_cg_start, dim3(nv), dim3(NT), 0, st, n, g.b, g.q, g.r, g.p, g.part);
  hipLaunchKernelGGL(k_cg_scalar<2>, dim3(1), dim3(RNT), 0, st, g.part, (int64_t)nv, g.sc);
  return hipGetLastError();
}

hipError_t launch_cg_iterations(const CgArgs& g, int64_t count, hipStream_t st) {
  const int64_t n = g.n;
  const unsigned nmv = (unsigned)cg_mv_blocks(n), nv = (unsigned)((n + VCHUNK - 1) / VCHUNK);
  for (int64_t it = 0; it < count; ++it) {
    hipLaunchKernelGGL(k_cg_matvec_dot, dim3(nmv), dim3(NT), 0, st, n, g.row_ptr, g.col, g.val, g.p, g.q, g.part, g.sc);
    hipLaunchKernelGGL(k_cg_scalar<0>, dim3(1), dim3(RNT), 0, st, g.part, (int64_t)nmv, g.sc);
    hipLaunchKernelGGL(k_cg_update, dim3(nv), dim3(NT), 0, st, n, g.x, g.r, g.p, g.q, g.part, g.sc);
    hipLaunchKernelGGL(k_cg_scalar<1>, dim3(1), dim3(RNT), 0, st, g.part, (int64_t)nv, g.sc);
    hipLaunchKernelGGL(k_cg_direction, dim3(nv), dim3(NT), 0, st, n, g.r, g.p, g.sc);
  }
  return hipGetLastError();
}

}  // namespace dpg
