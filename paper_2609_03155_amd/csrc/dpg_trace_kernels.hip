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
#include "dpg_kernels.h"

namespace dpg {

namespace {

constexpr int NT = 256;

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

}  // namespace

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
