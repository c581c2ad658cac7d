/*
 * Extended-precision local solve of one cell -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/ and bench.py's accuracy report call this (through
 * oracle/xsolve.py).  It shares no code with the HIP library.
 *
 * Given FP64 inputs G (n x n, Hermitian positive definite), B (n x k), l (n)
 * and r (n), all complex, it evaluates in x87 long double (64-bit
 * significand, unit roundoff 2^-64 ~ 5.4e-20) the plain definitions of the
 * optimal-test elimination of Sec. 2.3:
 *     K = B^H G^{-1} B,   le = B^H G^{-1} l,   eta^2 = r^H G^{-1} r,
 * with G^{-1} applied through G = L L^H:  W = L^{-1} [B l r],
 *     K = W_B^H W_B,  le = W_B^H w_l,  eta^2 = w_r^H w_r.
 * With kappa(G) <= 1e9 the extended result is within ~1e-10 kappa u_ext of
 * the exact solve of the FP64 inputs, i.e. exact to FP64 working accuracy;
 * it measures the forward error of an FP64 solve of the same inputs.
 *
 * Arrays are C order (row-major), complex interleaved (re, im) doubles:
 *   G[(i*n + j)*2 + {0,1}] = G_ij,  B[(i*k + a)*2 + .] = B_ia,
 *   K[(a*k + b)*2 + .] = K_ab (output), le[a*2 + .] (output),
 *   norms[0] = r^H G^{-1} r (0 when r is NULL), norms[1] = l^H G^{-1} l.
 * Only the lower triangle of G (j <= i) is read.
 * Returns 0, or the 1-based column of the first non-positive pivot.
 */
#include <math.h>
#include <stdlib.h>

typedef long double ld;

int xsolve(int n, int k, const double* G, const double* B, const double* l, const double* r, double* K, double* le,
           double* norms) {
  const int m = k + 2; /* right-hand sides: the k columns of B, l, r */
  ld* Lr = (ld*)calloc((size_t)n * n, sizeof(ld));
  ld* Li = (ld*)calloc((size_t)n * n, sizeof(ld));
  ld* Wr = (ld*)calloc((size_t)m * n, sizeof(ld)); /* W transposed: W^T[a][i] */
  ld* Wi = (ld*)calloc((size_t)m * n, sizeof(ld));
  int fail = 0;
  if (!Lr || !Li || !Wr || !Wi) {
    fail = -1;
    goto done;
  }
  /* Cholesky by columns: L_jj = sqrt(G_jj - sum_{q<j} |L_jq|^2),
   * L_ij = (G_ij - sum_{q<j} L_iq conj(L_jq)) / L_jj for i > j. */
  for (int j = 0; j < n && !fail; ++j) {
    ld d = (ld)G[((size_t)j * n + j) * 2];
    for (int q = 0; q < j; ++q) d -= Lr[(size_t)j * n + q] * Lr[(size_t)j * n + q] + Li[(size_t)j * n + q] * Li[(size_t)j * n + q];
    if (!(d > 0)) {
      fail = j + 1;
      break;
    }
    const ld ljj = sqrtl(d);
    Lr[(size_t)j * n + j] = ljj;
    Li[(size_t)j * n + j] = 0;
    const ld* ajr = Lr + (size_t)j * n;
    const ld* aji = Li + (size_t)j * n;
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < n; ++i) {
      ld sr = (ld)G[((size_t)i * n + j) * 2], si = (ld)G[((size_t)i * n + j) * 2 + 1];
      const ld* air = Lr + (size_t)i * n;
      const ld* aii = Li + (size_t)i * n;
      for (int q = 0; q < j; ++q) {
        /* L_iq conj(L_jq) */
        sr -= air[q] * ajr[q] + aii[q] * aji[q];
        si -= aii[q] * ajr[q] - air[q] * aji[q];
      }
      Lr[(size_t)i * n + j] = sr / ljj;
      Li[(size_t)i * n + j] = si / ljj;
    }
  }
  if (fail) goto done;
  /* forward substitution, one right-hand side per thread: L w = rhs */
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < m; ++a) {
    ld* wr = Wr + (size_t)a * n;
    ld* wi = Wi + (size_t)a * n;
    for (int i = 0; i < n; ++i) {
      ld sr = 0, si = 0;
      if (a < k) {
        sr = (ld)B[((size_t)i * k + a) * 2];
        si = (ld)B[((size_t)i * k + a) * 2 + 1];
      } else if (a == k) {
        sr = (ld)l[(size_t)i * 2];
        si = (ld)l[(size_t)i * 2 + 1];
      } else if (r) {
        sr = (ld)r[(size_t)i * 2];
        si = (ld)r[(size_t)i * 2 + 1];
      }
      const ld* lr = Lr + (size_t)i * n;
      const ld* li = Li + (size_t)i * n;
      for (int q = 0; q < i; ++q) {
        sr -= lr[q] * wr[q] - li[q] * wi[q];
        si -= lr[q] * wi[q] + li[q] * wr[q];
      }
      wr[i] = sr / lr[i];
      wi[i] = si / lr[i];
    }
  }
  /* K_ab = sum_i conj(W_ia) W_ib (a = k: le), eta^2 = |w_r|^2 */
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a <= k; ++a) {
    const ld* ar = Wr + (size_t)a * n;
    const ld* ai = Wi + (size_t)a * n;
    for (int b = 0; b < k; ++b) {
      const ld* br = Wr + (size_t)b * n;
      const ld* bi = Wi + (size_t)b * n;
      ld sr = 0, si = 0;
      for (int i = 0; i < n; ++i) {
        sr += ar[i] * br[i] + ai[i] * bi[i];
        si += ar[i] * bi[i] - ai[i] * br[i];
      }
      if (a < k) {
        K[((size_t)a * k + b) * 2] = (double)sr;
        K[((size_t)a * k + b) * 2 + 1] = (double)si;
      } else {
        /* le_b = sum_i conj(W_ib) w_l,i = conj(sum_i conj(w_l,i) W_ib) */
        le[(size_t)b * 2] = (double)sr;
        le[(size_t)b * 2 + 1] = -(double)si;
      }
    }
  }
  for (int t = 0; t < 2; ++t) {
    /* |w_r|^2, then |w_l|^2 */
    const ld* zr = Wr + (size_t)(k + 1 - t) * n;
    const ld* zi = Wi + (size_t)(k + 1 - t) * n;
    ld s = 0;
    for (int i = 0; i < n; ++i) s += zr[i] * zr[i] + zi[i] * zi[i];
    norms[t] = (double)s;
  }
done:
  free(Lr);
  free(Li);
  free(Wr);
  free(Wi);
  return fail;
}
