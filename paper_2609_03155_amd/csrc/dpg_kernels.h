// Internal interface between the host API (dpg_api.cpp) and the HIP kernels
// (dpg_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace dpg {

// Device copies of the reference tables of one (p, dp) pair (see dpg_tables.h).
struct DevTables {
  int p, dp, s, r, n1, nq, nfq, N, Np, nc, m1, nu, nt1, nt, k, kp, nvp, nrows;
  int64_t ldz;             // leading dimension of a cell's workspace (nrows + 4: breaks power-of-two strides)
  int64_t zstride;         // complex elements between consecutive cells' workspaces
  const double* vol_w;     // [nq]
  const double* vol_pts;   // [nq][3]
  const double* vol_v;     // [nq][Np]
  const double* vol_c;     // [nq][Np][3]
  const int8_t* comp;      // [Np]
  const double* vol_phi;   // [nq][m1]
  const double* face_w;    // [6][nfq]
  const double* face_pts;  // [6][nfq][3]
  const double* face_v;    // [6][nfq][Np]
  const double* face_phi;  // [6][nfq][m1]
  const double* Cref;      // [N][N]
  const double* CrefT;     // [N][N] transpose
  const double* RtT;       // [6][N][N]  RtT[f][j][i] = Rt_f[i][j]
  const double* T;         // [6][N][nt1]
  const double* Tsum;      // [N][nt1] sum of T over the faces
  const double* sf_tab;    // [2][n1][n1] q_k(x_q) then q_k'(x_q), [k][q]: 1D factors of the test basis
  const double* sf_side;   // [2][n1] q_k(0), q_k(1)
  const double* sf_phi;    // [p+1][n1] 1D Lagrange factors of the DG basis at the Gauss points
  const double* sf_phis;   // [2][p+1] the same at 0 and 1
  int sf_cap;              // column tiles per chunk of the sum-factorised formation (4 or 8; autotuned)
};

// Per-call problem data (device pointers) plus derived scalars.
struct ProbArgs {
  const double* vertices;
  const int64_t* cells;
  const double* eps;
  const double* mu;
  const int8_t* face_kind;
  const double* zinv;
  double omega, alpha, inv_len;
  // TE_mn port
  int has_port;
  double pk1, pk2, pk3re, pk3im, pkc2, pmu_re, pmu_im;
};

// Per-chunk workspace of one degree group.
struct ChunkArgs {
  const int64_t* cell_ids;   // [n] global cell id per chunk-local cell
  int64_t n;                 // cells in the chunk
  double2* Z;                // [n][nvp cols][nrows] augmented lower factor, column-major
  double* dscale;            // [n][nvp] Jacobi scaling of the test rows
  double* met;               // [n][met_stride] point metrics: volume Gc|Gm (6 nq each), Robin-face Q (36 nfq),
                             // volume w det J^{-T} (9 nq, [a][c] = w det (J^{-1})_{ac}) and w J (9 nq)
  uint16_t* wsplit;          // split path: [n][6][kp][nvp] bf16 planes of W^H (re0,re1,re2,im0,im1,im2)
  double* fr;                // [n][fr_stride] real copy of the factorised F block (column-major, fr_ld), or null
  int split;                 // 1: K_aug from the bf16 split planes, eta by an FP64 reduction
  const int64_t* K_off;      // [n_cells+1] global output offsets (complex elements)
  const int64_t* v_off;
  int64_t cell_base;         // outputs are indexed relative to this cell (range solves)
  int64_t K_base, v_base;    // K_off[cell_base], v_off[cell_base]
  const double2* x;          // trial+trace coefficients, or null
  double2* K;                // outputs
  double2* l;
  double* eta;
  int32_t* info;
};

// Inputs of the condensation kernels: the local solve's K_e and l_e.
struct CondArgs {
  const double2* Ke;         // K_e of all cells (output layout of the local solve)
  const double2* le;
  const int64_t* Ke_off;     // [n_cells+1] K_off, v_off of the plan
  const int64_t* le_off;
  int64_t Ke_base, le_base;  // Ke_off[first], le_off[first] of the buffers' first cell
  int nu;                    // interior unknowns (first nu rows/columns of K_e)
  int kfull;                 // K_e dimension, nu + n_t
  // reconstruction only: the cells' local trace coefficients t_K (n_t each,
  // at tk_off[cell]) in, the whole coefficient vectors [u ; t_K] out (at
  // le_off[cell], the layout of l_e)
  const double2* tk;
  const int64_t* tk_off;
  double2* xout;
};

// Device data of one CG solve (CSR matrix, vectors, partial sums, scalars).
struct CgArgs {
  int64_t n;
  const int64_t* row_ptr;
  const int32_t* col;
  const double2* val;
  const double2* b;
  double2* x;                // start in, iterate out
  double2 *r, *p, *q;        // residual, direction, A p
  double* part;              // [cg_part_len(n)] partial sums of the reductions
  double* sc;                // [CG_NSC] iteration scalars
};
enum { CG_RR = 0, CG_ALPHA = 1, CG_BETA = 2, CG_BN2 = 3, CG_DONE = 4, CG_ITERS = 5, CG_TOL2 = 6, CG_NSC = 8 };

// Optional per-kernel timing: when `on`, each launch is bracketed by two HIP
// events recorded on the launch stream; `recs` keeps (class, begin, end).
struct Prof {
  bool on = false;
  struct Rec {
    int cls;
    hipEvent_t b, e;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int cls, hipStream_t st) {
    if (!on) return;
    Rec r{cls, take(), take()};
    (void)hipEventRecord(r.b, st);
    recs.push_back(r);
  }
  void end(hipStream_t st) {
    if (on && !recs.empty()) (void)hipEventRecord(recs.back().e, st);
  }
};

// Launchers (enqueue on `stream`, return the HIP launch status).
hipError_t launch_formation(const DevTables& t, const ProbArgs& pa, const ChunkArgs& ca, hipStream_t st,
                            Prof* prof = nullptr);
hipError_t launch_factor(const DevTables& t, const ChunkArgs& ca, hipStream_t st, Prof* prof = nullptr);
hipError_t launch_herk(const DevTables& t, const ChunkArgs& ca, hipStream_t st, Prof* prof = nullptr);
// Condensation A_K = M3 - M2^H M1^{-1} M2, b_K = l_t - M2^H M1^{-1} l_u: load of the
// augmented matrix into the workspace, and the final subtraction (the
// factorisation and HERK in between are launch_factor / launch_herk on the
// condensation tables).
hipError_t launch_cond_load(const DevTables& t, const ChunkArgs& ca, const CondArgs& a, hipStream_t st);
hipError_t launch_cond_finish(const DevTables& t, const ChunkArgs& ca, const CondArgs& a, hipStream_t st);
// to[z] = sum_{k in [ptr[z], ptr[z+1])} from[src[k]]  (assembly by gathering)
hipError_t launch_gather(int64_t n, const int64_t* ptr, const int64_t* src, const double2* from, double2* to,
                         hipStream_t st);
// y = A x for a complex CSR matrix
hipError_t launch_csr_matvec(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const double2* val,
                             const double2* x, double2* y, hipStream_t st);
// Reconstruction of the interior unknowns: load of D M1 D with the row
// (D (l_u - M2 t_K))^H appended, and the backward substitution after the
// factorisation (launch_factor on the reconstruction tables).
hipError_t launch_recon_load(const DevTables& t, const ChunkArgs& ca, const CondArgs& a, hipStream_t st);
hipError_t launch_recon_back(const DevTables& t, const ChunkArgs& ca, const CondArgs& a, hipStream_t st);
// out[i] = t[glob[i]] (0 where glob[i] < 0)
hipError_t launch_scatter(int64_t n, const int64_t* glob, const double2* t, double2* out, hipStream_t st);
// CG: doubles of the partial-sum buffer for n unknowns; r = b - A x, p = r and
// the start scalars (sc[CG_TOL2] and sc[CG_DONE] = 0 set by the caller); then
// `count` iterations
int64_t cg_part_len(int64_t n);
hipError_t launch_cg_start(const CgArgs& g, hipStream_t st);
hipError_t launch_cg_iterations(const CgArgs& g, int64_t count, hipStream_t st);
// Per-cell integrals {omega (eps_im |E|^2 + mu_im |H|^2) / 2, |E|^2, |H|^2} of
// the DG fields of x (v_off layout) into out[3 gc + .] for the n cells of one
// degree group (table t).
hipError_t launch_power(const DevTables& t, const ProbArgs& pa, const int64_t* cell_ids, int64_t n, const double2* x,
                        const int64_t* v_off, double* out, hipStream_t st);
// Dörfler marking: flags[i] = +1 (refine), -1 (coarsen) or 0 from values[i]
// (n cells).  Its temporaries: `workspace` (256-byte aligned, at least
// dorfler_mark_workspace(n) bytes; stream-ordered, no allocation; *too_small
// is set and nothing runs if it is smaller or misaligned), or, when
// workspace is null, an allocation of its own, after which the stream is
// synchronised.
hipError_t dorfler_mark_workspace(int64_t n, size_t* bytes);
hipError_t dorfler_mark(int64_t n, const double* values, double fr, double fc, int8_t* flags, void* workspace,
                        size_t workspace_bytes, hipStream_t st, bool* too_small);
// The same marking with its temporaries in a static device array of
// kMarkScratchBytes per GPU (no allocation, no synchronisation); n up to
// kMarkMaxCells.  *too_large is set (and nothing runs) when n or the
// temporaries exceed the array.  Calls that overlap on one GPU race.
constexpr size_t kMarkScratchBytes = (size_t)64 << 20;
constexpr int64_t kMarkMaxCells = (int64_t)1 << 20;
hipError_t dorfler_mark_noalloc(int64_t n, const double* values, double fr, double fc, int8_t* flags,
                                hipStream_t st, bool* too_large);
// doubles of per-point metrics kept per cell (ChunkArgs::met)
__host__ __device__ inline int64_t met_stride(const DevTables& t) { return 30 * (int64_t)t.nq + 36 * (int64_t)t.nfq; }
// real copy of the factorised F block (the leading 64 floor(Np/64) rows and
// columns): leading dimension (padded off a power of two) and doubles per cell
__host__ __device__ inline int64_t fr_ld(const DevTables& t) { return (int64_t)(t.Np / 64) * 64 + 4; }
__host__ __device__ inline int64_t fr_stride(const DevTables& t) { return fr_ld(t) * (t.Np / 64) * 64; }
// bf16 planes per cell of the split path
__host__ __device__ inline int64_t split_elems(const DevTables& t) { return 6 * (int64_t)t.kp * t.nvp; }
// Raise the dynamic-LDS limit of the kernels that stage whole tiles (once per process).
hipError_t configure_kernels();
// G, B_f, l of `n` cells into dense per-cell arrays (parity entries): unscaled,
// or, when rvec and dvec are given, the Jacobi-scaled D G D, D B_f, D l, D r and d.
hipError_t launch_extract(const DevTables& t, const ChunkArgs& ca, double2* G, double2* Bf, double2* lvec,
                          hipStream_t st, double2* rvec = nullptr, double* dvec = nullptr);

}  // namespace dpg
