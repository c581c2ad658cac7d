// Host side of the C ABI (include/dpg.h): plans, reference-table upload,
// workspace sizing and the stream-ordered launch sequence of the local solve.
#include "dpg.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <stdexcept>
#include <vector>

#include "dpg_kernels.h"
#include "dpg_tables.h"
#include "dpg_trace.h"

namespace {

constexpr double kC0 = 299792458.0;   // speed of light in vacuum (App. A scaling of omega)

struct DegreeGroup {
  int p = 0;
  dpg::Dims d{};
  dpg::DevTables dt{};
  std::vector<void*> bufs;            // device table allocations
  std::vector<int64_t> cells;         // global cell ids of this degree, ascending
  int64_t* cells_dev = nullptr;
  int64_t chunk = 0;                  // cells per chunk (workspace capacity)
  int64_t run_chunk = 0;              // cells per launch sequence (<= chunk; autotuned)
  double cost = 0.0;                  // algorithmic flops of all its cells (queue order)
  int64_t per_cell = 0;               // workspace bytes per cell
  // workspace of this group alone, so that groups can run concurrently
  double2* Z = nullptr;
  double* dscale = nullptr;
  double* met = nullptr;
  uint16_t* wsplit = nullptr;
  double* fr = nullptr;               // real copy of each cell's factorised F block
  hipStream_t stream = nullptr;       // branch stream of the concurrent schedule
  hipEvent_t done = nullptr;
  dpg::DevTables ct{};                // condensation: factorisation tables of the K_e-based matrix
  dpg::DevTables rt{};                // reconstruction: the same with the single right-hand-side row
};

// Algorithmic flops of one cell: the sum-factorised formation (per
// component pair and (i2, j2) block: the q2 and q1 passes and the (term, q0)
// GEMM of the S/M kernel, the same per (a, c) for D and R; G_IF from its
// tables), complex Cholesky, triangular solves, HERK and the two GEMVs; only
// their ratios matter here (queue order and workspace shares).
double cell_flops(int p, int dp) {
  const double s = p + dp + 1, r = p + 1;
  const double N = 3 * s * (s + 1) * (s + 1), nv = 2 * N, m1 = (p + 1.0) * (p + 1) * (p + 1);
  const double nu = 6 * m1, nt = 24 * r * r, k = nu + nt;
  const int Q1 = p + dp + 2, P1 = p + 1, S = Q1 - 1;
  auto n = [&](int comp, int d) { return (double)(comp == d ? S : Q1); };
  double form = 8.0 * N * N;
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b <= a; ++b) {
      const double R = n(a, 0) * n(b, 0), ncb = n(a, 1) * n(b, 1);
      const double nblk = a == b ? n(a, 2) * (n(a, 2) + 1) / 2 : n(a, 2) * n(b, 2);
      form += nblk * (15.0 * Q1 * Q1 * Q1 + 10 * ncb * Q1 * Q1 + 10 * R * ncb * Q1);
    }
    const double R = n(a, 0) * P1, ncb = n(a, 1) * P1, nblk = n(a, 2) * P1;
    form += 3 * nblk * (9.0 * Q1 * Q1 * Q1 + 6 * ncb * Q1 * Q1 + 6 * R * ncb * Q1);
  }
  return form + 4.0 / 3.0 * nv * nv * nv + 4 * nv * nv * nu + 2 * nv * nv * nt + 4 * k * k * nv + 32 * nv * k;
}

}  // namespace

struct dpg_plan_s {
  int device = 0;
  int dp = 1;
  int64_t n_cells = 0;
  std::vector<int64_t> K_off, v_off;
  int64_t* K_off_dev = nullptr;
  int64_t* v_off_dev = nullptr;
  std::vector<DegreeGroup> groups;    // in queue order: decreasing total cost
  std::vector<int8_t> degree;         // per cell (host)
  std::vector<int64_t> A_off, b_off;  // condensed cell matrices / right-hand sides (complex elements)
  int64_t* A_off_dev = nullptr;
  int64_t* b_off_dev = nullptr;
  double* cond_eta = nullptr;         // [n_cells] scratch of the condensation HERK
  std::vector<void*> misc;            // other device allocations
  hipEvent_t fork = nullptr;
  bool concurrent = true;             // degree groups on parallel branches
  dpg::Prof prof;
};

struct dpg_trace_system_s {
  int device = 0;
  int64_t n_cells = 0, n_dofs = 0, nnz = 0;
  std::vector<int64_t> glob;          // [b_off[n]] global id per local trace function, -1 removed
  int64_t* row_ptr = nullptr;         // device CSR structure
  int32_t* col = nullptr;
  int64_t* contrib_ptr = nullptr;     // device gather lists of the values and of the right-hand side
  int64_t* contrib = nullptr;
  int64_t* rhs_ptr = nullptr;
  int64_t* rhs_contrib = nullptr;
  int64_t* glob_dev = nullptr;        // device copy of glob (trace scatter)
  // CG on this system (dpg_trace_system_cg), allocated with it: the vectors
  // r, p, q, the partial sums and scalars, pinned host slots for the
  // scalars and two events
  double2* cg_vec = nullptr;
  double* cg_part = nullptr;
  double* cg_sc = nullptr;
  double* cg_host = nullptr;
  hipEvent_t cg_ev[2] = {nullptr, nullptr};
};

struct dpg_graph_s {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

struct HipError {
  hipError_t e;
};

thread_local char g_last_error[256] = "no error";

void set_error(const char* where, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
}

#define HIP_CHECK(call)                          \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) {                      \
      set_error(#call, e_);                      \
      throw HipError{e_};                        \
    }                                            \
  } while (0)

void hip_check(hipError_t e) {
  if (e != hipSuccess) {
    set_error("hip call", e);
    throw HipError{e};
  }
}

template <class T>
T* upload(std::vector<void*>& owner, const std::vector<T>& v) {
  T* p = nullptr;
  size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&p), bytes));
  owner.push_back(p);
  if (!v.empty()) HIP_CHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

void build_group(DegreeGroup& g, int dp) {
  dpg::RefTables rt = dpg::build_tables(g.p, dp);
  const dpg::Dims& d = rt.d;
  g.d = d;
  std::vector<double> CT((size_t)d.N * d.N), RtT((size_t)6 * d.N * d.N);
  for (int i = 0; i < d.N; ++i)
    for (int j = 0; j < d.N; ++j) CT[(size_t)j * d.N + i] = rt.Cref[(size_t)i * d.N + j];
  for (int f = 0; f < 6; ++f)
    for (int i = 0; i < d.N; ++i)
      for (int j = 0; j < d.N; ++j)
        RtT[((size_t)f * d.N + j) * d.N + i] = rt.Rt[((size_t)f * d.N + i) * d.N + j];
  const int nc = d.N / 3;
  dpg::DevTables& t = g.dt;
  t.p = d.p;
  t.dp = d.dp;
  t.s = d.s;
  t.r = d.r;
  t.n1 = d.n1;
  t.nq = d.nq;
  t.nfq = d.nfq;
  t.N = d.N;
  t.Np = d.Np;
  t.nc = nc;
  t.m1 = d.m1;
  t.nu = d.nu;
  t.nt1 = d.nt1;
  t.nt = d.nt;
  t.k = d.k;
  t.kp = d.kp;
  t.nvp = d.nvp;
  t.nrows = d.nrows;
  // Padded strides: columns and cells would otherwise sit at power-of-two
  // distances (16 KiB, multiples of 2 MiB), which maps concurrent tiles onto
  // the same HBM channels.
  t.ldz = d.nrows + 4;
  t.zstride = t.ldz * d.nvp + 36;
  t.vol_w = upload(g.bufs, rt.vol_w);
  t.vol_pts = upload(g.bufs, rt.vol_pts);
  t.vol_v = upload(g.bufs, rt.vol_v);
  t.vol_c = upload(g.bufs, rt.vol_c);
  t.comp = upload(g.bufs, rt.comp);
  t.vol_phi = upload(g.bufs, rt.vol_phi);
  t.face_w = upload(g.bufs, rt.face_w);
  t.face_pts = upload(g.bufs, rt.face_pts);
  t.face_v = upload(g.bufs, rt.face_v);
  t.face_phi = upload(g.bufs, rt.face_phi);
  t.Cref = upload(g.bufs, rt.Cref);
  t.CrefT = upload(g.bufs, CT);
  t.RtT = upload(g.bufs, RtT);
  t.T = upload(g.bufs, rt.T);
  {
    // the trace pairing summed over the six faces (cells without Robin faces use it as is)
    std::vector<double> ts((size_t)d.N * d.nt1, 0.0);
    for (int f = 0; f < 6; ++f)
      for (size_t e = 0; e < ts.size(); ++e) ts[e] += rt.T[(size_t)f * ts.size() + e];
    t.Tsum = upload(g.bufs, ts);
  }
  t.sf_tab = upload(g.bufs, rt.sf_tab);
  t.sf_side = upload(g.bufs, rt.sf_side);
  t.sf_phi = upload(g.bufs, rt.sf_phi);
  t.sf_phis = upload(g.bufs, rt.sf_phis);
  t.sf_cap = 8;
}

void free_plan(dpg_plan_s* p) {
  if (!p) return;
  for (auto& g : p->groups) {
    for (void* b : g.bufs) (void)hipFree(b);
    if (g.cells_dev) (void)hipFree(g.cells_dev);
    if (g.Z) (void)hipFree(g.Z);
    if (g.dscale) (void)hipFree(g.dscale);
    if (g.met) (void)hipFree(g.met);
    if (g.wsplit) (void)hipFree(g.wsplit);
    if (g.fr) (void)hipFree(g.fr);
    if (g.stream) (void)hipStreamDestroy(g.stream);
    if (g.done) (void)hipEventDestroy(g.done);
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
  for (void* b : p->misc) (void)hipFree(b);
  for (auto& r : p->prof.recs) {
    (void)hipEventDestroy(r.b);
    (void)hipEventDestroy(r.e);
  }
  for (auto e : p->prof.pool) (void)hipEventDestroy(e);
  delete p;
}

bool make_prob_args(const dpg_problem* pr, dpg::ProbArgs& pa) {
  if (!pr || pr->n_cells < 0) return false;
  if (pr->n_cells > 0 && (!pr->vertices || !pr->cells || !pr->eps || !pr->mu || !pr->face_kind || !pr->zinv))
    return false;
  if (!(pr->freq_hz > 0.0) || !(pr->length_m > 0.0) || !(pr->alpha > 0.0)) return false;
  pa.vertices = pr->vertices;
  pa.cells = pr->cells;
  pa.eps = pr->eps;
  pa.mu = pr->mu;
  pa.face_kind = pr->face_kind;
  pa.zinv = pr->zinv;
  pa.omega = pr->length_m * 2.0 * M_PI * pr->freq_hz / kC0;
  pa.alpha = pr->alpha;
  pa.inv_len = 1.0 / pr->length_m;
  const dpg_port& po = pr->port;
  pa.has_port = 0;
  pa.pk1 = pa.pk2 = pa.pk3re = pa.pk3im = pa.pkc2 = 0.0;
  pa.pmu_re = po.mu_re;
  pa.pmu_im = po.mu_im;
  if (po.a > 0.0 && po.b > 0.0 && (po.m > 0 || po.n > 0)) {
    pa.pk1 = po.m * M_PI / po.a;
    pa.pk2 = po.n * M_PI / po.b;
    pa.pkc2 = pa.pk1 * pa.pk1 + pa.pk2 * pa.pk2;
    std::complex<double> eps(po.eps_re, po.eps_im), mu(po.mu_re, po.mu_im);
    std::complex<double> k3 = std::sqrt(pa.omega * pa.omega * eps * mu - pa.pkc2);
    pa.pk3re = k3.real();
    pa.pk3im = k3.imag();
    pa.has_port = 1;
  }
  return true;
}

dpg_status check_solve_args(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count, const double* K,
                            const double* l, const double* eta, const int32_t* info, int32_t precision,
                            dpg::ProbArgs& pa) {
  if (!plan || first < 0 || count < 0 || first + count > plan->n_cells) return DPG_ERR_ARG;
  if (count > 0 && (!K || !l || !eta || !info)) return DPG_ERR_ARG;
  if (precision != DPG_FP64 && precision != DPG_SPLIT_FP32) return DPG_ERR_ARG;
  if (!make_prob_args(prob, pa) || prob->n_cells != plan->n_cells) return DPG_ERR_ARG;
  return DPG_OK;
}

// Enqueues the local solve of cells [first, first + count) on `st`.  Degree
// groups are taken in queue order (decreasing cost); with concurrency on and
// more than one group in the range, each group runs on its own branch
// stream, forked from and joined back into `st` with events, so that the
// launches of cheap degrees fill the tails of the expensive ones.  Under
// stream capture the branches become parallel branches of the graph.
dpg_status enqueue_solve(dpg_plan P, const dpg::ProbArgs& pa, int64_t first, int64_t count, const double* x,
                         double* K, double* l, double* eta, int32_t* info, int32_t precision, hipStream_t st,
                         bool profile) {
  struct Job {
    DegreeGroup* g;
    int64_t lo, hi;
  };
  std::vector<Job> jobs;
  for (auto& g : P->groups) {
    // this degree's cells inside [first, first + count): a contiguous run of its sorted list
    const int64_t lo = std::lower_bound(g.cells.begin(), g.cells.end(), first) - g.cells.begin();
    const int64_t hi = std::lower_bound(g.cells.begin(), g.cells.end(), first + count) - g.cells.begin();
    if (hi > lo) jobs.push_back({&g, lo, hi});
  }
  const bool par = P->concurrent && jobs.size() > 1;
  hipError_t e = hipSuccess;
  if (par) e = hipEventRecord(P->fork, st);
  for (const Job& jb : jobs) {
    DegreeGroup& g = *jb.g;
    hipStream_t s = par ? g.stream : st;
    if (par && e == hipSuccess) e = hipStreamWaitEvent(s, P->fork, 0);
    for (int64_t s0 = jb.lo; s0 < jb.hi && e == hipSuccess; s0 += g.run_chunk) {
      dpg::ChunkArgs ca{};
      ca.cell_ids = g.cells_dev + s0;
      ca.n = std::min<int64_t>(g.run_chunk, jb.hi - s0);
      ca.Z = g.Z;
      ca.dscale = g.dscale;
      ca.met = g.met;
      ca.wsplit = g.wsplit;
      ca.fr = g.fr;
      ca.split = precision == DPG_SPLIT_FP32 ? 1 : 0;
      ca.K_off = P->K_off_dev;
      ca.v_off = P->v_off_dev;
      ca.cell_base = first;
      ca.K_base = P->K_off[first];
      ca.v_base = P->v_off[first];
      ca.x = reinterpret_cast<const double2*>(x);
      ca.K = reinterpret_cast<double2*>(K);
      ca.l = reinterpret_cast<double2*>(l);
      ca.eta = eta;
      ca.info = info;
      dpg::Prof* pr = profile ? &P->prof : nullptr;
      e = dpg::launch_formation(g.dt, pa, ca, s, pr);
      if (e == hipSuccess) e = dpg::launch_factor(g.dt, ca, s, pr);
      if (e == hipSuccess) e = dpg::launch_herk(g.dt, ca, s, pr);
    }
    if (par && e == hipSuccess) e = hipEventRecord(g.done, s);
  }
  if (par)
    for (const Job& jb : jobs)
      if (e == hipSuccess) e = hipStreamWaitEvent(st, jb.g->done, 0);
  if (e != hipSuccess) {
    set_error("dpg local solve enqueue", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

// Formation of `count` consecutive cells of one degree and extraction of
// their dense local matrices (the parity entries): unscaled G, B_f, l, or,
// with rvec and dvec, the Jacobi-scaled system the factorisation reads.
dpg_status form_cells(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count, const double* x,
                      double* G, double* Bf, double* lvec, double* rvec, double* dvec, int32_t* info, void* stream) {
  if (!plan || !G || !Bf || !lvec || !info || first < 0 || count <= 0 || first + count > plan->n_cells)
    return DPG_ERR_ARG;
  dpg::ProbArgs pa;
  if (!make_prob_args(prob, pa) || prob->n_cells != plan->n_cells) return DPG_ERR_ARG;
  DegreeGroup* grp = nullptr;
  for (auto& g : plan->groups) {
    bool all = true;
    for (int64_t c = first; c < first + count && all; ++c) {
      auto it = std::lower_bound(g.cells.begin(), g.cells.end(), c);
      all = (it != g.cells.end() && *it == c);
    }
    if (all) {
      grp = &g;
      break;
    }
  }
  if (!grp) return DPG_ERR_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
  std::vector<int64_t> ids(count);
  for (int64_t c = 0; c < count; ++c) ids[c] = first + c;
  int64_t* ids_dev = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&ids_dev), sizeof(int64_t) * count) != hipSuccess) return DPG_ERR_ALLOC;
  dpg_status rc = DPG_OK;
  if (hipMemcpyAsync(ids_dev, ids.data(), sizeof(int64_t) * count, hipMemcpyHostToDevice, st) != hipSuccess)
    rc = DPG_ERR_HIP;
  const dpg::Dims& d = grp->d;
  const int64_t nv = 2 * d.N;
  const bool scaled = rvec && dvec;
  for (int64_t s0 = 0; s0 < count && rc == DPG_OK; s0 += grp->chunk) {
    dpg::ChunkArgs ca{};
    ca.cell_ids = ids_dev + s0;
    ca.n = std::min<int64_t>(grp->chunk, count - s0);
    ca.Z = grp->Z;
    ca.dscale = grp->dscale;
    ca.met = grp->met;
    ca.fr = grp->fr;   // the formation writes the real F block there
    ca.K_off = plan->K_off_dev;
    ca.v_off = plan->v_off_dev;
    ca.cell_base = first;
    ca.v_base = plan->v_off[first];
    ca.x = reinterpret_cast<const double2*>(x);
    ca.info = info;
    if (dpg::launch_formation(grp->dt, pa, ca, st) != hipSuccess ||
        dpg::launch_extract(grp->dt, ca, reinterpret_cast<double2*>(G) + s0 * nv * nv,
                            reinterpret_cast<double2*>(Bf) + s0 * nv * d.k,
                            reinterpret_cast<double2*>(lvec) + s0 * nv, st,
                            scaled ? reinterpret_cast<double2*>(rvec) + s0 * nv : nullptr,
                            scaled ? dvec + s0 * nv : nullptr) != hipSuccess)
      rc = DPG_ERR_HIP;
  }
  // the id buffer must outlive the enqueued work
  if (hipStreamSynchronize(st) != hipSuccess) rc = DPG_ERR_HIP;
  (void)hipFree(ids_dev);
  return rc;
}

}  // namespace

extern "C" {

const char* dpg_last_error(void) { return g_last_error; }

const char* dpg_status_string(dpg_status s) {
  switch (s) {
    case DPG_OK: return "ok";
    case DPG_ERR_ARG: return "invalid argument";
    case DPG_ERR_ALLOC: return "allocation failed";
    case DPG_ERR_HIP: return "HIP runtime error";
    case DPG_ERR_UNSUPPORTED: return "unsupported request";
    case DPG_ERR_CELL: return "a cell failed (see info[])";
  }
  return "unknown status";
}

dpg_status dpg_sync(void* stream, const int32_t* info, int64_t n, int64_t* n_failed, int64_t* first_failed) {
  if (n_failed) *n_failed = 0;
  if (first_failed) *first_failed = -1;
  if (n < 0 || (n > 0 && !info)) return DPG_ERR_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("dpg_sync: stream", e);
    return DPG_ERR_HIP;
  }
  if (n == 0) return DPG_OK;
  std::vector<int32_t> h((size_t)n);
  e = hipMemcpyAsync(h.data(), info, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_error("dpg_sync: info", e);
    return DPG_ERR_HIP;
  }
  int64_t cnt = 0, first = -1;
  for (int64_t c = 0; c < n; ++c)
    if (h[(size_t)c] != 0) {
      if (first < 0) first = c;
      ++cnt;
    }
  if (n_failed) *n_failed = cnt;
  if (first_failed) *first_failed = first;
  return cnt ? DPG_ERR_CELL : DPG_OK;
}

dpg_status dpg_local_dims(int32_t p, int32_t dp, int32_t* n_test, int32_t* n_interior, int32_t* n_trace) {
  if (p < 1 || p > 4 || dp < 1 || dp > 2 || !n_test || !n_interior || !n_trace) return DPG_ERR_ARG;
  const int s = p + dp + 1, r = p + 1;
  *n_test = 6 * s * (s + 1) * (s + 1);
  *n_interior = 6 * (p + 1) * (p + 1) * (p + 1);
  *n_trace = 24 * r * r;
  return DPG_OK;
}

dpg_status dpg_plan_create(int32_t device, const int8_t* degree_host, int64_t n_cells, int32_t dp,
                           int64_t max_workspace_bytes, dpg_plan* plan) {
  if (!plan || n_cells < 0 || (n_cells > 0 && !degree_host) || dp < 1 || dp > 2 || max_workspace_bytes < 0)
    return DPG_ERR_ARG;
  *plan = nullptr;
  for (int64_t c = 0; c < n_cells; ++c)
    if (degree_host[c] < 1 || degree_host[c] > 4) return DPG_ERR_ARG;
  dpg_plan_s* P = nullptr;
  try {
    if (hipSetDevice(device) != hipSuccess) return DPG_ERR_ARG;
    HIP_CHECK(dpg::configure_kernels());
    P = new dpg_plan_s();
    P->device = device;
    P->dp = dp;
    P->n_cells = n_cells;
    P->K_off.resize(n_cells + 1);
    P->v_off.resize(n_cells + 1);
    P->K_off[0] = P->v_off[0] = 0;
    for (int64_t c = 0; c < n_cells; ++c) {
      const int p = degree_host[c];
      const int64_t k = 6 * (int64_t)(p + 1) * (p + 1) * (p + 1) + 24 * (int64_t)(p + 1) * (p + 1);
      P->K_off[c + 1] = P->K_off[c] + k * k;
      P->v_off[c + 1] = P->v_off[c] + k;
    }
    P->K_off_dev = upload(P->misc, P->K_off);
    P->v_off_dev = upload(P->misc, P->v_off);
    P->degree.assign(degree_host, degree_host + n_cells);
    P->A_off.assign(n_cells + 1, 0);
    P->b_off.assign(n_cells + 1, 0);
    for (int64_t c = 0; c < n_cells; ++c) {
      const int64_t r = degree_host[c] + 1, nt = 24 * r * r;
      P->A_off[c + 1] = P->A_off[c] + nt * nt;
      P->b_off[c + 1] = P->b_off[c] + nt;
    }
    P->A_off_dev = upload(P->misc, P->A_off);
    P->b_off_dev = upload(P->misc, P->b_off);
    P->cond_eta = upload(P->misc, std::vector<double>(std::max<int64_t>(1, n_cells), 0.0));
    for (int p = 1; p <= 4; ++p) {
      DegreeGroup g;
      g.p = p;
      for (int64_t c = 0; c < n_cells; ++c)
        if (degree_host[c] == p) g.cells.push_back(c);
      if (g.cells.empty()) continue;
      build_group(g, dp);
      {
        // condensation matrix: columns = interior unknowns (padded to 64),
        // rows below = (D M2)^H, (D l_u)^H; every tile complex (Np = 0)
        dpg::DevTables& c = g.ct;
        c = g.dt;
        const int nt = g.d.nt;
        c.Np = 0;
        c.nvp = (g.d.nu + 63) / 64 * 64;
        c.k = nt;
        c.kp = (nt + 2 + 63) / 64 * 64;
        c.nrows = c.nvp + c.kp;
        c.ldz = c.nrows + 4;
        c.zstride = c.ldz * c.nvp + 36;
        if (c.zstride > g.dt.zstride) throw std::bad_alloc();
        // reconstruction matrix: the same columns, one row block below them
        // whose first row is (D (l_u - M2 t_K))^H
        dpg::DevTables& r = g.rt;
        r = c;
        r.k = 0;
        r.kp = 64;
        r.nrows = r.nvp + r.kp;
        r.ldz = r.nrows + 4;
        r.zstride = r.ldz * r.nvp + 36;
      }
      std::vector<void*> tmp;
      g.cells_dev = upload(tmp, g.cells);
      P->groups.push_back(std::move(g));
    }
    // queue order: most expensive degree first
    for (auto& g : P->groups) g.cost = cell_flops(g.p, dp) * (double)g.cells.size();
    std::stable_sort(P->groups.begin(), P->groups.end(),
                     [](const DegreeGroup& a, const DegreeGroup& b) { return a.cost > b.cost; });
    size_t free_b = 0, total_b = 0;
    HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
    const double budget = max_workspace_bytes > 0 ? (double)max_workspace_bytes : 0.4 * (double)free_b;
    for (auto& g : P->groups) {
      const int64_t mper = dpg::met_stride(g.dt);
      g.per_cell = g.dt.zstride * 16 + (int64_t)g.d.nvp * 8 + mper * 8 + dpg::split_elems(g.dt) * 2 +
                   dpg::fr_stride(g.dt) * 8;
    }
    // Each group first gets room for enough cells that one factorisation step
    // has about kFillTiles row tiles (a few waves of workgroups on every CU),
    // so that even a cheap degree's launches fill the device; the rest of the
    // budget is shared in proportion to cost, capped at what all a group's
    // cells need (water filling over the remaining groups).
    constexpr int64_t kFillTiles = 16384;
    std::vector<int64_t> base_cells(P->groups.size());
    double base = 0.0;
    for (size_t q = 0; q < P->groups.size(); ++q) {
      const DegreeGroup& g = P->groups[q];
      const int64_t fill = std::max<int64_t>(64, kFillTiles / (g.d.nrows / 64));
      base_cells[q] = std::min<int64_t>(fill, (int64_t)g.cells.size());
      base += (double)g.per_cell * (double)base_cells[q];
    }
    const double bscale = base > budget ? budget / base : 1.0;
    for (auto& b : base_cells) b = (int64_t)(bscale * (double)b);
    std::vector<int> open(P->groups.size());
    for (size_t q = 0; q < open.size(); ++q) open[q] = (int)q;
    double left = std::max(0.0, budget - bscale * base);
    for (bool capped = true; capped && !open.empty();) {
      capped = false;
      double csum = 0.0;
      for (int q : open) csum += P->groups[q].cost;
      std::vector<int> keep;
      double used = 0.0;
      for (int q : open) {
        DegreeGroup& g = P->groups[q];
        const double need = (double)g.per_cell * (double)(g.cells.size() - base_cells[q]);
        if (left * g.cost / csum >= need) {
          g.chunk = (int64_t)g.cells.size();
          used += need;
          capped = true;
        } else {
          keep.push_back(q);
        }
      }
      if (capped) {
        left -= used;
        open.swap(keep);
      } else {
        for (int q : open) {
          DegreeGroup& g = P->groups[q];
          const int64_t ch = base_cells[q] + (int64_t)(left * g.cost / csum / (double)g.per_cell);
          g.chunk = std::max<int64_t>(1, std::min<int64_t>(ch, (int64_t)g.cells.size()));
        }
      }
    }
    for (auto& g : P->groups) {
      g.run_chunk = g.chunk;
      const int64_t mper = dpg::met_stride(g.dt);
      if (hipMalloc(reinterpret_cast<void**>(&g.Z), (size_t)g.chunk * g.dt.zstride * 16) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&g.dscale), (size_t)g.chunk * g.d.nvp * 8) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&g.met), (size_t)g.chunk * mper * 8) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&g.wsplit), (size_t)g.chunk * dpg::split_elems(g.dt) * 2) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&g.fr), (size_t)g.chunk * dpg::fr_stride(g.dt) * 8) != hipSuccess) {
        free_plan(P);
        return DPG_ERR_ALLOC;
      }
      HIP_CHECK(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
      HIP_CHECK(hipEventCreateWithFlags(&g.done, hipEventDisableTiming));
    }
    HIP_CHECK(hipEventCreateWithFlags(&P->fork, hipEventDisableTiming));
    *plan = P;
    return DPG_OK;
  } catch (const HipError&) {
    free_plan(P);
    return DPG_ERR_HIP;
  } catch (const std::bad_alloc&) {
    free_plan(P);
    return DPG_ERR_ALLOC;
  } catch (...) {
    free_plan(P);
    return DPG_ERR_ARG;
  }
}

dpg_status dpg_plan_destroy(dpg_plan plan) {
  if (!plan) return DPG_ERR_ARG;
  (void)hipSetDevice(plan->device);
  free_plan(plan);
  return DPG_OK;
}

dpg_status dpg_plan_offsets(dpg_plan plan, int64_t* K_off, int64_t* v_off) {
  if (!plan || !K_off || !v_off) return DPG_ERR_ARG;
  std::memcpy(K_off, plan->K_off.data(), sizeof(int64_t) * plan->K_off.size());
  std::memcpy(v_off, plan->v_off.data(), sizeof(int64_t) * plan->v_off.size());
  return DPG_OK;
}

dpg_status dpg_plan_layout(dpg_plan plan, int32_t p, int64_t* n_test_padded, int64_t* n_rhs_padded,
                           int64_t* chunk_cells) {
  if (!plan || !n_test_padded || !n_rhs_padded || !chunk_cells) return DPG_ERR_ARG;
  for (auto& g : plan->groups)
    if (g.p == p) {
      *n_test_padded = g.d.nvp;
      *n_rhs_padded = g.d.kp;
      *chunk_cells = g.chunk;
      return DPG_OK;
    }
  return DPG_ERR_ARG;
}

dpg_status dpg_local_solve_range(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count,
                                 const double* x, double* K, double* l, double* eta, int32_t* info,
                                 int32_t precision, void* stream) {
  dpg::ProbArgs pa;
  const dpg_status rc = check_solve_args(plan, prob, first, count, K, l, eta, info, precision, pa);
  if (rc != DPG_OK || count == 0) return rc;
  if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
  return enqueue_solve(plan, pa, first, count, x, K, l, eta, info, precision,
                       reinterpret_cast<hipStream_t>(stream), plan->prof.on);
}

dpg_status dpg_local_solve(dpg_plan plan, const dpg_problem* prob, const double* x, double* K, double* l,
                           double* eta, int32_t* info, int32_t precision, void* stream) {
  if (!plan) return DPG_ERR_ARG;
  if (plan->n_cells > 0 && (!K || !l || !eta || !info)) return DPG_ERR_ARG;
  return dpg_local_solve_range(plan, prob, 0, plan->n_cells, x, K, l, eta, info, precision, stream);
}

dpg_status dpg_plan_set_concurrency(dpg_plan plan, int32_t enable) {
  if (!plan) return DPG_ERR_ARG;
  plan->concurrent = enable != 0;
  return DPG_OK;
}

dpg_status dpg_plan_autotune(dpg_plan plan, const dpg_problem* prob, const double* x, double* K, double* l,
                             double* eta, int32_t* info, int32_t precision, void* stream, double* best_ms) {
  dpg::ProbArgs pa;
  dpg_status rc = check_solve_args(plan, prob, 0, plan ? plan->n_cells : 0, K, l, eta, info, precision, pa);
  if (rc != DPG_OK) return rc;
  if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return DPG_ERR_HIP;
  // Times one whole solve with the plan's current settings.
  auto timed = [&](float& ms) -> dpg_status {
    ms = 0.f;
    if (hipEventRecord(t0, st) != hipSuccess) return DPG_ERR_HIP;
    const dpg_status r = enqueue_solve(plan, pa, 0, plan->n_cells, x, K, l, eta, info, precision, st, false);
    if (r != DPG_OK) return r;
    if (hipEventRecord(t1, st) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
        hipEventElapsedTime(&ms, t0, t1) != hipSuccess)
      return DPG_ERR_HIP;
    return DPG_OK;
  };
  const bool conc0 = plan->concurrent;
  float best = 0.f;
  {
    float warm = 0.f;   // first touch of tables, workspace and outputs
    rc = timed(warm);
  }
  // 1. cells per launch sequence of each degree group, the others fixed
  plan->concurrent = false;
  for (auto& g : plan->groups) {
    if (rc != DPG_OK) break;
    int64_t cand[3] = {g.chunk, (g.chunk + 1) / 2, (g.chunk + 3) / 4};
    int64_t pick = g.chunk;
    float pick_ms = 0.f;
    for (int c = 0; c < 3 && rc == DPG_OK; ++c) {
      if (c > 0 && cand[c] == cand[c - 1]) continue;
      g.run_chunk = cand[c];
      float ms = 0.f;
      rc = timed(ms);
      if (rc == DPG_OK && (c == 0 || ms < pick_ms)) {
        pick_ms = ms;
        pick = cand[c];
      }
    }
    g.run_chunk = pick;
    best = pick_ms;
  }
  // 2. tile shape of the sum-factorised formation of each group: column
  // tiles per chunk (8, or 4: less LDS, more workgroups per CU)
  for (auto& g : plan->groups) {
    if (rc != DPG_OK) break;
    const int cand[2] = {8, 4};
    int pick = g.dt.sf_cap;
    float pick_ms = 0.f;
    for (int c = 0; c < 2 && rc == DPG_OK; ++c) {
      g.dt.sf_cap = cand[c];
      float ms = 0.f;
      rc = timed(ms);
      if (rc == DPG_OK && (c == 0 || ms < pick_ms)) {
        pick_ms = ms;
        pick = cand[c];
      }
    }
    g.dt.sf_cap = pick;
    best = pick_ms;
  }
  // 3. concurrent degree branches or one stream
  if (rc == DPG_OK && plan->groups.size() > 1) {
    plan->concurrent = true;
    float ms = 0.f;
    rc = timed(ms);
    if (rc == DPG_OK) {
      if (ms < best) best = ms;
      else plan->concurrent = false;
    }
  }
  if (rc != DPG_OK) plan->concurrent = conc0;
  // leave the outputs of the chosen settings
  float ms = 0.f;
  if (rc == DPG_OK) rc = timed(ms);
  if (best_ms) *best_ms = rc == DPG_OK ? (double)ms : 0.0;
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  return rc;
}

dpg_status dpg_plan_tiles(dpg_plan plan, int32_t p, int32_t* form_col_tiles) {
  if (!plan || !form_col_tiles) return DPG_ERR_ARG;
  for (auto& g : plan->groups)
    if (g.p == p) {
      *form_col_tiles = g.dt.sf_cap;
      return DPG_OK;
    }
  return DPG_ERR_ARG;
}

dpg_status dpg_plan_set_tiles(dpg_plan plan, int32_t p, int32_t form_col_tiles) {
  if (!plan || (form_col_tiles != 4 && form_col_tiles != 8)) return DPG_ERR_ARG;
  for (auto& g : plan->groups)
    if (g.p == p) {
      g.dt.sf_cap = form_col_tiles;
      return DPG_OK;
    }
  return DPG_ERR_ARG;
}

dpg_status dpg_plan_tuning(dpg_plan plan, int32_t p, int64_t* run_chunk, int32_t* concurrent) {
  if (!plan || !run_chunk || !concurrent) return DPG_ERR_ARG;
  for (auto& g : plan->groups)
    if (g.p == p) {
      *run_chunk = g.run_chunk;
      *concurrent = plan->concurrent ? 1 : 0;
      return DPG_OK;
    }
  return DPG_ERR_ARG;
}

dpg_status dpg_graph_create(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count, const double* x,
                            double* K, double* l, double* eta, int32_t* info, int32_t precision, dpg_graph* out) {
  if (!out) return DPG_ERR_ARG;
  *out = nullptr;
  dpg::ProbArgs pa;
  dpg_status rc = check_solve_args(plan, prob, first, count, K, l, eta, info, precision, pa);
  if (rc != DPG_OK) return rc;
  if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
  dpg_graph_s* G = new (std::nothrow) dpg_graph_s();
  if (!G) return DPG_ERR_ALLOC;
  G->device = plan->device;
  if (count > 0) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      rc = enqueue_solve(plan, pa, first, count, x, K, l, eta, info, precision, cs, false);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cs, &g);   // always ends the capture
      G->graph = g;
      if (e == hipSuccess && rc == DPG_OK) e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
      set_error("dpg_graph_create", e);
      if (rc == DPG_OK) rc = DPG_ERR_HIP;
    }
  }
  if (rc != DPG_OK) {
    (void)dpg_graph_destroy(G);
    return rc;
  }
  *out = G;
  return DPG_OK;
}

dpg_status dpg_graph_launch(dpg_graph graph, void* stream) {
  if (!graph) return DPG_ERR_ARG;
  if (!graph->exec) return DPG_OK;   // empty range
  if (hipSetDevice(graph->device) != hipSuccess) return DPG_ERR_HIP;
  const hipError_t e = hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_error("dpg_graph_launch", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

dpg_status dpg_graph_destroy(dpg_graph graph) {
  if (!graph) return DPG_ERR_ARG;
  (void)hipSetDevice(graph->device);
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return DPG_OK;
}

dpg_status dpg_plan_trace_offsets(dpg_plan plan, int64_t* A_off, int64_t* b_off) {
  if (!plan || !A_off || !b_off) return DPG_ERR_ARG;
  std::memcpy(A_off, plan->A_off.data(), sizeof(int64_t) * plan->A_off.size());
  std::memcpy(b_off, plan->b_off.data(), sizeof(int64_t) * plan->b_off.size());
  return DPG_OK;
}

dpg_status dpg_condense(dpg_plan plan, const double* K, const double* l, double* A, double* b, int32_t* info,
                        void* stream) {
  if (!plan) return DPG_ERR_ARG;
  if (plan->n_cells == 0) return DPG_OK;
  if (!K || !l || !A || !b || !info) return DPG_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  for (auto& g : plan->groups) {
    const int64_t nc = (int64_t)g.cells.size();
    for (int64_t s0 = 0; s0 < nc && e == hipSuccess; s0 += g.chunk) {
      dpg::ChunkArgs ca{};
      ca.cell_ids = g.cells_dev + s0;
      ca.n = std::min<int64_t>(g.chunk, nc - s0);
      ca.Z = g.Z;
      ca.split = 0;
      ca.K_off = plan->A_off_dev;
      ca.v_off = plan->b_off_dev;
      ca.K = reinterpret_cast<double2*>(A);
      ca.l = reinterpret_cast<double2*>(b);
      ca.eta = plan->cond_eta;
      ca.info = info;
      dpg::CondArgs cg{};
      cg.Ke = reinterpret_cast<const double2*>(K);
      cg.le = reinterpret_cast<const double2*>(l);
      cg.Ke_off = plan->K_off_dev;
      cg.le_off = plan->v_off_dev;
      cg.nu = g.d.nu;
      cg.kfull = g.d.k;
      e = dpg::launch_cond_load(g.ct, ca, cg, st);
      if (e == hipSuccess) e = dpg::launch_factor(g.ct, ca, st, nullptr);
      if (e == hipSuccess) e = dpg::launch_herk(g.ct, ca, st, nullptr);
      if (e == hipSuccess) e = dpg::launch_cond_finish(g.ct, ca, cg, st);
    }
  }
  if (e != hipSuccess) {
    set_error("dpg_condense", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

dpg_status dpg_trace_numbering(const int64_t* cells_host, const int8_t* face_kind_host, const int8_t* degree_host,
                               int64_t n_cells, int64_t* glob, int64_t* n_dofs) {
  if (n_cells < 0 || !n_dofs || (n_cells > 0 && (!cells_host || !face_kind_host || !degree_host || !glob)))
    return DPG_ERR_ARG;
  for (int64_t c = 0; c < n_cells; ++c)
    if (degree_host[c] < 1 || degree_host[c] > 4) return DPG_ERR_ARG;
  try {
    std::vector<int64_t> toff, g;
    dpg::trace_numbering(cells_host, face_kind_host, degree_host, n_cells, toff, g, *n_dofs);
    if (!g.empty()) std::memcpy(glob, g.data(), sizeof(int64_t) * g.size());
    return DPG_OK;
  } catch (const std::invalid_argument&) {
    return DPG_ERR_ARG;
  } catch (const std::bad_alloc&) {
    return DPG_ERR_ALLOC;
  }
}

dpg_status dpg_trace_system_create(dpg_plan plan, const int64_t* cells_host, const int8_t* face_kind_host,
                                   dpg_trace_system* out) {
  if (!plan || !out || (plan->n_cells > 0 && (!cells_host || !face_kind_host))) return DPG_ERR_ARG;
  *out = nullptr;
  dpg_trace_system_s* S = nullptr;
  try {
    if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
    S = new dpg_trace_system_s();
    S->device = plan->device;
    S->n_cells = plan->n_cells;
    std::vector<int64_t> toff;
    dpg::trace_numbering(cells_host, face_kind_host, plan->degree.data(), plan->n_cells, toff, S->glob, S->n_dofs);
    std::vector<int64_t> row_ptr, cptr, contrib, rptr, rcontrib;
    std::vector<int32_t> col;
    dpg::trace_csr(toff, S->glob, plan->A_off, plan->b_off, S->n_dofs, row_ptr, col, cptr, contrib, rptr, rcontrib);
    S->nnz = (int64_t)col.size();
    std::vector<void*> own;
    S->row_ptr = upload(own, row_ptr);
    S->col = upload(own, col);
    S->contrib_ptr = upload(own, cptr);
    S->contrib = upload(own, contrib);
    S->rhs_ptr = upload(own, rptr);
    S->rhs_contrib = upload(own, rcontrib);
    S->glob_dev = upload(own, S->glob);
    if (S->n_dofs > 0) {
      HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&S->cg_vec), sizeof(double2) * 3 * S->n_dofs));
      HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&S->cg_part), sizeof(double) * dpg::cg_part_len(S->n_dofs)));
      HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&S->cg_sc), sizeof(double) * dpg::CG_NSC));
      HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&S->cg_host), sizeof(double) * 3 * dpg::CG_NSC,
                              hipHostMallocDefault));
      for (auto& e : S->cg_ev) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    *out = S;
    return DPG_OK;
  } catch (const std::invalid_argument&) {
    (void)dpg_trace_system_destroy(S);
    return DPG_ERR_ARG;
  } catch (const HipError&) {
    (void)dpg_trace_system_destroy(S);
    return DPG_ERR_HIP;
  } catch (const std::bad_alloc&) {
    (void)dpg_trace_system_destroy(S);
    return DPG_ERR_ALLOC;
  }
}

dpg_status dpg_trace_system_destroy(dpg_trace_system sys) {
  if (!sys) return DPG_ERR_ARG;
  (void)hipSetDevice(sys->device);
  for (void* p : {(void*)sys->row_ptr, (void*)sys->col, (void*)sys->contrib_ptr, (void*)sys->contrib,
                  (void*)sys->rhs_ptr, (void*)sys->rhs_contrib, (void*)sys->glob_dev, (void*)sys->cg_vec,
                  (void*)sys->cg_part, (void*)sys->cg_sc})
    if (p) (void)hipFree(p);
  if (sys->cg_host) (void)hipHostFree(sys->cg_host);
  for (auto e : sys->cg_ev)
    if (e) (void)hipEventDestroy(e);
  delete sys;
  return DPG_OK;
}

dpg_status dpg_trace_system_info(dpg_trace_system sys, int64_t* n_dofs, int64_t* nnz) {
  if (!sys || !n_dofs || !nnz) return DPG_ERR_ARG;
  *n_dofs = sys->n_dofs;
  *nnz = sys->nnz;
  return DPG_OK;
}

dpg_status dpg_trace_system_numbering(dpg_trace_system sys, int64_t* glob) {
  if (!sys || !glob) return DPG_ERR_ARG;
  std::memcpy(glob, sys->glob.data(), sizeof(int64_t) * sys->glob.size());
  return DPG_OK;
}

dpg_status dpg_trace_system_csr(dpg_trace_system sys, const int64_t** row_ptr, const int32_t** col) {
  if (!sys || !row_ptr || !col) return DPG_ERR_ARG;
  *row_ptr = sys->row_ptr;
  *col = sys->col;
  return DPG_OK;
}

dpg_status dpg_assemble(dpg_trace_system sys, const double* A, const double* b, double* vals, double* rhs,
                        void* stream) {
  if (!sys || (sys->nnz > 0 && (!A || !vals)) || (sys->n_dofs > 0 && (!b || !rhs))) return DPG_ERR_ARG;
  if (hipSetDevice(sys->device) != hipSuccess) return DPG_ERR_HIP;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = dpg::launch_gather(sys->nnz, sys->contrib_ptr, sys->contrib, reinterpret_cast<const double2*>(A),
                                    reinterpret_cast<double2*>(vals), st);
  if (e == hipSuccess)
    e = dpg::launch_gather(sys->n_dofs, sys->rhs_ptr, sys->rhs_contrib, reinterpret_cast<const double2*>(b),
                           reinterpret_cast<double2*>(rhs), st);
  if (e != hipSuccess) {
    set_error("dpg_assemble", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

dpg_status dpg_csr_matvec(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const double* vals,
                          const double* x, double* y, void* stream) {
  if (n_rows < 0 || (n_rows > 0 && (!row_ptr || !col || !vals || !x || !y))) return DPG_ERR_ARG;
  const hipError_t e = dpg::launch_csr_matvec(n_rows, row_ptr, col, reinterpret_cast<const double2*>(vals),
                                              reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y),
                                              reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_error("dpg_csr_matvec", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

dpg_status dpg_trace_system_scatter(dpg_trace_system sys, const double* t, double* t_local, void* stream) {
  if (!sys || (!sys->glob.empty() && (!t_local || (sys->n_dofs > 0 && !t)))) return DPG_ERR_ARG;
  if (hipSetDevice(sys->device) != hipSuccess) return DPG_ERR_HIP;
  const hipError_t e = dpg::launch_scatter((int64_t)sys->glob.size(), sys->glob_dev, reinterpret_cast<const double2*>(t),
                                           reinterpret_cast<double2*>(t_local), reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_error("dpg_trace_system_scatter", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

namespace {

// CG iterations on g (vectors, partial sums and scalars already in g) with
// the pinned host slots `host` [3 CG_NSC] and two events; returns after
// synchronising st.  Throws HipError.
void cg_run(dpg::CgArgs& g, double* host, hipEvent_t* ev, double tol, int64_t max_iter, int64_t* iters,
            double* relres, hipStream_t st) {
  for (int k = 0; k < 3 * dpg::CG_NSC; ++k) host[k] = 0.0;
  host[dpg::CG_TOL2] = tol * tol;
  HIP_CHECK(hipMemcpyAsync(g.sc, host, sizeof(double) * dpg::CG_NSC, hipMemcpyHostToDevice, st));
  hip_check(dpg::launch_cg_start(g, st));
  // Batches of iterations; the flag of batch k is read while batch k+1 runs
  // (iterations past convergence return at once).
  constexpr int64_t kBatch = 16;
  int64_t launched = 0;
  for (int64_t k = 0; launched < max_iter; ++k) {
    const int64_t nb = std::min<int64_t>(kBatch, max_iter - launched);
    hip_check(dpg::launch_cg_iterations(g, nb, st));
    launched += nb;
    double* slot = host + dpg::CG_NSC * (1 + (k & 1));
    HIP_CHECK(hipMemcpyAsync(slot, g.sc, sizeof(double) * dpg::CG_NSC, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipEventRecord(ev[k & 1], st));
    if (k > 0) {
      HIP_CHECK(hipEventSynchronize(ev[(k - 1) & 1]));
      if (host[dpg::CG_NSC * (1 + ((k - 1) & 1)) + dpg::CG_DONE] != 0.0) break;
    }
  }
  HIP_CHECK(hipMemcpyAsync(host + dpg::CG_NSC, g.sc, sizeof(double) * dpg::CG_NSC, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  const double* f = host + dpg::CG_NSC;
  *iters = (int64_t)f[dpg::CG_ITERS];
  *relres = f[dpg::CG_BN2] > 0.0 ? std::sqrt(f[dpg::CG_RR] / f[dpg::CG_BN2]) : 0.0;
}

}  // namespace

dpg_status dpg_cg_solve(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const double* vals, const double* b,
                        double* x, double tol, int64_t max_iter, int64_t* iters, double* relres, void* stream) {
  if (n_rows < 0 || max_iter < 0 || !(tol >= 0.0) || !iters || !relres) return DPG_ERR_ARG;
  if (n_rows > 0 && (!row_ptr || !col || !vals || !b || !x)) return DPG_ERR_ARG;
  *iters = 0;
  *relres = 0.0;
  if (n_rows == 0) return DPG_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<void*> own;
  double* host = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  dpg_status rc = DPG_OK;
  try {
    dpg::CgArgs g{};
    g.n = n_rows;
    g.row_ptr = row_ptr;
    g.col = col;
    g.val = reinterpret_cast<const double2*>(vals);
    g.b = reinterpret_cast<const double2*>(b);
    g.x = reinterpret_cast<double2*>(x);
    double2* vec = nullptr;
    HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&vec), sizeof(double2) * 3 * n_rows));
    own.push_back(vec);
    g.r = vec;
    g.p = vec + n_rows;
    g.q = vec + 2 * n_rows;
    HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&g.part), sizeof(double) * dpg::cg_part_len(n_rows)));
    own.push_back(g.part);
    HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&g.sc), sizeof(double) * dpg::CG_NSC));
    own.push_back(g.sc);
    // pinned host slots: the start scalars, then two slots the scalars are
    // copied back to after each batch of iterations
    HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&host), sizeof(double) * 3 * dpg::CG_NSC, hipHostMallocDefault));
    for (auto& e : ev) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    cg_run(g, host, ev, tol, max_iter, iters, relres, st);
  } catch (const HipError&) {
    rc = DPG_ERR_HIP;
  }
  if (rc != DPG_OK) (void)hipStreamSynchronize(st);
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  if (host) (void)hipHostFree(host);
  for (void* p : own) (void)hipFree(p);
  return rc;
}

dpg_status dpg_trace_system_cg(dpg_trace_system sys, const double* vals, const double* b, double* x, double tol,
                               int64_t max_iter, int64_t* iters, double* relres, void* stream) {
  if (!sys || max_iter < 0 || !(tol >= 0.0) || !iters || !relres) return DPG_ERR_ARG;
  if (sys->n_dofs > 0 && (!vals || !b || !x)) return DPG_ERR_ARG;
  *iters = 0;
  *relres = 0.0;
  if (sys->n_dofs == 0) return DPG_OK;
  if (hipSetDevice(sys->device) != hipSuccess) return DPG_ERR_HIP;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  try {
    dpg::CgArgs g{};
    g.n = sys->n_dofs;
    g.row_ptr = sys->row_ptr;
    g.col = sys->col;
    g.val = reinterpret_cast<const double2*>(vals);
    g.b = reinterpret_cast<const double2*>(b);
    g.x = reinterpret_cast<double2*>(x);
    g.r = sys->cg_vec;
    g.p = sys->cg_vec + sys->n_dofs;
    g.q = sys->cg_vec + 2 * sys->n_dofs;
    g.part = sys->cg_part;
    g.sc = sys->cg_sc;
    cg_run(g, sys->cg_host, sys->cg_ev, tol, max_iter, iters, relres, st);
  } catch (const HipError&) {
    (void)hipStreamSynchronize(st);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

dpg_status dpg_power_dissipation(dpg_plan plan, const dpg_problem* prob, const double* x, double* power,
                                 void* stream) {
  if (!plan) return DPG_ERR_ARG;
  dpg::ProbArgs pa;
  if (!make_prob_args(prob, pa) || prob->n_cells != plan->n_cells) return DPG_ERR_ARG;
  if (plan->n_cells == 0) return DPG_OK;
  if (!x || !power) return DPG_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  for (auto& g : plan->groups) {
    if (e != hipSuccess) break;
    e = dpg::launch_power(g.dt, pa, g.cells_dev, (int64_t)g.cells.size(), reinterpret_cast<const double2*>(x),
                          plan->v_off_dev, power, st);
  }
  if (e != hipSuccess) {
    set_error("dpg_power_dissipation", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

dpg_status dpg_dorfler_mark_workspace_size(int64_t n, size_t* bytes) {
  if (n < 0 || n > INT32_MAX || !bytes) return DPG_ERR_ARG;
  const hipError_t e = dpg::dorfler_mark_workspace(n, bytes);
  if (e != hipSuccess) {
    set_error("dpg_dorfler_mark_workspace_size", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

dpg_status dpg_dorfler_mark(int64_t n, const double* values, double refine_fraction, double coarsen_fraction,
                            int8_t* flags, void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 0 || n > INT32_MAX || !(refine_fraction >= 0.0 && refine_fraction <= 1.0) ||
      !(coarsen_fraction >= 0.0 && coarsen_fraction <= 1.0))
    return DPG_ERR_ARG;
  if (n == 0) return DPG_OK;
  if (!values || !flags) return DPG_ERR_ARG;
  bool too_small = false;
  const hipError_t e = dpg::dorfler_mark(n, values, refine_fraction, coarsen_fraction, flags, workspace,
                                         workspace_bytes, reinterpret_cast<hipStream_t>(stream), &too_small);
  if (e != hipSuccess) {
    set_error("dpg_dorfler_mark", e);
    return DPG_ERR_HIP;
  }
  if (too_small) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "dpg_dorfler_mark: workspace of %zu bytes too small or not 256-byte aligned", workspace_bytes);
    return DPG_ERR_ARG;
  }
  return DPG_OK;
}

dpg_status dpg_dorfler_mark_noalloc(int64_t n, const double* values, double refine_fraction,
                                    double coarsen_fraction, int8_t* flags, void* stream) {
  if (n < 0 || n > INT32_MAX || !(refine_fraction >= 0.0 && refine_fraction <= 1.0) ||
      !(coarsen_fraction >= 0.0 && coarsen_fraction <= 1.0))
    return DPG_ERR_ARG;
  if (n == 0) return DPG_OK;
  if (!values || !flags) return DPG_ERR_ARG;
  if (n > dpg::kMarkMaxCells) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "dpg_dorfler_mark_noalloc: %lld cells exceed the static scratch limit of %lld",
                  (long long)n, (long long)dpg::kMarkMaxCells);
    return DPG_ERR_UNSUPPORTED;
  }
  bool too_large = false;
  const hipError_t e = dpg::dorfler_mark_noalloc(n, values, refine_fraction, coarsen_fraction, flags,
                                                 reinterpret_cast<hipStream_t>(stream), &too_large);
  if (e != hipSuccess) {
    set_error("dpg_dorfler_mark_noalloc", e);
    return DPG_ERR_HIP;
  }
  if (too_large) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "dpg_dorfler_mark_noalloc: the temporaries of %lld cells exceed the static scratch of %zu bytes",
                  (long long)n, dpg::kMarkScratchBytes);
    return DPG_ERR_UNSUPPORTED;
  }
  return DPG_OK;
}

dpg_status dpg_reconstruct(dpg_plan plan, const double* K, const double* l, const double* t_local, double* x,
                           int32_t* info, void* stream) {
  if (!plan) return DPG_ERR_ARG;
  if (plan->n_cells == 0) return DPG_OK;
  if (!K || !l || !t_local || !x || !info) return DPG_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  for (auto& g : plan->groups) {
    const int64_t nc = (int64_t)g.cells.size();
    for (int64_t s0 = 0; s0 < nc && e == hipSuccess; s0 += g.chunk) {
      dpg::ChunkArgs ca{};
      ca.cell_ids = g.cells_dev + s0;
      ca.n = std::min<int64_t>(g.chunk, nc - s0);
      ca.Z = g.Z;
      ca.split = 0;
      ca.info = info;
      dpg::CondArgs cg{};
      cg.Ke = reinterpret_cast<const double2*>(K);
      cg.le = reinterpret_cast<const double2*>(l);
      cg.Ke_off = plan->K_off_dev;
      cg.le_off = plan->v_off_dev;
      cg.nu = g.d.nu;
      cg.kfull = g.d.k;
      cg.tk = reinterpret_cast<const double2*>(t_local);
      cg.tk_off = plan->b_off_dev;
      cg.xout = reinterpret_cast<double2*>(x);
      e = dpg::launch_recon_load(g.rt, ca, cg, st);
      if (e == hipSuccess) e = dpg::launch_factor(g.rt, ca, st, nullptr);
      if (e == hipSuccess) e = dpg::launch_recon_back(g.rt, ca, cg, st);
    }
  }
  if (e != hipSuccess) {
    set_error("dpg_reconstruct", e);
    return DPG_ERR_HIP;
  }
  return DPG_OK;
}

dpg_status dpg_plan_set_profiling(dpg_plan plan, int32_t enable) {
  if (!plan) return DPG_ERR_ARG;
  plan->prof.on = enable != 0;
  return DPG_OK;
}

dpg_status dpg_plan_profile(dpg_plan plan, double* ms, int64_t* launches) {
  if (!plan || !ms || !launches) return DPG_ERR_ARG;
  for (int k = 0; k < DPG_K_COUNT; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  dpg_status rc = DPG_OK;
  for (auto& r : plan->prof.recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.e) != hipSuccess || hipEventElapsedTime(&t, r.b, r.e) != hipSuccess) rc = DPG_ERR_HIP;
    if (r.cls >= 0 && r.cls < DPG_K_COUNT) {
      ms[r.cls] += t;
      launches[r.cls] += 1;
    }
    plan->prof.pool.push_back(r.b);
    plan->prof.pool.push_back(r.e);
  }
  plan->prof.recs.clear();
  return rc;
}

dpg_status dpg_form_local(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count, double* G,
                          double* Bf, double* lvec, int32_t* info, void* stream) {
  return form_cells(plan, prob, first, count, nullptr, G, Bf, lvec, nullptr, nullptr, info, stream);
}

dpg_status dpg_form_augmented(dpg_plan plan, const dpg_problem* prob, int64_t first, int64_t count, const double* x,
                              double* Gs, double* Bs, double* ls, double* rs, double* d, int32_t* info,
                              void* stream) {
  if (!rs || !d) return DPG_ERR_ARG;
  return form_cells(plan, prob, first, count, x, Gs, Bs, ls, rs, d, info, stream);
}

}  // extern "C"
