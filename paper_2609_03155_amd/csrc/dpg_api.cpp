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

namespace {

constexpr double kC0 = 299792458.0;   // speed of light in vacuum (App. A scaling of omega)

struct DegreeGroup {
  int p = 0;
  dpg::Dims d{};
  dpg::DevTables dt{};
  std::vector<void*> bufs;            // device table allocations
  std::vector<int64_t> cells;         // global cell ids of this degree, ascending
  int64_t* cells_dev = nullptr;
  int64_t chunk = 0;                  // cells per chunk
};

}  // namespace

struct dpg_plan_s {
  int device = 0;
  int dp = 1;
  int64_t n_cells = 0;
  std::vector<int64_t> K_off, v_off;
  int64_t* K_off_dev = nullptr;
  int64_t* v_off_dev = nullptr;
  std::vector<DegreeGroup> groups;
  double2* Z = nullptr;
  double* dscale = nullptr;
  double* met = nullptr;
  uint16_t* wsplit = nullptr;
  std::vector<void*> misc;            // other device allocations
  dpg::Prof prof;
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
  // S/M formation tiles: component pairs (a >= b) x 64-blocks (lower for a == b)
  const int nc = d.N / 3, ncb = (nc + 63) / 64;
  std::vector<int4> tiles;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b <= a; ++b)
      for (int I = 0; I < ncb; ++I)
        for (int J = 0; J < ncb; ++J)
          if (a > b || J <= I) tiles.push_back(make_int4(a, b, I, J));
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
  t.sm_tiles = upload(g.bufs, tiles);
  t.n_sm_tiles = (int)tiles.size();
}

void free_plan(dpg_plan_s* p) {
  if (!p) return;
  for (auto& g : p->groups) {
    for (void* b : g.bufs) (void)hipFree(b);
    if (g.cells_dev) (void)hipFree(g.cells_dev);
  }
  for (void* b : p->misc) (void)hipFree(b);
  for (auto& r : p->prof.recs) {
    (void)hipEventDestroy(r.b);
    (void)hipEventDestroy(r.e);
  }
  for (auto e : p->prof.pool) (void)hipEventDestroy(e);
  if (p->Z) (void)hipFree(p->Z);
  if (p->dscale) (void)hipFree(p->dscale);
  if (p->met) (void)hipFree(p->met);
  if (p->wsplit) (void)hipFree(p->wsplit);
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
  }
  return "unknown status";
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
    for (int p = 1; p <= 4; ++p) {
      DegreeGroup g;
      g.p = p;
      for (int64_t c = 0; c < n_cells; ++c)
        if (degree_host[c] == p) g.cells.push_back(c);
      if (g.cells.empty()) continue;
      build_group(g, dp);
      std::vector<void*> tmp;
      g.cells_dev = upload(tmp, g.cells);
      P->groups.push_back(std::move(g));
    }
    size_t free_b = 0, total_b = 0;
    HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
    int64_t budget = max_workspace_bytes > 0 ? max_workspace_bytes : (int64_t)(0.4 * (double)free_b);
    size_t zmax = 0, dmax = 0, mmax = 0, smax = 0;
    for (auto& g : P->groups) {
      const int64_t mper = 12 * (int64_t)g.d.nq + 36 * (int64_t)g.d.nfq;
      const int64_t sper = dpg::split_elems(g.dt);
      const int64_t per = g.dt.zstride * 16 + (int64_t)g.d.nvp * 8 + mper * 8 + sper * 2;
      int64_t ch = std::max<int64_t>(1, budget / per);
      ch = std::min<int64_t>(ch, (int64_t)g.cells.size());
      g.chunk = ch;
      zmax = std::max(zmax, (size_t)ch * g.dt.zstride * 16);
      dmax = std::max(dmax, (size_t)ch * g.d.nvp * 8);
      mmax = std::max(mmax, (size_t)(ch * mper * 8));
      smax = std::max(smax, (size_t)(ch * sper * 2));
    }
    if (zmax) {
      if (hipMalloc(reinterpret_cast<void**>(&P->Z), zmax) != hipSuccess) {
        free_plan(P);
        return DPG_ERR_ALLOC;
      }
      if (hipMalloc(reinterpret_cast<void**>(&P->dscale), dmax) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&P->met), mmax) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&P->wsplit), smax) != hipSuccess) {
        free_plan(P);
        return DPG_ERR_ALLOC;
      }
    }
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
  if (!plan || first < 0 || count < 0 || first + count > plan->n_cells) return DPG_ERR_ARG;
  if (count > 0 && (!K || !l || !eta || !info)) return DPG_ERR_ARG;
  if (precision != DPG_FP64 && precision != DPG_SPLIT_FP32) return DPG_ERR_ARG;
  dpg::ProbArgs pa;
  if (!make_prob_args(prob, pa) || prob->n_cells != plan->n_cells) return DPG_ERR_ARG;
  if (count == 0) return DPG_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipSetDevice(plan->device) != hipSuccess) return DPG_ERR_HIP;
  for (auto& g : plan->groups) {
    // this degree's cells inside [first, first + count): a contiguous run of its sorted list
    const int64_t lo = std::lower_bound(g.cells.begin(), g.cells.end(), first) - g.cells.begin();
    const int64_t hi = std::lower_bound(g.cells.begin(), g.cells.end(), first + count) - g.cells.begin();
    for (int64_t s0 = lo; s0 < hi; s0 += g.chunk) {
      dpg::ChunkArgs ca{};
      ca.cell_ids = g.cells_dev + s0;
      ca.n = std::min<int64_t>(g.chunk, hi - s0);
      ca.Z = plan->Z;
      ca.dscale = plan->dscale;
      ca.met = plan->met;
      ca.wsplit = plan->wsplit;
      ca.split = precision == DPG_SPLIT_FP32 ? 1 : 0;
      ca.K_off = plan->K_off_dev;
      ca.v_off = plan->v_off_dev;
      ca.cell_base = first;
      ca.K_base = plan->K_off[first];
      ca.v_base = plan->v_off[first];
      ca.x = reinterpret_cast<const double2*>(x);
      ca.K = reinterpret_cast<double2*>(K);
      ca.l = reinterpret_cast<double2*>(l);
      ca.eta = eta;
      ca.info = info;
      dpg::Prof* pr = plan->prof.on ? &plan->prof : nullptr;
      hipError_t e = dpg::launch_formation(g.dt, pa, ca, st, pr);
      if (e == hipSuccess) e = dpg::launch_factor(g.dt, ca, st, pr);
      if (e == hipSuccess) e = dpg::launch_herk(g.dt, ca, st, pr);
      if (e != hipSuccess) {
        set_error("dpg_local_solve launch", e);
        return DPG_ERR_HIP;
      }
    }
  }
  return DPG_OK;
}

dpg_status dpg_local_solve(dpg_plan plan, const dpg_problem* prob, const double* x, double* K, double* l,
                           double* eta, int32_t* info, int32_t precision, void* stream) {
  if (!plan) return DPG_ERR_ARG;
  if (plan->n_cells > 0 && (!K || !l || !eta || !info)) return DPG_ERR_ARG;
  return dpg_local_solve_range(plan, prob, 0, plan->n_cells, x, K, l, eta, info, precision, stream);
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
  for (int64_t s0 = 0; s0 < count && rc == DPG_OK; s0 += grp->chunk) {
    dpg::ChunkArgs ca{};
    ca.cell_ids = ids_dev + s0;
    ca.n = std::min<int64_t>(grp->chunk, count - s0);
    ca.Z = plan->Z;
    ca.dscale = plan->dscale;
    ca.met = plan->met;
    ca.K_off = plan->K_off_dev;
    ca.v_off = plan->v_off_dev;
    ca.x = nullptr;
    ca.info = info;
    if (dpg::launch_formation(grp->dt, pa, ca, st) != hipSuccess ||
        dpg::launch_extract(grp->dt, ca, reinterpret_cast<double2*>(G) + s0 * nv * nv,
                            reinterpret_cast<double2*>(Bf) + s0 * nv * d.k,
                            reinterpret_cast<double2*>(lvec) + s0 * nv, st) != hipSuccess)
      rc = DPG_ERR_HIP;
  }
  // the id buffer must outlive the enqueued work
  if (hipStreamSynchronize(st) != hipSuccess) rc = DPG_ERR_HIP;
  (void)hipFree(ids_dev);
  return rc;
}

}  // extern "C"
