// Host side of the condensed trace system (paper §2.3: static condensation
// and the global linear system of the trace unknowns): numbering of the
// global trace unknowns of a conforming hexahedral mesh and the CSR
// structure of the assembled matrix, with the gather lists that let the
// device assemble it without atomics.
//
// Numbering rule (see include/dpg.h, dpg_trace_system_create):
//  * a cell's local trace functions (12 r^2 per field, Ehat then Hhat) live
//    on its 12 edges (r each) or 6 faces (2 r (r-1) each), in the local
//    order: edges along x at (y,z) = (0,0),(1,0),(0,1),(1,1), then along y,
//    then along z; faces x-,x+,y-,y+,z-,z+, each first the functions whose
//    component is the lower tangential axis, then the other, bubble degree
//    m = 2..r, along-degree i fastest;
//  * edges are identified by their (start, end) global vertices along the
//    component axis, faces by their sorted vertex quadruple; all cells must
//    agree on edge directions and face axes (ERR_ARG otherwise);
//  * minimum rule on shared entities for mixed degrees;
//  * removed: Ehat on entities inside PEC faces; Hhat face functions of
//    Robin faces and Hhat edge functions all of whose cell faces are Robin;
//  * ids in order of first appearance, cells in order, local order within.
#include "dpg_trace.h"

#include <algorithm>
#include <array>
#include <map>
#include <stdexcept>
#include <unordered_map>

namespace dpg {

namespace {

constexpr int kPEC = 1, kPort = 2, kRobin0 = 3;

inline int lvert(int i, int j, int k) { return 4 * k + 2 * j + i; }

// local vertices (start, end) of edge e and its component axis
void edge_ends(int e, int& axis, int& v0, int& v1) {
  axis = e / 4;
  const int tb = e % 2, tc = (e % 4) / 2;
  int ijk0[3], ijk1[3];
  int o[2], n = 0;
  for (int ax = 0; ax < 3; ++ax)
    if (ax != axis) o[n++] = ax;
  ijk0[axis] = 0;
  ijk1[axis] = 1;
  ijk0[o[0]] = ijk1[o[0]] = tb;
  ijk0[o[1]] = ijk1[o[1]] = tc;
  v0 = lvert(ijk0[0], ijk0[1], ijk0[2]);
  v1 = lvert(ijk1[0], ijk1[1], ijk1[2]);
}

// local vertices of face f at (t1, t2) = (0,0), (1,0), (0,1), (1,1)
std::array<int, 4> face_verts(int f) {
  const int nax = f / 2, side = f % 2;
  int t[2], n = 0;
  for (int ax = 0; ax < 3; ++ax)
    if (ax != nax) t[n++] = ax;
  std::array<int, 4> out{};
  int q = 0;
  for (int u2 = 0; u2 < 2; ++u2)
    for (int u1 = 0; u1 < 2; ++u1) {
      int ijk[3];
      ijk[nax] = side;
      ijk[t[0]] = u1;
      ijk[t[1]] = u2;
      out[q++] = lvert(ijk[0], ijk[1], ijk[2]);
    }
  return out;
}

bool face_has(int f, int v) {
  const auto fv = face_verts(f);
  return std::find(fv.begin(), fv.end(), v) != fv.end();
}

struct EdgeKey {
  int64_t a, b;
  bool operator==(const EdgeKey& o) const { return a == o.a && b == o.b; }
};
struct EdgeHash {
  size_t operator()(const EdgeKey& k) const { return std::hash<int64_t>()(k.a * 1000003 ^ k.b); }
};
using FaceKey = std::array<int64_t, 4>;   // sorted global vertices

struct EdgeInfo {
  int rmin = 1 << 30;
  bool pec = false;
  bool all_robin = true;
  int64_t id[2] = {-1, -1};   // first id of the field's functions (consecutive along i)
};
struct FaceInfo {
  int rmin = 1 << 30;
  bool pec = false, robin = false;
  std::array<int64_t, 3> orient{};   // global vertices at (0,0), (1,0), (0,1)
  bool have_orient = false;
};

bool robin(int k) { return k == kPort || k == kRobin0; }

}  // namespace

void trace_numbering(const int64_t* cells, const int8_t* face_kind, const int8_t* degree, int64_t n,
                     std::vector<int64_t>& toff, std::vector<int64_t>& glob, int64_t& n_dofs) {
  std::unordered_map<EdgeKey, EdgeInfo, EdgeHash> edges;
  std::map<FaceKey, FaceInfo> faces;
  toff.assign(n + 1, 0);
  for (int64_t c = 0; c < n; ++c) {
    const int r = degree[c] + 1;
    toff[c + 1] = toff[c] + 24 * (int64_t)r * r;
    const int64_t* V = cells + 8 * c;
    const int8_t* fk = face_kind + 6 * c;
    for (int e = 0; e < 12; ++e) {
      int ax, v0, v1;
      edge_ends(e, ax, v0, v1);
      const EdgeKey key{V[v0], V[v1]};
      if (edges.count(EdgeKey{V[v1], V[v0]})) throw std::invalid_argument("edge direction");
      EdgeInfo& ei = edges[key];
      ei.rmin = std::min(ei.rmin, r);
      bool allr = true;
      for (int f = 0; f < 6; ++f)
        if (face_has(f, v0) && face_has(f, v1)) {
          if (fk[f] == kPEC) ei.pec = true;
          if (!robin(fk[f])) allr = false;
        }
      ei.all_robin = ei.all_robin && allr;
    }
    for (int f = 0; f < 6; ++f) {
      const auto fv = face_verts(f);
      FaceKey key{V[fv[0]], V[fv[1]], V[fv[2]], V[fv[3]]};
      std::sort(key.begin(), key.end());
      FaceInfo& fi = faces[key];
      const std::array<int64_t, 3> o{V[fv[0]], V[fv[1]], V[fv[2]]};
      if (fi.have_orient && fi.orient != o) throw std::invalid_argument("face axes");
      fi.orient = o;
      fi.have_orient = true;
      fi.rmin = std::min(fi.rmin, r);
      if (fk[f] == kPEC) fi.pec = true;
      if (robin(fk[f])) fi.robin = true;
    }
  }
  // ids in order of first appearance
  glob.assign(toff[n], -1);
  std::map<std::tuple<int, FaceKey, int, int, int>, int64_t> face_ids;   // (field, face, group, m, i)
  std::unordered_map<EdgeKey, std::array<std::vector<int64_t>, 2>, EdgeHash> edge_ids;
  int64_t next = 0;
  for (int64_t c = 0; c < n; ++c) {
    const int r = degree[c] + 1;
    const int64_t* V = cells + 8 * c;
    const int nt1 = 12 * r * r;
    for (int field = 0; field < 2; ++field)
      for (int lt = 0; lt < nt1; ++lt) {
        int64_t id = -1;
        if (lt < 12 * r) {
          const int e = lt / r, i = lt % r;
          int ax, v0, v1;
          edge_ends(e, ax, v0, v1);
          const EdgeKey key{V[v0], V[v1]};
          const EdgeInfo& ei = edges[key];
          if (i >= ei.rmin) continue;
          if (field == 0 && ei.pec) continue;
          if (field == 1 && ei.all_robin) continue;
          auto& ids = edge_ids[key][field];
          if (ids.empty()) ids.assign(ei.rmin, -1);
          if (ids[i] < 0) ids[i] = next++;
          id = ids[i];
        } else {
          const int q = lt - 12 * r, per = 2 * r * (r - 1);
          const int f = q / per, w = q % per;
          const int grp = w / (r * (r - 1)), rest = w % (r * (r - 1));
          const int m = 2 + rest / r, i = rest % r;
          const auto fv = face_verts(f);
          FaceKey key{V[fv[0]], V[fv[1]], V[fv[2]], V[fv[3]]};
          std::sort(key.begin(), key.end());
          const FaceInfo& fi = faces[key];
          if (m > fi.rmin || i >= fi.rmin) continue;
          if (field == 0 && fi.pec) continue;
          if (field == 1 && fi.robin) continue;
          auto it = face_ids.find(std::make_tuple(field, key, grp, m, i));
          if (it == face_ids.end()) it = face_ids.emplace(std::make_tuple(field, key, grp, m, i), next++).first;
          id = it->second;
        }
        glob[toff[c] + field * nt1 + lt] = id;
      }
  }
  n_dofs = next;
}

void trace_csr(const std::vector<int64_t>& toff, const std::vector<int64_t>& glob, const std::vector<int64_t>& A_off,
               const std::vector<int64_t>& b_off, int64_t n_dofs, std::vector<int64_t>& row_ptr,
               std::vector<int32_t>& col, std::vector<int64_t>& contrib_ptr, std::vector<int64_t>& contrib,
               std::vector<int64_t>& rhs_ptr, std::vector<int64_t>& rhs_contrib) {
  const int64_t n = (int64_t)toff.size() - 1;
  // incidence: for every unknown, its (cell, local index) occurrences
  std::vector<int64_t> inc_ptr(n_dofs + 1, 0);
  for (int64_t c = 0; c < n; ++c)
    for (int64_t q = toff[c]; q < toff[c + 1]; ++q)
      if (glob[q] >= 0) ++inc_ptr[glob[q] + 1];
  for (int64_t g = 0; g < n_dofs; ++g) inc_ptr[g + 1] += inc_ptr[g];
  std::vector<int64_t> inc_cell(inc_ptr[n_dofs]), inc_loc(inc_ptr[n_dofs]);
  {
    std::vector<int64_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int64_t c = 0; c < n; ++c)
      for (int64_t q = toff[c]; q < toff[c + 1]; ++q)
        if (glob[q] >= 0) {
          const int64_t g = glob[q];
          inc_cell[fill[g]] = c;
          inc_loc[fill[g]] = q - toff[c];
          ++fill[g];
        }
  }
  // rhs gather: b_K(local) -> unknown
  rhs_ptr.assign(inc_ptr.begin(), inc_ptr.end());
  rhs_contrib.resize(inc_ptr[n_dofs]);
  for (int64_t k = 0; k < inc_ptr[n_dofs]; ++k) rhs_contrib[k] = b_off[inc_cell[k]] + inc_loc[k];
  // rows: for unknown g, every (cell containing g) x (kept local function of that cell)
  row_ptr.assign(n_dofs + 1, 0);
  col.clear();
  contrib_ptr.assign(1, 0);
  contrib.clear();
  struct Ent {
    int64_t h, src;
  };
  std::vector<Ent> ents;
  for (int64_t g = 0; g < n_dofs; ++g) {
    ents.clear();
    for (int64_t k = inc_ptr[g]; k < inc_ptr[g + 1]; ++k) {
      const int64_t c = inc_cell[k], a = inc_loc[k];
      const int64_t nt = toff[c + 1] - toff[c];
      for (int64_t b = 0; b < nt; ++b) {
        const int64_t h = glob[toff[c] + b];
        if (h >= 0) ents.push_back({h, A_off[c] + b * nt + a});   // A_K(a, b), column-major
      }
    }
    std::sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) { return x.h < y.h || (x.h == y.h && x.src < y.src); });
    for (size_t k = 0; k < ents.size(); ++k) {
      if (k == 0 || ents[k].h != ents[k - 1].h) {
        col.push_back((int32_t)ents[k].h);
        contrib_ptr.push_back(contrib_ptr.back());
      }
      contrib.push_back(ents[k].src);
      ++contrib_ptr.back();
    }
    row_ptr[g + 1] = (int64_t)col.size();
  }
}

}  // namespace dpg
