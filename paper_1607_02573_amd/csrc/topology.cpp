// Host edge topology of a tetrahedral mesh (paper Section 2.1: lowest-order
// Nedelec elements carry one unknown per oriented edge).
//
// Edges are the unique vertex pairs (lo, hi) of the tetrahedra, numbered in
// lexicographic order and oriented lo -> hi; a tetrahedron with ascending
// vertices v0<v1<v2<v3 lists its edges as (0,1),(0,2),(0,3),(1,2),(1,3),(2,3),
// so every local edge has the global orientation.  Edges lying on a PEC face
// (E x n = 0, equation (eqmetal)) are eliminated; the remaining edges in
// ascending order are the unknowns.  The CSR pattern of A couples two
// unknowns when their edges share a tetrahedron; for each row it also keeps
// the (tetrahedron, local edge) and (boundary face, local edge) pairs that
// contribute to it, so that the device can gather A's values row by row in a
// fixed order (no atomics, bitwise reproducible).
#include <algorithm>
#include <numeric>
#include <thread>

#include "common.hpp"
#include "parallel.hpp"

namespace mw {

static const int kTetEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
static const int kTriEdge[3][2] = {{0, 1}, {0, 2}, {1, 2}};

void build_topology(const mw_mesh& m, Topology& T) {
  MW_CHECK(m.nv > 0 && m.nt > 0 && m.xyz && m.tet, MW_EINVAL, "mesh: empty or NULL arrays");
  MW_CHECK(m.nbf >= 0 && (m.nbf == 0 || (m.bface && m.btag)), MW_EINVAL, "mesh: NULL face arrays");
  const int32_t nv = m.nv, nt = m.nt, nbf = m.nbf;
  T.nv = nv; T.nt = nt; T.nbf = nbf;
  T.xyz.assign(m.xyz, m.xyz + (size_t)nv * 3);
  T.tet.resize((size_t)nt * 4);
  for (int64_t t = 0; t < nt; ++t) {
    int32_t v[4];
    for (int k = 0; k < 4; ++k) {
      v[k] = m.tet[t * 4 + k];
      MW_CHECK(v[k] >= 0 && v[k] < nv, MW_EINVAL, "mesh: tetrahedron vertex out of range");
    }
    std::sort(v, v + 4);
    MW_CHECK(v[0] != v[1] && v[1] != v[2] && v[2] != v[3], MW_EINVAL, "mesh: degenerate tetrahedron");
    for (int k = 0; k < 4; ++k) T.tet[t * 4 + k] = v[k];
  }

  // ---- vertex -> tetrahedra (ascending tet ids)
  std::vector<int64_t> vt_ptr(nv + 1, 0);
  for (int64_t i = 0; i < (int64_t)nt * 4; ++i) vt_ptr[T.tet[i] + 1]++;
  for (int32_t v = 0; v < nv; ++v) vt_ptr[v + 1] += vt_ptr[v];
  std::vector<int32_t> vt(vt_ptr[nv]);
  {
    std::vector<int64_t> fill(vt_ptr.begin(), vt_ptr.end() - 1);
    for (int32_t t = 0; t < nt; ++t)
      for (int k = 0; k < 4; ++k) vt[fill[T.tet[t * 4 + k]]++] = t;
  }

  // ---- edges: neighbours hi > lo of every vertex lo, sorted and unique
  std::vector<int64_t> lo_ptr(nv + 1, 0);
  for (int32_t t = 0; t < nt; ++t)
    for (auto& e : kTetEdge) lo_ptr[T.tet[t * 4 + e[0]] + 1]++;
  for (int32_t v = 0; v < nv; ++v) lo_ptr[v + 1] += lo_ptr[v];
  std::vector<int32_t> hi(lo_ptr[nv]);
  {
    std::vector<int64_t> fill(lo_ptr.begin(), lo_ptr.end() - 1);
    for (int32_t t = 0; t < nt; ++t)
      for (auto& e : kTetEdge) hi[fill[T.tet[t * 4 + e[0]]]++] = T.tet[t * 4 + e[1]];
  }
  std::vector<int64_t> ecount(nv + 1, 0);
  parallel_for(nv, [&](int64_t v) {
    auto b = hi.begin() + lo_ptr[v], e = hi.begin() + lo_ptr[v + 1];
    std::sort(b, e);
    ecount[v + 1] = std::unique(b, e) - b;
  });
  std::vector<int64_t> e_ptr(nv + 1, 0);  // first edge id of vertex lo
  for (int32_t v = 0; v < nv; ++v) e_ptr[v + 1] = e_ptr[v] + ecount[v + 1];
  const int64_t ne = e_ptr[nv];
  T.edges.resize(ne * 2);
  parallel_for(nv, [&](int64_t v) {
    for (int64_t k = 0; k < ecount[v + 1]; ++k) {
      T.edges[(e_ptr[v] + k) * 2] = v;
      T.edges[(e_ptr[v] + k) * 2 + 1] = hi[lo_ptr[v] + k];
    }
  });
  auto edge_id = [&](int32_t a, int32_t b) -> int64_t {
    if (a > b) std::swap(a, b);
    const int32_t* beg = hi.data() + lo_ptr[a];
    const int32_t* end = beg + ecount[a + 1];
    const int32_t* it = std::lower_bound(beg, end, b);
    if (it == end || *it != b) return -1;
    return e_ptr[a] + (it - beg);
  };
  T.t2e.resize((size_t)nt * 6);
  parallel_for(nt, [&](int64_t t) {
    for (int p = 0; p < 6; ++p)
      T.t2e[t * 6 + p] = (int32_t)edge_id(T.tet[t * 4 + kTetEdge[p][0]], T.tet[t * 4 + kTetEdge[p][1]]);
  });

  // ---- boundary faces: canonical order, owner tetrahedron, edges
  T.bface.resize((size_t)nbf * 3);
  T.btag.assign(m.btag, m.btag + nbf);
  T.bf_owner.assign(nbf, -1);
  T.bf2e.resize((size_t)nbf * 3);
  std::vector<int> bad(1, 0);
  parallel_for(nbf, [&](int64_t f) {
    int32_t v[3] = {m.bface[f * 3], m.bface[f * 3 + 1], m.bface[f * 3 + 2]};
    std::sort(v, v + 3);
    if (v[0] < 0 || v[2] >= nv || v[0] == v[1] || v[1] == v[2]) { bad[0] = 1; return; }
    for (int k = 0; k < 3; ++k) T.bface[f * 3 + k] = v[k];
    int owners = 0;
    for (int64_t q = vt_ptr[v[0]]; q < vt_ptr[v[0] + 1]; ++q) {
      int32_t t = vt[q];
      const int32_t* tv = &T.tet[(size_t)t * 4];
      bool h1 = false, h2 = false;
      for (int k = 0; k < 4; ++k) { h1 |= tv[k] == v[1]; h2 |= tv[k] == v[2]; }
      if (h1 && h2) { if (!owners) T.bf_owner[f] = t; owners++; }
    }
    if (owners != 1) { bad[0] = 2; return; }
    for (int q = 0; q < 3; ++q) T.bf2e[f * 3 + q] = (int32_t)edge_id(v[kTriEdge[q][0]], v[kTriEdge[q][1]]);
  });
  MW_CHECK(bad[0] != 1, MW_EINVAL, "mesh: boundary face vertex out of range or degenerate");
  MW_CHECK(bad[0] != 2, MW_EINVAL, "mesh: a labelled face is not a boundary face of exactly one tetrahedron");
  for (int32_t f = 0; f < nbf; ++f) MW_CHECK(T.btag[f] >= MW_TAG_PEC, MW_EINVAL, "mesh: invalid face tag");

  // ---- PEC elimination and unknown numbering
  T.pec.assign(ne, 0);
  for (int32_t f = 0; f < nbf; ++f)
    if (T.btag[f] == MW_TAG_PEC)
      for (int q = 0; q < 3; ++q) T.pec[T.bf2e[f * 3 + q]] = 1;
  T.dof.assign(ne, -1);
  T.free_edge.clear();
  for (int64_t e = 0; e < ne; ++e)
    if (!T.pec[e]) { T.dof[e] = (int32_t)T.free_edge.size(); T.free_edge.push_back((int32_t)e); }
  const int64_t n = T.n();
  MW_CHECK(n > 0, MW_EINVAL, "mesh: every edge is PEC");

  // ---- edge -> (tet, local edge) and edge -> (non-PEC face, local edge)
  std::vector<int64_t> et_ptr(ne + 1, 0);
  for (int64_t i = 0; i < (int64_t)nt * 6; ++i) et_ptr[T.t2e[i] + 1]++;
  for (int64_t e = 0; e < ne; ++e) et_ptr[e + 1] += et_ptr[e];
  std::vector<int32_t> et(et_ptr[ne]);
  {
    std::vector<int64_t> fill(et_ptr.begin(), et_ptr.end() - 1);
    for (int32_t t = 0; t < nt; ++t)
      for (int p = 0; p < 6; ++p) et[fill[T.t2e[(size_t)t * 6 + p]]++] = t * 6 + p;
  }
  std::vector<int64_t> ef_ptr(ne + 1, 0);
  for (int32_t f = 0; f < nbf; ++f)
    if (T.btag[f] != MW_TAG_PEC)
      for (int q = 0; q < 3; ++q) ef_ptr[T.bf2e[f * 3 + q] + 1]++;
  for (int64_t e = 0; e < ne; ++e) ef_ptr[e + 1] += ef_ptr[e];
  std::vector<int32_t> ef(ef_ptr[ne]);
  {
    std::vector<int64_t> fill(ef_ptr.begin(), ef_ptr.end() - 1);
    for (int32_t f = 0; f < nbf; ++f)
      if (T.btag[f] != MW_TAG_PEC)
        for (int q = 0; q < 3; ++q) ef[fill[T.bf2e[f * 3 + q]]++] = f * 3 + q;
  }

  // ---- CSR pattern of A and per-row contribution lists
  T.rt_ptr.assign(n + 1, 0);
  T.rf_ptr.assign(n + 1, 0);
  std::vector<int64_t> rowlen(n + 1, 0);
  parallel_for(n, [&](int64_t r) {
    int64_t e = T.free_edge[r];
    T.rt_ptr[r + 1] = et_ptr[e + 1] - et_ptr[e];
    T.rf_ptr[r + 1] = ef_ptr[e + 1] - ef_ptr[e];
    std::vector<int32_t> cols;
    cols.reserve(64);
    for (int64_t q = et_ptr[e]; q < et_ptr[e + 1]; ++q) {
      int32_t t = et[q] / 6;
      for (int k = 0; k < 6; ++k) {
        int32_t d = T.dof[T.t2e[(size_t)t * 6 + k]];
        if (d >= 0) cols.push_back(d);
      }
    }
    std::sort(cols.begin(), cols.end());
    rowlen[r + 1] = std::unique(cols.begin(), cols.end()) - cols.begin();
  });
  T.row_ptr.assign(n + 1, 0);
  for (int64_t r = 0; r < n; ++r) {
    T.row_ptr[r + 1] = T.row_ptr[r] + rowlen[r + 1];
    T.rt_ptr[r + 1] += T.rt_ptr[r];
    T.rf_ptr[r + 1] += T.rf_ptr[r];
  }
  T.col.resize(T.row_ptr[n]);
  T.rt.resize(T.rt_ptr[n]);
  T.rf.resize(T.rf_ptr[n]);
  parallel_for(n, [&](int64_t r) {
    int64_t e = T.free_edge[r];
    std::vector<int32_t> cols;
    cols.reserve(64);
    int64_t w = T.rt_ptr[r];
    for (int64_t q = et_ptr[e]; q < et_ptr[e + 1]; ++q) {
      T.rt[w++] = et[q];
      int32_t t = et[q] / 6;
      for (int k = 0; k < 6; ++k) {
        int32_t d = T.dof[T.t2e[(size_t)t * 6 + k]];
        if (d >= 0) cols.push_back(d);
      }
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    std::copy(cols.begin(), cols.end(), T.col.begin() + T.row_ptr[r]);
    w = T.rf_ptr[r];
    for (int64_t q = ef_ptr[e]; q < ef_ptr[e + 1]; ++q) T.rf[w++] = ef[q];
  });
}

}  // namespace mw
