// Host side of the one-level ORAS preconditioner (paper Section 3).
//
//  * T_i^delta: T_i^{delta-1} plus every tetrahedron sharing a vertex with it
//    ("adjacent" read as vertex adjacency: the only reading under which the
//    support of the P1 function chi~_i stays inside T_i^delta);
//  * R_i: restriction to the non-PEC edges of T_i^delta; locally numbered in
//    reverse Cuthill-McKee order of the graph of B_i (banded dense factors);
//  * partition of unity, equations (algebPartUnity) and (chi):
//    chi~_i = 1 on the nodes of T_i^0, 0 on the other nodes of T_i^delta,
//    chi_i = chi~_i / sum_j chi~_j, and D_i[e] is chi_i at the midpoint of e
//    (the mean of its end values), so that sum_i R_i^T D_i R_i = I;
//  * B_i: the Maxwell operator of the tetrahedra of T_i^delta, with the
//    physical boundary terms of the labelled faces they own, plus the
//    impedance transmission term i k int (E x n).(v x n) on every face of
//    T_i^delta that is shared with a tetrahedron outside it (k from the
//    owning tetrahedron, evaluated on the device so that it follows eps).
// This file builds the index lists; the dense B_i are filled on the device.
#include <algorithm>

#include "common.hpp"
#include "parallel.hpp"

namespace mw {

// local faces of a tetrahedron with ascending vertices and the tet-local
// edges (in the face's (0,1),(0,2),(1,2) order) that bound them
static const int kFaceVert[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
static const int kFaceEdge[4][3] = {{0, 1, 3}, {0, 2, 4}, {1, 2, 5}, {3, 4, 5}};

namespace {
struct SubTmp {
  int32_t n_lead = 0;
  std::vector<int32_t> fgrp;   // per 32-row group: first column of the rows' envelope
  std::vector<int32_t> hgrp;   // per 32-row group: one past the last column whose envelope reaches it
  std::vector<int32_t> tets, edges, lt_loc, lf_vert, lf_owner, lf_kind, lf_loc;
  std::vector<double> D;
  std::vector<int64_t> rtl_ptr, rfl_ptr;
  std::vector<int32_t> rtl, rfl;
};
struct Scratch {
  std::vector<int32_t> node0, node, tet, edge, eloc;
};

// Breadth-first levels of the component of `start` (level[] = -1 for unseen
// vertices on entry); returns the vertices in visiting order and sets `depth`.
std::vector<int32_t> bfs_levels(int32_t start, const std::vector<int32_t>& ptr, const std::vector<int32_t>& adj,
                                std::vector<int32_t>& level, int32_t& depth) {
  std::vector<int32_t> seq{start};
  level[start] = 0;
  depth = 0;
  for (size_t h = 0; h < seq.size(); ++h) {
    const int32_t u = seq[h];
    for (int32_t q = ptr[u]; q < ptr[u + 1]; ++q)
      if (level[adj[q]] < 0) {
        level[adj[q]] = level[u] + 1;
        depth = std::max(depth, level[u] + 1);
        seq.push_back(adj[q]);
      }
  }
  return seq;
}

// Reverse Cuthill-McKee order of a symmetric graph (Cuthill & McKee 1969,
// reversed as in George & Liu, Computer Solution of Large Sparse Positive
// Definite Systems, 1981): per connected component, a pseudo-peripheral start
// (repeated breadth-first search from a vertex of least degree in the last
// level while the depth grows), then a breadth-first order that visits each
// vertex's unnumbered neighbours by increasing degree (ties: lower index); the
// whole sequence reversed.  Keeps the nonzeros of every row close to the
// diagonal, and factorisation without interchanges fills only that envelope.
std::vector<int32_t> rcm_order(int32_t n, const std::vector<int32_t>& ptr, const std::vector<int32_t>& adj) {
  auto deg = [&](int32_t v) { return ptr[v + 1] - ptr[v]; };
  std::vector<int32_t> order, level(n, -1), mark(n, 0);
  order.reserve(n);
  for (int32_t seed = 0; seed < n; ++seed) {
    if (mark[seed]) continue;
    int32_t start = seed, depth = 0;
    std::vector<int32_t> comp = bfs_levels(start, ptr, adj, level, depth);
    for (int round = 0; round < 8; ++round) {
      int32_t best = -1;
      for (int32_t v : comp)
        if (level[v] == depth && (best < 0 || deg(v) < deg(best) || (deg(v) == deg(best) && v < best))) best = v;
      for (int32_t v : comp) level[v] = -1;
      int32_t d2 = 0;
      std::vector<int32_t> c2 = bfs_levels(best, ptr, adj, level, d2);
      comp.swap(c2);               // same vertex set, levels now from `best`
      if (d2 <= depth) break;
      start = best;
      depth = d2;
    }
    for (int32_t v : comp) level[v] = -1;
    // Cuthill-McKee sweep of the component
    const size_t first = order.size();
    order.push_back(start);
    mark[start] = 1;
    std::vector<int32_t> nbr;
    for (size_t h = first; h < order.size(); ++h) {
      const int32_t u = order[h];
      nbr.clear();
      for (int32_t q = ptr[u]; q < ptr[u + 1]; ++q)
        if (!mark[adj[q]]) { mark[adj[q]] = 1; nbr.push_back(adj[q]); }
      std::sort(nbr.begin(), nbr.end(), [&](int32_t a, int32_t b) {
        return deg(a) != deg(b) ? deg(a) < deg(b) : a < b;
      });
      order.insert(order.end(), nbr.begin(), nbr.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}
}  // namespace

void build_decomposition(const Topology& T, const int32_t* part, int32_t nsub, int32_t delta,
                         int32_t block, Decomposition& out) {
  const int32_t nv = T.nv, nt = T.nt;
  const int64_t ne = T.ne(), n = T.n();
  MW_CHECK(nsub >= 1, MW_EINVAL, "n_sub must be >= 1");
  MW_CHECK(delta >= 1, MW_EINVAL, "overlap must be >= 1");
  MW_CHECK(part != nullptr, MW_EINVAL, "tet_part is NULL");
  for (int32_t t = 0; t < nt; ++t)
    MW_CHECK(part[t] >= 0 && part[t] < nsub, MW_EINVAL, "tet_part value out of [0, n_sub)");

  // part -> tetrahedra
  std::vector<int64_t> pt_ptr(nsub + 1, 0);
  for (int32_t t = 0; t < nt; ++t) pt_ptr[part[t] + 1]++;
  for (int32_t i = 0; i < nsub; ++i) {
    MW_CHECK(pt_ptr[i + 1] > 0, MW_EINVAL, "tet_part leaves subdomain " + std::to_string(i) + " empty");
    pt_ptr[i + 1] += pt_ptr[i];
  }
  std::vector<int32_t> pt(nt);
  {
    std::vector<int64_t> fill(pt_ptr.begin(), pt_ptr.end() - 1);
    for (int32_t t = 0; t < nt; ++t) pt[fill[part[t]]++] = t;
  }
  // vertex -> tetrahedra
  std::vector<int64_t> vt_ptr(nv + 1, 0);
  for (int64_t i = 0; i < (int64_t)nt * 4; ++i) vt_ptr[T.tet[i] + 1]++;
  for (int32_t v = 0; v < nv; ++v) vt_ptr[v + 1] += vt_ptr[v];
  std::vector<int32_t> vt(vt_ptr[nv]);
  {
    std::vector<int64_t> fill(vt_ptr.begin(), vt_ptr.end() - 1);
    for (int32_t t = 0; t < nt; ++t)
      for (int k = 0; k < 4; ++k) vt[fill[T.tet[(size_t)t * 4 + k]]++] = t;
  }
  // number of subdomains whose T_j^0 holds each node (denominator of (chi))
  std::vector<float> cnt(nv, 0.f);
  parallel_for(nv, [&](int64_t v) {
    // distinct parts among the tetrahedra around v (at most their number)
    int32_t small[64];
    std::vector<int32_t> big;
    const int64_t deg = vt_ptr[v + 1] - vt_ptr[v];
    int32_t* seen = small;
    if (deg > 64) {
      big.resize(deg);
      seen = big.data();
    }
    int ns = 0;
    for (int64_t q = vt_ptr[v]; q < vt_ptr[v + 1]; ++q) {
      int32_t p = part[vt[q]];
      bool dup = false;
      for (int k = 0; k < ns; ++k) dup |= seen[k] == p;
      if (!dup) seen[ns++] = p;
    }
    cnt[v] = (float)ns;
  });
  // neighbour across each tetrahedron face, and labelled boundary face of it
  std::vector<int32_t> nb((size_t)nt * 4, -1), tf2bf((size_t)nt * 4, -1);
  parallel_for(nt, [&](int64_t t) {
    const int32_t* tv = &T.tet[t * 4];
    for (int f = 0; f < 4; ++f) {
      int32_t a = tv[kFaceVert[f][0]], b = tv[kFaceVert[f][1]], c = tv[kFaceVert[f][2]];
      for (int64_t q = vt_ptr[a]; q < vt_ptr[a + 1]; ++q) {
        int32_t u = vt[q];
        if (u == t) continue;
        const int32_t* uv = &T.tet[(size_t)u * 4];
        bool hb = false, hc = false;
        for (int k = 0; k < 4; ++k) { hb |= uv[k] == b; hc |= uv[k] == c; }
        if (hb && hc) { nb[t * 4 + f] = u; break; }
      }
    }
  });
  for (int32_t f = 0; f < T.nbf; ++f) {
    int32_t t = T.bf_owner[f];
    const int32_t* tv = &T.tet[(size_t)t * 4];
    for (int lf = 0; lf < 4; ++lf)
      if (tv[kFaceVert[lf][0]] == T.bface[f * 3] && tv[kFaceVert[lf][1]] == T.bface[f * 3 + 1] &&
          tv[kFaceVert[lf][2]] == T.bface[f * 3 + 2])
        tf2bf[(size_t)t * 4 + lf] = f;
  }

  std::vector<SubTmp> sub(nsub);
  std::vector<Scratch> scr(host_threads());
  parallel_items(nsub, [&](int w, int64_t i) {
    Scratch& s = scr[w];
    if (s.node.empty()) {
      s.node0.assign(nv, -1); s.node.assign(nv, -1); s.tet.assign(nt, -1);
      s.edge.assign(ne, -1); s.eloc.assign(ne, -1);
    }
    SubTmp& o = sub[i];
    const int32_t stamp = (int32_t)i;
    std::vector<int32_t> front;
    for (int64_t q = pt_ptr[i]; q < pt_ptr[i + 1]; ++q) {
      int32_t t = pt[q];
      s.tet[t] = stamp;
      o.tets.push_back(t);
      for (int k = 0; k < 4; ++k) {
        int32_t v = T.tet[(size_t)t * 4 + k];
        if (s.node0[v] != stamp) { s.node0[v] = stamp; s.node[v] = stamp; front.push_back(v); }
      }
    }
    for (int32_t d = 0; d < delta; ++d) {
      std::vector<int32_t> added;
      for (int32_t v : front)
        for (int64_t q = vt_ptr[v]; q < vt_ptr[v + 1]; ++q) {
          int32_t t = vt[q];
          if (s.tet[t] != stamp) { s.tet[t] = stamp; o.tets.push_back(t); added.push_back(t); }
        }
      front.clear();
      for (int32_t t : added)
        for (int k = 0; k < 4; ++k) {
          int32_t v = T.tet[(size_t)t * 4 + k];
          if (s.node[v] != stamp) { s.node[v] = stamp; front.push_back(v); }
        }
    }
    std::sort(o.tets.begin(), o.tets.end());
    for (int32_t t : o.tets)
      for (int p = 0; p < 6; ++p) {
        int32_t e = T.t2e[(size_t)t * 6 + p];
        if (!T.pec[e] && s.edge[e] != stamp) { s.edge[e] = stamp; o.edges.push_back(e); }
      }
    std::sort(o.edges.begin(), o.edges.end());
    const int32_t ni = (int32_t)o.edges.size();
    // weights, then the local numbering: reverse Cuthill-McKee on the graph
    // of B_i (two unknowns coupled when they share a tetrahedron), so that
    // the dense factors are banded and the triangular solves skip the zero
    // tiles outside the envelope; n_lead counts the leading unknowns with
    // D = 0 (discarded after the local solve: the backward substitution
    // stops at the first block holding a weighted unknown)
    std::vector<double> Dg(ni);
    for (int32_t l = 0; l < ni; ++l) {
      int64_t e = o.edges[l];
      int32_t a = (int32_t)T.edges[e * 2], b = (int32_t)T.edges[e * 2 + 1];
      double ca = s.node0[a] == stamp ? 1.0 / cnt[a] : 0.0;
      double cb = s.node0[b] == stamp ? 1.0 / cnt[b] : 0.0;
      Dg[l] = 0.5 * (ca + cb);
    }
    {
      for (int32_t l = 0; l < ni; ++l) s.eloc[o.edges[l]] = l;
      std::vector<int64_t> pairs;
      for (int32_t t : o.tets) {
        int32_t loc[6];
        int m = 0;
        for (int p = 0; p < 6; ++p) {
          int32_t e = T.t2e[(size_t)t * 6 + p];
          if (!T.pec[e]) loc[m++] = s.eloc[e];
        }
        for (int a = 0; a < m; ++a)
          for (int b = 0; b < m; ++b)
            if (a != b) pairs.push_back((int64_t)loc[a] * ni + loc[b]);
      }
      std::sort(pairs.begin(), pairs.end());
      pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
      std::vector<int32_t> gptr(ni + 1, 0), gadj(pairs.size());
      for (size_t q = 0; q < pairs.size(); ++q) {
        gptr[pairs[q] / ni + 1]++;
        gadj[q] = (int32_t)(pairs[q] % ni);
      }
      for (int32_t l = 0; l < ni; ++l) gptr[l + 1] += gptr[l];
      std::vector<int32_t> ord = rcm_order(ni, gptr, gadj);
      int32_t z = 0;
      while (z < ni && Dg[ord[z]] == 0.0) ++z;
      o.n_lead = z;
      // envelope of B_i in the new order: first coupled column of every row
      // (the pattern is symmetric, so this also bounds every column from
      // above); factorisation without interchanges fills only inside it
      {
        std::vector<int32_t> inv(ni);
        for (int32_t k = 0; k < ni; ++k) inv[ord[k]] = k;
        const int32_t npad0 = (int32_t)round_up(std::max(ni, 1), block);
        o.fgrp.assign(npad0 / 32, 0);
        for (int32_t g = 0; g < npad0 / 32; ++g) o.fgrp[g] = 32 * g;
        // hgrp[g]: columns c with first(c) <= 32g + 31 end before it
        o.hgrp.assign(npad0 / 32, 0);
        std::vector<int32_t> best(npad0 / 32, -1);
        for (int32_t k = 0; k < ni; ++k) {
          int32_t f = k;
          for (int32_t q = gptr[ord[k]]; q < gptr[ord[k] + 1]; ++q) f = std::min(f, inv[gadj[q]]);
          o.fgrp[k / 32] = std::min(o.fgrp[k / 32], f);
          best[f / 32] = std::max(best[f / 32], k);
        }
        int32_t run = -1;
        for (int32_t g = 0; g < npad0 / 32; ++g) {
          run = std::max(run, best[g]);
          o.hgrp[g] = std::max(32 * g + 32, run + 1);
        }
      }
      std::vector<int32_t> e2(ni);
      o.D.resize(ni);
      for (int32_t l = 0; l < ni; ++l) { e2[l] = o.edges[ord[l]]; o.D[l] = Dg[ord[l]]; }
      o.edges.swap(e2);
    }
    for (int32_t l = 0; l < ni; ++l) s.eloc[o.edges[l]] = l;
    auto lidx = [&](int32_t e) -> int32_t { return T.pec[e] ? -1 : s.eloc[e]; };
    o.lt_loc.resize(o.tets.size() * 6);
    for (size_t k = 0; k < o.tets.size(); ++k) {
      int32_t t = o.tets[k];
      for (int p = 0; p < 6; ++p) o.lt_loc[k * 6 + p] = lidx(T.t2e[(size_t)t * 6 + p]);
      for (int f = 0; f < 4; ++f) {
        int32_t u = nb[(size_t)t * 4 + f];
        int32_t kind;
        if (u >= 0) {
          if (s.tet[u] == stamp) continue;      // interior face of T_i^delta
          kind = -1;                            // interface face
        } else {
          int32_t bf = tf2bf[(size_t)t * 4 + f];
          if (bf < 0 || T.btag[bf] == MW_TAG_PEC) continue;  // natural or PEC: no term
          kind = bf;
        }
        for (int k2 = 0; k2 < 3; ++k2) {
          o.lf_vert.push_back(T.tet[(size_t)t * 4 + kFaceVert[f][k2]]);
          o.lf_loc.push_back(lidx(T.t2e[(size_t)t * 6 + kFaceEdge[f][k2]]));
        }
        o.lf_owner.push_back(t);
        o.lf_kind.push_back(kind);
      }
    }
    // per local row: contributing (entry, local edge) pairs, in entry order
    const int32_t npad = (int32_t)round_up(std::max(ni, 1), block);
    o.rtl_ptr.assign(npad + 1, 0);
    for (int32_t v : o.lt_loc) if (v >= 0) o.rtl_ptr[v + 1]++;
    for (int32_t l = 0; l < npad; ++l) o.rtl_ptr[l + 1] += o.rtl_ptr[l];
    o.rtl.resize(o.rtl_ptr[npad]);
    {
      std::vector<int64_t> fill(o.rtl_ptr.begin(), o.rtl_ptr.end() - 1);
      for (size_t k = 0; k < o.lt_loc.size(); ++k)
        if (o.lt_loc[k] >= 0) o.rtl[fill[o.lt_loc[k]]++] = (int32_t)k;   // k = entry*6 + p
    }
    o.rfl_ptr.assign(npad + 1, 0);
    for (int32_t v : o.lf_loc) if (v >= 0) o.rfl_ptr[v + 1]++;
    for (int32_t l = 0; l < npad; ++l) o.rfl_ptr[l + 1] += o.rfl_ptr[l];
    o.rfl.resize(o.rfl_ptr[npad]);
    {
      std::vector<int64_t> fill(o.rfl_ptr.begin(), o.rfl_ptr.end() - 1);
      for (size_t k = 0; k < o.lf_loc.size(); ++k)
        if (o.lf_loc[k] >= 0) o.rfl[fill[o.lf_loc[k]]++] = (int32_t)k;   // k = entry*3 + p
    }
  });

  // ---- concatenate
  Decomposition& D = out;
  D = Decomposition();
  D.nsub = nsub; D.delta = delta;
  D.n_loc.resize(nsub); D.n_pad.resize(nsub); D.n_lead.resize(nsub);
  {
    size_t mg = 1;
    for (int32_t i = 0; i < nsub; ++i) mg = std::max(mg, sub[i].fgrp.size());
    D.fenv_stride = (int32_t)mg;
    D.fenv.assign((size_t)nsub * mg, 0);
    D.fenv_hi.assign((size_t)nsub * mg, 0);
    for (int32_t i = 0; i < nsub; ++i) {
      std::copy(sub[i].fgrp.begin(), sub[i].fgrp.end(), D.fenv.begin() + (size_t)i * mg);
      std::copy(sub[i].hgrp.begin(), sub[i].hgrp.end(), D.fenv_hi.begin() + (size_t)i * mg);
    }
  }
  D.loc_off.assign(nsub + 1, 0); D.fac_off.assign(nsub + 1, 0);
  D.lt_off.assign(nsub + 1, 0); D.lf_off.assign(nsub + 1, 0);
  for (int32_t i = 0; i < nsub; ++i) {
    D.n_loc[i] = (int32_t)sub[i].edges.size();
    D.n_lead[i] = sub[i].n_lead;
    D.n_pad[i] = (int32_t)round_up(std::max(D.n_loc[i], 1), block);
    D.loc_off[i + 1] = D.loc_off[i] + D.n_pad[i];
    D.fac_off[i + 1] = D.fac_off[i] + (int64_t)D.n_pad[i] * D.n_pad[i];
    D.lt_off[i + 1] = D.lt_off[i] + (int64_t)sub[i].tets.size();
    D.lf_off[i + 1] = D.lf_off[i] + (int64_t)sub[i].lf_owner.size();
  }
  // factor storage tables (64-row blocks; block size and n_pad are multiples of 64)
  {
    int32_t mp = 0;
    for (int32_t i = 0; i < nsub; ++i) mp = std::max(mp, D.n_pad[i]);
    D.bstride = std::max(1, mp / 64);
    const size_t tot = (size_t)nsub * D.bstride;
    D.boff_dense.assign(tot, 0); D.boff_band.assign(tot, 0);
    D.blo_dense.assign(tot, 0); D.blo_band.assign(tot, 0);
    D.bw_dense.assign(tot, 0); D.bw_band.assign(tot, 0);
    D.fac_off_band.assign(nsub + 1, 0);
    for (int32_t i = 0; i < nsub; ++i) {
      const int32_t np = D.n_pad[i];
      const int32_t* fe = D.fenv.data() + (size_t)i * D.fenv_stride;
      const int32_t* fh = D.fenv_hi.data() + (size_t)i * D.fenv_stride;
      int64_t off = 0;
      for (int32_t b = 0; b < np / 64; ++b) {
        const size_t e = (size_t)i * D.bstride + b;
        D.boff_dense[e] = (int64_t)64 * b * np;
        D.blo_dense[e] = 0;
        D.bw_dense[e] = np;
        int32_t lo = std::min(std::min(fe[2 * b], fe[2 * b + 1]) & ~63, 64 * b);
        int32_t hi = (int32_t)round_up(std::max(fh[2 * b], fh[2 * b + 1]), 64);
        hi = std::max(hi, std::min(np, 64 * b + 128));
        hi = std::min(std::max(hi, 64 * b + 64), np);
        D.blo_band[e] = lo;
        D.bw_band[e] = hi - lo;
        D.boff_band[e] = off;
        off += (int64_t)64 * (hi - lo);
      }
      D.fac_off_band[i + 1] = D.fac_off_band[i] + off;
    }
  }
  const int64_t sp = D.loc_off[nsub];
  D.sub_dof.assign(sp, -1);
  D.D.assign(sp, 0.0);
  D.lt_tet.resize(D.lt_off[nsub]); D.lt_loc.resize(D.lt_off[nsub] * 6);
  D.lf_vert.resize(D.lf_off[nsub] * 3); D.lf_loc.resize(D.lf_off[nsub] * 3);
  D.lf_owner.resize(D.lf_off[nsub]); D.lf_kind.resize(D.lf_off[nsub]);
  D.rtl_ptr.assign(sp + 1, 0); D.rfl_ptr.assign(sp + 1, 0);
  int64_t nrtl = 0, nrfl = 0;
  for (int32_t i = 0; i < nsub; ++i) { nrtl += sub[i].rtl.size(); nrfl += sub[i].rfl.size(); }
  D.rtl.resize(nrtl); D.rfl.resize(nrfl);
  {
    int64_t wt = 0, wf = 0;
    for (int32_t i = 0; i < nsub; ++i) {
      const SubTmp& o = sub[i];
      int64_t r0 = D.loc_off[i];
      for (int32_t l = 0; l < D.n_loc[i]; ++l) {
        D.sub_dof[r0 + l] = T.dof[o.edges[l]];
        D.D[r0 + l] = o.D[l];
      }
      std::copy(o.tets.begin(), o.tets.end(), D.lt_tet.begin() + D.lt_off[i]);
      std::copy(o.lt_loc.begin(), o.lt_loc.end(), D.lt_loc.begin() + D.lt_off[i] * 6);
      std::copy(o.lf_vert.begin(), o.lf_vert.end(), D.lf_vert.begin() + D.lf_off[i] * 3);
      std::copy(o.lf_loc.begin(), o.lf_loc.end(), D.lf_loc.begin() + D.lf_off[i] * 3);
      std::copy(o.lf_owner.begin(), o.lf_owner.end(), D.lf_owner.begin() + D.lf_off[i]);
      std::copy(o.lf_kind.begin(), o.lf_kind.end(), D.lf_kind.begin() + D.lf_off[i]);
      for (int32_t l = 0; l < D.n_pad[i]; ++l) {
        D.rtl_ptr[r0 + l + 1] = D.rtl_ptr[r0 + l] + (o.rtl_ptr[l + 1] - o.rtl_ptr[l]);
        D.rfl_ptr[r0 + l + 1] = D.rfl_ptr[r0 + l] + (o.rfl_ptr[l + 1] - o.rfl_ptr[l]);
      }
      std::copy(o.rtl.begin(), o.rtl.end(), D.rtl.begin() + wt);
      std::copy(o.rfl.begin(), o.rfl.end(), D.rfl.begin() + wf);
      wt += o.rtl.size(); wf += o.rfl.size();
    }
  }
  // prolongation copies of every dof, ascending subdomain order
  // (copies with a zero weight contribute nothing and are left out)
  D.cp_ptr.assign(n + 1, 0);
  for (int64_t r = 0; r < sp; ++r) if (D.sub_dof[r] >= 0 && D.D[r] != 0.0) D.cp_ptr[D.sub_dof[r] + 1]++;
  for (int64_t g = 0; g < n; ++g) {
    MW_CHECK(D.cp_ptr[g + 1] > 0, MW_EINVAL, "decomposition leaves an unknown uncovered");
    D.cp_ptr[g + 1] += D.cp_ptr[g];
  }
  D.cp_row.resize(D.cp_ptr[n]);
  {
    // ascending subdomain order for every unknown
    std::vector<int64_t> fill(D.cp_ptr.begin(), D.cp_ptr.end() - 1);
    for (int64_t r = 0; r < sp; ++r)
      if (D.sub_dof[r] >= 0 && D.D[r] != 0.0) D.cp_row[fill[D.sub_dof[r]]++] = r;
  }
}

// Non-overlapping partition T_i of the tetrahedra (Section 3 starts from one;
// the paper takes it from a graph partitioner) by recursive coordinate
// bisection of the tetrahedron centroids: the current set is split across
// the axis of largest centroid extent (ties: lowest axis) so that the lower
// side holds floor(count * nl / np) tetrahedra for nl = floor(np / 2) of its
// np parts, ordered by (coordinate, tetrahedron id); each side is split
// again until one part is left.  Every part then holds floor(nt / nsub) or
// one more tetrahedron; only the mesh geometry decides, so any tetrahedral
// mesh can be split.
void partition_rcb(const Topology& T, int32_t nsub, std::vector<int32_t>& part) {
  const int32_t nt = T.nt;
  MW_CHECK(nsub >= 1 && nsub <= nt, MW_EINVAL, "n_sub must lie in [1, number of tetrahedra]");
  std::vector<double> cen((size_t)nt * 3);
  for (int32_t t = 0; t < nt; ++t)
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += T.xyz[3 * (size_t)T.tet[4 * (size_t)t + k] + a];
      cen[3 * (size_t)t + a] = 0.25 * s;
    }
  std::vector<int32_t> ids(nt);
  for (int32_t t = 0; t < nt; ++t) ids[t] = t;
  part.assign(nt, 0);
  struct Range { int64_t lo, hi; int32_t p0, np; };
  std::vector<Range> todo{{0, nt, 0, nsub}};
  while (!todo.empty()) {
    Range r = todo.back();
    todo.pop_back();
    if (r.np == 1) {
      for (int64_t k = r.lo; k < r.hi; ++k) part[ids[k]] = r.p0;
      continue;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t k = r.lo; k < r.hi; ++k)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], cen[3 * (size_t)ids[k] + a]);
        hi[a] = std::max(hi[a], cen[3 * (size_t)ids[k] + a]);
      }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    const int32_t nl = r.np / 2;
    const int64_t cut = r.lo + (r.hi - r.lo) * nl / r.np;
    auto less = [&](int32_t a, int32_t b) {
      const double xa = cen[3 * (size_t)a + ax], xb = cen[3 * (size_t)b + ax];
      return xa < xb || (xa == xb && a < b);
    };
    if (cut > r.lo && cut < r.hi) std::nth_element(ids.begin() + r.lo, ids.begin() + cut, ids.begin() + r.hi, less);
    todo.push_back({cut, r.hi, r.p0 + nl, r.np - nl});
    todo.push_back({r.lo, cut, r.p0, nl});
  }
}

}  // namespace mw
