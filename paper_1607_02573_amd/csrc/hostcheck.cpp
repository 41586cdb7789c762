// Host-only inspection of the edge topology and the overlapping
// decomposition (no device needed): lets the host logic be checked against
// an independent implementation on machines without a GPU.
#include <cstring>
#include <numeric>

#include "blockls.hpp"
#include "common.hpp"

using namespace mw;

#include <functional>

static thread_local std::string g_host_err;

static mw_status hguard(const std::function<void()>& f) {
  try {
    f();
    return MW_OK;
  } catch (const Error& e) {
    g_host_err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_host_err = e.what();
    return MW_EINVAL;
  }
}

extern "C" {

const char* mw_host_last_error(void) { return g_host_err.c_str(); }

mw_status mw_host_topology(const mw_mesh* mesh, int64_t* n, int64_t* nnz, int64_t* n_edges, int32_t* edge_of_dof,
                           int64_t* row_ptr, int32_t* col) {
  return hguard([&] {
    MW_CHECK(mesh && n && nnz && n_edges, MW_EINVAL, "NULL argument");
    Topology T;
    build_topology(*mesh, T);
    *n = T.n();
    *nnz = (int64_t)T.col.size();
    *n_edges = T.ne();
    if (edge_of_dof) std::copy(T.free_edge.begin(), T.free_edge.end(), edge_of_dof);
    if (row_ptr) std::copy(T.row_ptr.begin(), T.row_ptr.end(), row_ptr);
    if (col) std::copy(T.col.begin(), T.col.end(), col);
  });
}

mw_status mw_host_decomposition(const mw_mesh* mesh, const int32_t* tet_part, int32_t n_sub, int32_t overlap,
                                int32_t* n_loc, int64_t* n_faces, int32_t* sub_dof, double* D) {
  return hguard([&] {
    MW_CHECK(mesh && tet_part && n_loc, MW_EINVAL, "NULL argument");
    Topology T;
    build_topology(*mesh, T);
    Decomposition Dc;
    build_decomposition(T, tet_part, n_sub, overlap, 64, Dc);
    int64_t w = 0;
    for (int32_t i = 0; i < n_sub; ++i) {
      n_loc[i] = Dc.n_loc[i];
      if (n_faces) n_faces[i] = Dc.lf_off[i + 1] - Dc.lf_off[i];
      for (int32_t l = 0; l < Dc.n_loc[i]; ++l) {
        if (sub_dof) sub_dof[w] = Dc.sub_dof[Dc.loc_off[i] + l];
        if (D) D[w] = Dc.D[Dc.loc_off[i] + l];
        ++w;
      }
    }
  });
}

mw_status mw_host_factor_storage(const mw_mesh* mesh, const int32_t* tet_part, int32_t n_sub, int32_t overlap,
                                 int32_t sub, int32_t* blk_lo, int32_t* blk_hi, int64_t* dense_elems,
                                 int64_t* band_elems) {
  return hguard([&] {
    MW_CHECK(mesh && tet_part, MW_EINVAL, "NULL argument");
    Topology T;
    build_topology(*mesh, T);
    Decomposition Dc;
    build_decomposition(T, tet_part, n_sub, overlap, 64, Dc);
    MW_CHECK(sub >= 0 && sub < n_sub, MW_EINVAL, "subdomain out of range");
    if (dense_elems) *dense_elems = Dc.fac_off.back();
    if (band_elems) *band_elems = Dc.fac_off_band.back();
    for (int32_t b = 0; b < Dc.n_pad[sub] / 64; ++b) {
      const size_t e = (size_t)sub * Dc.bstride + b;
      if (blk_lo) blk_lo[b] = Dc.blo_band[e];
      if (blk_hi) blk_hi[b] = Dc.blo_band[e] + Dc.bw_band[e];
    }
  });
}

mw_status mw_host_partition(const mw_mesh* mesh, int32_t n_sub, int32_t* tet_part) {
  return hguard([&] {
    MW_CHECK(mesh && tet_part, MW_EINVAL, "NULL argument");
    Topology T;
    build_topology(*mesh, T);
    std::vector<int32_t> part;
    partition_rcb(T, n_sub, part);
    std::copy(part.begin(), part.end(), tet_part);
  });
}

mw_status mw_host_block_lstsq(int32_t steps, int32_t width, const mw_complex* S0, const mw_complex* H, double thr,
                              double* resid, mw_complex* Y) {
  return hguard([&] {
    MW_CHECK(steps >= 0 && width >= 1 && width <= BW && H, MW_EINVAL, "invalid block least-squares arguments");
    const zc* Hz = reinterpret_cast<const zc*>(H);
    if (steps == 0) {
      double dmax = 0.0;
      for (int c = 0; c < BW; ++c) dmax = std::max(dmax, Hz[c * BW + c].real());
      std::vector<zc> R(BW * BW);
      int nd = chol_upper(Hz, BW, thr * thr * dmax, R.data());
      if (resid) resid[0] = nd;
      if (Y) std::copy(R.begin(), R.end(), reinterpret_cast<zc*>(Y));
      return;
    }
    MW_CHECK(S0 != nullptr, MW_EINVAL, "NULL argument");
    const int64_t ldh = (int64_t)steps * BW;
    BlockLS ls;
    ls.start(steps, reinterpret_cast<const zc*>(S0), width);
    std::vector<zc> Hc((size_t)(steps + 1) * BW * BW), R(BW * BW);
    for (int j = 0; j < steps; ++j) {
      for (int64_t r = 0; r < (int64_t)(j + 1) * BW; ++r)
        for (int t = 0; t < BW; ++t) Hc[r * BW + t] = Hz[r * ldh + (int64_t)j * BW + t];
      for (int r = 0; r < BW; ++r)
        for (int t = 0; t < BW; ++t) R[r * BW + t] = Hz[((int64_t)(j + 1) * BW + r) * ldh + (int64_t)j * BW + t];
      ls.add(Hc.data(), R.data());
      if (resid)
        for (int c = 0; c < BW; ++c) resid[(int64_t)j * BW + c] = ls.resid(c);
    }
    if (Y) ls.solve(reinterpret_cast<zc*>(Y));
  });
}

}  // extern "C"
