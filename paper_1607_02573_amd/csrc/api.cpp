// C ABI of the library (include/mw.h): context and problem objects, the
// byte budget, and the host drivers of assembly, subdomain factorisation and
// the preconditioned pseudo-block GMRES.  All arithmetic runs in the HIP
// kernels; the host only orders launches, moves index lists and reads back
// per-column convergence flags.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <type_traits>
#include <mutex>
#include <numeric>

#include "blockls.hpp"
#include "internal.hpp"
#include "parallel.hpp"

using namespace mw;

static thread_local std::string g_last_error;

// Fixed device buffer of mw_apply_preconditioner_noalloc: the local vectors
// R_i v of every subdomain live here instead of in an allocated workspace.
// Each device that loads the library holds one copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in).
static __device__ __align__(256) char scratch[MW_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`; looked up once per
// device (at mw_create), with that device current.
void* scratch_for_device(int device, bool lookup) {
  MW_CHECK(device >= 0 && device < kMaxDevices, MW_EINVAL, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr && lookup) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      fail(MW_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}
}  // namespace

struct mw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;     // default stream of problems created on this context
  int64_t budget = 0;
  std::atomic<int64_t> used{0};     // bytes held; problems may be driven from several threads
};

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

DevBuf dalloc(mw_ctx* c, int64_t bytes) {
  DevBuf b;
  if (bytes <= 0) return b;
  int64_t cur = c->used.load();
  do {
    if (cur + bytes > c->budget)
      fail(MW_ENOMEM, "HBM budget exceeded: need " + std::to_string(bytes) + " more bytes, " +
                          std::to_string(c->budget - cur) + " of " + std::to_string(c->budget) + " left");
  } while (!c->used.compare_exchange_weak(cur, cur + bytes));
  hipError_t e = hipMalloc(&b.p, (size_t)bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->used.fetch_sub(bytes);
    fail(MW_ENOMEM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  b.bytes = (size_t)bytes;
  b.ledger = &c->used;
  return b;
}

template <class T>
DevBuf upload(mw_ctx* c, hipStream_t st, const std::vector<T>& v) {
  DevBuf b = dalloc(c, (int64_t)(v.size() * sizeof(T)));
  if (!v.empty()) MW_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return b;
}

// A resizable device workspace (grown on demand, never shrunk).
struct Work {
  DevBuf b;
  void* get(mw_ctx* c, int64_t bytes) {
    if ((int64_t)b.bytes < bytes) {
      b.release();
      b = dalloc(c, bytes);
    }
    return b.p;
  }
};

// Device workspaces of one pseudo-block GMRES driver (mw_solve, or one
// batch), grown on demand.
struct GmresWork {
  Work V, X, B, Z, Y, H, Hr, cs, sn, g, y, h1, h2, hp, cf, nu, ee, part, npart, vec, ints, tmp, w_idx;
  Work cq, cw, cy;            // two-level: Q v, FP64 copy of an FP32 basis vector, coarse vector
  Work zc, rc;                // FP32 basis: preconditioned candidates and their triangular factor
  Work csc;                   // FP32 basis: 1 / ||u|| of the unnormalised candidate, per column
  hipStream_t st = nullptr;   // the stream this driver's work runs on
  std::array<Work*, 29> all() {
    return {&V, &X, &B, &Z, &Y, &H, &Hr, &cs, &sn, &g, &y, &h1, &h2, &hp, &cf, &nu, &ee, &part, &npart, &vec, &ints,
            &tmp, &w_idx, &cq, &cw, &cy, &zc, &rc, &csc};
  }
  void release() {
    for (Work* w : all()) w->b.release();
  }
  int64_t held() {
    int64_t s = 0;
    for (Work* w : all()) s += (int64_t)w->b.bytes;
    return s;
  }
};

}  // namespace

struct mw_problem {
  mw_ctx* ctx = nullptr;
  Topology T;
  double k0 = 0;
  mw_complex beta_imp{0, 0};
  std::vector<mw_port> ports;
  // mesh and operator
  DevBuf xyz, tet, t2e, dof, bface, bf2e, fbeta, row_ptr, col, rt_ptr, rt, rf_ptr, rf, rorder;
  DevBuf sl_row, sl_off, sl_col, sl_idx, sl_val;   // sliced ELLPACK copy of A (products with few columns)
  DevBuf eps, E, val;
  // eps_r linear on every tetrahedron (mw_update_eps_vertex): vertex values,
  // and the (t*4 + slot) entries of every vertex for the vertex gradient
  bool eps_p1 = false;
  DevBuf eps_v, vt_ptr, vt;
  DeviceMesh dm;
  // ports
  DevBuf port_dev, port_ptr, ent_dof, ent_port, ent_ptr, ent_fq, pf_ptr, pf, pval, nu;
  DevicePorts dp;
  // decomposition and factors
  bool has_dec = false;
  uint64_t dec_key = 0;
  Decomposition D;
  DevBuf d_fac_off, d_loc_off, d_n_loc, d_n_pad, d_lt_off, d_lt_tet, d_lt_loc, d_lf_off, d_lf_vert, d_lf_owner,
      d_lf_kind, d_lf_loc, d_rtl_ptr, d_rtl, d_rfl_ptr, d_rfl, d_sub_dof, d_D, d_cp_ptr, d_cp_row, d_ipiv, d_ridx,
      d_info, d_amax, d_row_lo, d_env, d_fenv, d_fenvh, d_order;
  std::vector<int32_t> h_row_lo;
  std::vector<int2> h_env;
  DeviceDecomp dd;
  DevBuf F;
  int prec = -1;
  int factor_kind = MW_FACTOR_AUTO;   // requested
  int solve_form = MW_SOLVE_AUTO;      // requested (mw_set_solve_form)
  int basis = MW_BASIS_AUTO;           // Krylov basis precision (mw_set_krylov_basis)
  int factorization = 0;              // used by the current factors (MW_FACTOR_LU / MW_FACTOR_LDLT)
  bool factors_valid = false;
  // factor storage of F: banded (L D L^T, no interchanges) or dense (LU)
  bool banded = false;
  DevBuf d_boff_dense, d_blo_dense, d_bw_dense, d_boff_band, d_blo_band, d_bw_band, d_fac_off_band;
  // workspaces of mw_solve / mw_apply_preconditioner, and of small index lists
  GmresWork ws;
  Work w_small;
  hipStream_t stream = nullptr;    // every launch and copy of this problem
  int live_batches = 0;
  int live_users = 0;                // inversions driving this problem
  // bumped by every call that changes the operator or the factors (eps,
  // factorisation, release), so that callers can tell whether the factors
  // still belong to the permittivity they solved with
  int64_t state = 0;
  // the internal partition (tet_part == NULL) of the last decomposition
  std::vector<int32_t> own_part;
  // two-level preconditioner (mw_set_coarse_space): coarse space of the three
  // constant fields per subdomain, its structures for the current
  // decomposition, and the factors of E = Z^T A Z
  int coarse_kind = MW_COARSE_NONE;
  bool coarse_built = false, coarse_active = false;
  DevBuf c_tvec, c_row_sub, c_nb_ptr, c_nb, c_fac_off, c_loc_off, c_n_loc, c_n_pad, c_sub_dof, c_ipiv, c_ridx,
      c_info, c_amax, c_row_lo, c_fenv, c_fenvh, c_env, c_boff, c_blo, c_bw, Fc;
  std::vector<int32_t> ch_n_loc, ch_row_lo, ch_fenv;
  std::vector<int2> ch_env;
  DeviceCoarse cz;
  DeviceDecomp cdd;
  double t_assemble = 0, t_decompose = 0, t_factor = 0;
};

namespace {

mw_status guard(const std::function<void()>& f) {
  try {
    f();
    return MW_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host out of memory";
    return MW_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return MW_EINVAL;
  }
}

void check_prob(mw_problem* p) { MW_CHECK(p != nullptr && p->ctx != nullptr, MW_EINVAL, "problem is NULL"); }

}  // namespace

namespace mw {
mw_status guarded(const std::function<void()>& f) { return guard(f); }
hipStream_t problem_stream(mw_problem* p) {
  check_prob(p);
  return p->stream;
}
int problem_device(mw_problem* p) {
  check_prob(p);
  return p->ctx->device;
}
DevBuf problem_alloc(mw_problem* p, int64_t bytes) {
  check_prob(p);
  return dalloc(p->ctx, bytes);
}
void problem_spmm(mw_problem* p, const double2* X, double2* Y, int nc, int64_t ld, const double2* Bsub) {
  check_prob(p);
  launch_spmm(p->dm, p->val.as<double2>(), X, ld, Y, ld, nc, Bsub, ld, p->stream);
}
void problem_retain(mw_problem* p) {
  check_prob(p);
  p->live_users++;
}
void problem_release(mw_problem* p) {
  if (p) p->live_users--;
}
DevBuf problem_upload(mw_problem* p, const void* host, int64_t bytes) {
  DevBuf b = problem_alloc(p, bytes);
  if (bytes > 0) MW_HIP(hipMemcpyAsync(b.p, host, (size_t)bytes, hipMemcpyHostToDevice, p->stream));
  return b;
}
}  // namespace mw

namespace {

void psync(mw_problem* p) { MW_HIP(hipStreamSynchronize(p->stream)); }

// ------------------------------------------------------------------ ports
void setup_ports(mw_problem* p) {
  mw_ctx* c = p->ctx;
  const Topology& T = p->T;
  int np = (int)p->ports.size();
  std::vector<PortDev> pd(np);
  for (int k = 0; k < np; ++k) {
    const mw_port& q = p->ports[k];
    pd[k].beta = make_double2(q.beta.re, q.beta.im);
    pd[k].radius = q.radius;
    pd[k].theta = q.theta;
    pd[k].width = q.width;
    for (int a = 0; a < 3; ++a) pd[k].pol[a] = q.pol[a];
  }
  // faces of every port, ascending face id
  std::vector<int64_t> pf_ptr(np + 1, 0);
  for (int32_t f = 0; f < T.nbf; ++f)
    if (T.btag[f] >= 1) pf_ptr[T.btag[f]]++;
  for (int k = 0; k < np; ++k) pf_ptr[k + 1] += pf_ptr[k];
  std::vector<int32_t> pf(pf_ptr[np]);
  {
    std::vector<int64_t> fill(pf_ptr.begin(), pf_ptr.end() - 1);
    for (int32_t f = 0; f < T.nbf; ++f)
      if (T.btag[f] >= 1) pf[fill[T.btag[f] - 1]++] = f;
  }
  // distinct unknowns of each port with their (face, local edge) contributions
  std::vector<int64_t> port_ptr(np + 1, 0), ent_ptr(1, 0);
  std::vector<int32_t> ent_dof, ent_port, ent_fq;
  for (int k = 0; k < np; ++k) {
    std::vector<std::pair<int32_t, int32_t>> dq;  // (dof, face*3+q)
    for (int64_t j = pf_ptr[k]; j < pf_ptr[k + 1]; ++j) {
      int32_t f = pf[j];
      for (int q = 0; q < 3; ++q) {
        int32_t d = T.dof[T.bf2e[(size_t)f * 3 + q]];
        if (d >= 0) dq.push_back({d, f * 3 + q});
      }
    }
    std::stable_sort(dq.begin(), dq.end(), [](auto& a, auto& b) { return a.first < b.first; });
    for (size_t a = 0; a < dq.size();) {
      size_t b = a;
      while (b < dq.size() && dq[b].first == dq[a].first) { ent_fq.push_back(dq[b].second); ++b; }
      ent_dof.push_back(dq[a].first);
      ent_port.push_back(k);
      ent_ptr.push_back((int64_t)ent_fq.size());
      a = b;
    }
    port_ptr[k + 1] = (int64_t)ent_dof.size();
  }
  p->port_dev = dalloc(c, (int64_t)std::max<size_t>(1, pd.size()) * sizeof(PortDev));
  if (np) MW_HIP(hipMemcpyAsync(p->port_dev.p, pd.data(), pd.size() * sizeof(PortDev), hipMemcpyHostToDevice, p->stream));
  p->port_ptr = upload(c, p->stream, port_ptr);
  p->ent_dof = upload(c, p->stream, ent_dof);
  p->ent_port = upload(c, p->stream, ent_port);
  p->ent_ptr = upload(c, p->stream, ent_ptr);
  p->ent_fq = upload(c, p->stream, ent_fq);
  p->pf_ptr = upload(c, p->stream, pf_ptr);
  p->pf = upload(c, p->stream, pf);
  p->pval = dalloc(c, (int64_t)std::max<size_t>(1, ent_dof.size()) * 8);
  p->nu = dalloc(c, (int64_t)std::max(1, np) * 8);
  DevicePorts& P = p->dp;
  P.nports = np;
  P.nent = (int64_t)ent_dof.size();
  P.ports = p->port_dev.as<PortDev>();
  P.port_ptr = p->port_ptr.as<int64_t>();
  P.ent_dof = p->ent_dof.as<int32_t>();
  P.ent_port = p->ent_port.as<int32_t>();
  P.ent_ptr = p->ent_ptr.as<int64_t>();
  P.ent_fq = p->ent_fq.as<int32_t>();
  P.pf_ptr = p->pf_ptr.as<int64_t>();
  P.pf = p->pf.as<int32_t>();
  P.pval = p->pval.as<double>();
  P.nu = p->nu.as<double>();
  launch_port_setup(p->dm, P, p->stream);
}

// Rows of A sorted by the Z-order (Morton) code of their edge midpoints,
// 10 bits per axis over the mesh's bounding box: consecutive rows of this
// order couple nearby unknowns, so the wide SpMM's reads of x rows stay in L2.
std::vector<int32_t> zorder_rows(const Topology& T) {
  const int64_t n = T.n();
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int32_t v = 0; v < T.nv; ++v)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], T.xyz[3 * v + a]);
      hi[a] = std::max(hi[a], T.xyz[3 * v + a]);
    }
  std::vector<std::pair<uint32_t, int32_t>> key(n);
  for (int64_t d = 0; d < n; ++d) {
    const int64_t e = T.free_edge[d];
    const int64_t va = T.edges[2 * e], vb = T.edges[2 * e + 1];
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
      const double x = 0.5 * (T.xyz[3 * va + a] + T.xyz[3 * vb + a]);
      const double t = hi[a] > lo[a] ? (x - lo[a]) / (hi[a] - lo[a]) : 0.0;
      q[a] = (uint32_t)std::min(1023.0, std::max(0.0, t * 1023.0));
    }
    uint32_t code = 0;
    for (int b = 0; b < 10; ++b)
      for (int a = 0; a < 3; ++a) code |= ((q[a] >> b) & 1u) << (3 * b + a);
    key[d] = {code, (int32_t)d};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> order(n);
  for (int64_t d = 0; d < n; ++d) order[d] = key[d].second;
  return order;
}

// Sliced ELLPACK layout of A's pattern (slices of 64 rows; the rows in the
// given order, sorted by decreasing length within windows of 512 so that a
// slice's rows have alike lengths): lane row (-1 padding), slice offsets,
// column of every slot (-1 padding) and its CSR position (-1 padding).
struct SellLayout {
  std::vector<int32_t> row, col, idx;
  std::vector<int64_t> off;
};
SellLayout build_sell(const Topology& T, const std::vector<int32_t>& order) {
  const int64_t n = T.n();
  std::vector<int32_t> rows(order);
  auto len = [&](int32_t r) { return T.row_ptr[r + 1] - T.row_ptr[r]; };
  for (int64_t w0 = 0; w0 < n; w0 += 512)
    std::stable_sort(rows.begin() + w0, rows.begin() + std::min<int64_t>(n, w0 + 512),
                     [&](int32_t a, int32_t b) { return len(a) > len(b); });
  const int64_t nsl = (n + 63) / 64;
  SellLayout L;
  L.row.assign(nsl * 64, -1);
  L.off.assign(nsl + 1, 0);
  for (int64_t s = 0; s < nsl; ++s) {
    int64_t w = 0;
    for (int64_t l = 0; l < 64 && s * 64 + l < n; ++l) {
      L.row[s * 64 + l] = rows[s * 64 + l];
      w = std::max<int64_t>(w, len(rows[s * 64 + l]));
    }
    L.off[s + 1] = L.off[s] + 64 * w;
  }
  L.col.assign(L.off[nsl], -1);
  L.idx.assign(L.off[nsl], -1);
  for (int64_t s = 0; s < nsl; ++s)
    for (int64_t l = 0; l < 64; ++l) {
      const int32_t r = L.row[s * 64 + l];
      if (r < 0) continue;
      for (int64_t k = 0; k < len(r); ++k) {
        const int64_t pos = L.off[s] + 64 * k + l;
        L.col[pos] = T.col[T.row_ptr[r] + k];
        L.idx[pos] = (int32_t)(T.row_ptr[r] + k);
      }
    }
  return L;
}

void assemble_values(mw_problem* p) {
  if (p->eps_p1)
    launch_element_matrices_p1(p->dm, p->eps_v.as<double2>(), p->k0, p->E.as<double2>(), p->eps.as<double2>(),
                               p->stream);
  else
    launch_element_matrices(p->dm, p->eps.as<double2>(), p->k0, p->E.as<double2>(), p->stream);
  launch_gather_csr(p->dm, p->E.as<double2>(), p->val.as<double2>(), p->stream);
  if (p->dm.sl_val)
    launch_sell_values((int64_t)(p->sl_idx.bytes / 4), p->sl_idx.as<int32_t>(), p->val.as<double2>(),
                       p->sl_val.as<double2>(), p->stream);
}

uint64_t hash_part(const int32_t* part, int32_t nt, int32_t nsub, int32_t delta) {
  uint64_t h = 1469598103934665603ull ^ (uint64_t)nsub * 1099511628211ull ^ ((uint64_t)delta << 32);
  if (part == nullptr) return h ^ 0x9e3779b97f4a7c15ull;   // the internal partition of nsub parts
  for (int32_t t = 0; t < nt; ++t) h = (h ^ (uint64_t)(uint32_t)part[t]) * 1099511628211ull;
  return h;
}

void upload_decomp(mw_problem* p) {
  mw_ctx* c = p->ctx;
  const Decomposition& D = p->D;
  p->d_fac_off = upload(c, p->stream, D.fac_off);
  p->d_fac_off_band = upload(c, p->stream, D.fac_off_band);
  p->d_boff_dense = upload(c, p->stream, D.boff_dense);
  p->d_blo_dense = upload(c, p->stream, D.blo_dense);
  p->d_bw_dense = upload(c, p->stream, D.bw_dense);
  p->d_boff_band = upload(c, p->stream, D.boff_band);
  p->d_blo_band = upload(c, p->stream, D.blo_band);
  p->d_bw_band = upload(c, p->stream, D.bw_band);
  p->d_loc_off = upload(c, p->stream, D.loc_off);
  p->d_n_loc = upload(c, p->stream, D.n_loc);
  p->d_n_pad = upload(c, p->stream, D.n_pad);
  p->d_lt_off = upload(c, p->stream, D.lt_off);
  p->d_lt_tet = upload(c, p->stream, D.lt_tet);
  p->d_lt_loc = upload(c, p->stream, D.lt_loc);
  p->d_lf_off = upload(c, p->stream, D.lf_off);
  p->d_lf_vert = upload(c, p->stream, D.lf_vert);
  p->d_lf_owner = upload(c, p->stream, D.lf_owner);
  p->d_lf_kind = upload(c, p->stream, D.lf_kind);
  p->d_lf_loc = upload(c, p->stream, D.lf_loc);
  p->d_rtl_ptr = upload(c, p->stream, D.rtl_ptr);
  p->d_rtl = upload(c, p->stream, D.rtl);
  p->d_rfl_ptr = upload(c, p->stream, D.rfl_ptr);
  p->d_rfl = upload(c, p->stream, D.rfl);
  p->d_sub_dof = upload(c, p->stream, D.sub_dof);
  p->d_D = upload(c, p->stream, D.D);
  p->d_cp_ptr = upload(c, p->stream, D.cp_ptr);
  p->d_cp_row = upload(c, p->stream, D.cp_row);
  p->d_ipiv = dalloc(c, D.sum_pad() * 4);
  p->d_ridx = dalloc(c, D.sum_pad() * 4);
  p->d_info = dalloc(c, (int64_t)D.nsub * 4);
  p->d_amax = dalloc(c, (int64_t)D.nsub * 8);
  p->h_row_lo.resize(D.nsub);
  for (int32_t i = 0; i < D.nsub; ++i) p->h_row_lo[i] = (D.n_lead[i] / 64) * 64;
  p->d_row_lo = upload(c, p->stream, p->h_row_lo);
  {
    // subdomains by decreasing size (ties by index): the triangular solves
    // start the longest sweeps first
    std::vector<int32_t> order(D.nsub);
    for (int32_t i = 0; i < D.nsub; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return D.n_pad[a] > D.n_pad[b]; });
    p->d_order = upload(c, p->stream, order);
  }
  DeviceDecomp& d = p->dd;
  d.nsub = D.nsub;
  d.n_glob = p->T.n();
  d.max_pad = *std::max_element(D.n_pad.begin(), D.n_pad.end());
  d.sum_pad = D.sum_pad();
  d.fac_off = p->d_fac_off.as<int64_t>();
  d.boff = p->d_boff_dense.as<int64_t>();
  d.blo = p->d_blo_dense.as<int32_t>();
  d.bw = p->d_bw_dense.as<int32_t>();
  d.bstride = D.bstride;
  d.loc_off = p->d_loc_off.as<int64_t>();
  d.n_loc = p->d_n_loc.as<int32_t>();
  d.n_pad = p->d_n_pad.as<int32_t>();
  d.lt_off = p->d_lt_off.as<int64_t>();
  d.lt_tet = p->d_lt_tet.as<int32_t>();
  d.lt_loc = p->d_lt_loc.as<int32_t>();
  d.lf_off = p->d_lf_off.as<int64_t>();
  d.lf_vert = p->d_lf_vert.as<int32_t>();
  d.lf_owner = p->d_lf_owner.as<int32_t>();
  d.lf_kind = p->d_lf_kind.as<int32_t>();
  d.lf_loc = p->d_lf_loc.as<int32_t>();
  d.rtl_ptr = p->d_rtl_ptr.as<int64_t>();
  d.rtl = p->d_rtl.as<int32_t>();
  d.rfl_ptr = p->d_rfl_ptr.as<int64_t>();
  d.rfl = p->d_rfl.as<int32_t>();
  d.sub_dof = p->d_sub_dof.as<int32_t>();
  d.D = p->d_D.as<double>();
  d.cp_ptr = p->d_cp_ptr.as<int64_t>();
  d.cp_row = p->d_cp_row.as<int64_t>();
  d.ipiv = p->d_ipiv.as<int32_t>();
  d.ridx = p->d_ridx.as<int32_t>();
  d.info = p->d_info.as<int32_t>();
  d.amax = p->d_amax.as<double>();
  d.h_n_loc = p->D.n_loc.data();
  d.row_lo = p->d_row_lo.as<int32_t>();
  d.h_row_lo = p->h_row_lo.data();
  d.order = p->d_order.as<int32_t>();
  p->d_fenv = upload(c, p->stream, D.fenv);
  d.fenv = p->d_fenv.as<int32_t>();
  p->d_fenvh = upload(c, p->stream, D.fenv_hi);
  d.fenv_hi = p->d_fenvh.as<int32_t>();
  d.h_fenv = p->D.fenv.data();
  d.fenv_stride = D.fenv_stride;
  d.env_stride = d.max_pad / 32;
  MW_CHECK(d.fenv_stride == d.env_stride, MW_EINVAL, "envelope tables of unequal strides");
  p->h_env.assign((size_t)d.nsub * d.env_stride, make_int2(0, 0));
  p->d_env = dalloc(c, (int64_t)p->h_env.size() * 8);
  d.env = p->d_env.as<int2>();
  d.h_env = p->h_env.data();
}

// Z = M^-1 V (n x nc, leading dimension ld), local workspace W.Y
// V complex FP64, or complex FP32 (a basis vector of the mixed-precision
// GMRES, with FP32 factors only)
// (vsc, optional: column c of V taken times vsc[c], a GMRES candidate stored
// before its normalisation)
template <class VT, class ZT = double2>
void one_level(mw_problem* p, GmresWork& W, const VT* V, ZT* Z, int nc, int64_t ld, const double* vsc = nullptr) {
  mw_ctx* c = p->ctx;
  int64_t n = p->T.n();
  if (p->prec == MW_C64) {
    float2* Y = (float2*)W.Y.get(c, p->dd.sum_pad * nc * 8);
    launch_restrict<float2, VT>(p->dd, V, ld, nc, Y, nc, W.st, vsc);
    lu_solve_batched<float2>(p->dd, p->F.as<float2>(), Y, nc, nc, W.st);
    launch_prolong<float2, ZT>(p->dd, n, Y, nc, nc, Z, ld, W.st);
  } else if constexpr (std::is_same<VT, double2>::value && std::is_same<ZT, double2>::value) {
    double2* Y = (double2*)W.Y.get(c, p->dd.sum_pad * nc * 16);
    launch_restrict<double2>(p->dd, V, ld, nc, Y, nc, W.st, vsc);
    lu_solve_batched<double2>(p->dd, p->F.as<double2>(), Y, nc, nc, W.st);
    launch_prolong<double2>(p->dd, n, Y, nc, nc, Z, ld, W.st);
  } else {
    MW_CHECK(false, MW_EINVAL, "FP32 Krylov vectors need FP32 subdomain factors");
  }
}

// two-level: q = Z E^-1 Z^T v, then Z = M^-1 (v - A q) + q; v - A q is
// formed in Z itself (the one-level restriction reads all of it before the
// prolongation overwrites it)
template <class C>
void two_level(mw_problem* p, GmresWork& W, const double2* V, double2* Z, int nc, int64_t ld) {
  mw_ctx* c = p->ctx;
  const int64_t n = p->T.n();
  const int ncp = p->cdd.max_pad;
  C* Yc = (C*)W.cy.get(c, (int64_t)ncp * nc * (int64_t)sizeof(C));
  double2* q = (double2*)W.cq.get(c, n * ld * 16);
  launch_coarse_restrict<C>(p->dd, p->cz, V, ld, nc, Yc, nc, ncp, W.st);
  lu_solve_batched<C>(p->cdd, p->Fc.as<C>(), Yc, nc, nc, W.st);
  launch_coarse_prolong<C>(p->dd, p->cz, n, Yc, nc, nc, q, ld, W.st);
  launch_spmm(p->dm, p->val.as<double2>(), q, ld, Z, ld, nc, V, ld, W.st);
  one_level<double2>(p, W, Z, Z, nc, ld);
  launch_axpy_cols(Z, q, n, ld, nc, W.st);
}

// Factorisation the next mw_factor_subdomains uses: L D L^T without
// interchanges when requested, or (automatic) when every tetrahedron is lossy
bool choose_sym(mw_problem* p) {
  if (p->factor_kind != MW_FACTOR_AUTO) return p->factor_kind == MW_FACTOR_LDLT;
  double* dmax = (double*)p->w_small.get(p->ctx, 8);
  double hmax = 0.0;
  launch_max_imag(p->eps.as<double2>(), p->T.nt, dmax, p->stream);
  MW_HIP(hipMemcpyAsync(&hmax, dmax, 8, hipMemcpyDeviceToHost, p->stream));
  MW_HIP(hipStreamSynchronize(p->stream));
  return hmax < 0.0;
}

// factor storage: banded for the factorisation without interchanges, dense
// for LU with interchanges; elements of the whole batch
int64_t factor_elems(const Decomposition& D, bool banded) {
  // (one dense 64-row block of slack after the banded storage: no kernel
  // reads outside its rows' stored columns, and none could leave the buffer)
  int32_t mp = 0;
  for (int32_t np : D.n_pad) mp = std::max(mp, np);
  return banded ? D.fac_off_band.back() + (int64_t)64 * mp : D.fac_off.back();
}
void set_layout(mw_problem* p, bool banded) {
  DeviceDecomp& d = p->dd;
  p->banded = banded;
  d.fac_off = (banded ? p->d_fac_off_band : p->d_fac_off).as<int64_t>();
  d.boff = (banded ? p->d_boff_band : p->d_boff_dense).as<int64_t>();
  d.blo = (banded ? p->d_blo_band : p->d_blo_dense).as<int32_t>();
  d.bw = (banded ? p->d_bw_band : p->d_bw_dense).as<int32_t>();
}

// Z = M^-1 V (one- or two-level) for nc columns of leading dimension ld
void apply_prec(mw_problem* p, GmresWork& W, const double2* V, double2* Z, int nc, int64_t ld) {
  MW_CHECK(p->factors_valid, MW_EINVAL, "no valid subdomain factors: call mw_factor_subdomains");
  if (!p->coarse_active) {
    one_level<double2>(p, W, V, Z, nc, ld);
  } else if (p->prec == MW_C64) {
    two_level<float2>(p, W, V, Z, nc, ld);
  } else {
    two_level<double2>(p, W, V, Z, nc, ld);
  }
}
// the same for an FP32 basis vector: the one-level restriction reads it
// directly; the two-level correction works on an FP64 copy
void apply_prec(mw_problem* p, GmresWork& W, const float2* V, double2* Z, int nc, int64_t ld) {
  MW_CHECK(p->factors_valid, MW_EINVAL, "no valid subdomain factors: call mw_factor_subdomains");
  if (!p->coarse_active) {
    one_level<float2>(p, W, V, Z, nc, ld);
    return;
  }
  double2* Vd = (double2*)W.cw.get(p->ctx, p->T.n() * ld * 16);
  launch_widen(V, Vd, p->T.n() * ld, W.st);
  apply_prec(p, W, (const double2*)Vd, Z, nc, ld);
}

// Structures of the coarse space for the current decomposition: edge vector
// of every unknown, subdomain of every local row, and per subdomain i the
// ascending list of subdomains j with E[(i,.),(j,.)] structurally nonzero (a
// row of i with D_i > 0 coupled by A to a row of j with D_j > 0)
void build_coarse(mw_problem* p) {
  mw_ctx* c = p->ctx;
  const Topology& T = p->T;
  const Decomposition& D = p->D;
  const int32_t nsub = D.nsub;
  const int64_t n = T.n();
  const int nc = 3 * nsub, ncp = (int)round_up(nc, 64);
  MW_CHECK(ncp <= 8192, MW_EINVAL,
           "coarse space of " + std::to_string(nc) + " unknowns exceeds the dense coarse factor's 8192 (n_sub <= 2730)");
  std::vector<double> tvec(3 * n);
  for (int64_t g = 0; g < n; ++g) {
    const int64_t e = T.free_edge[g];
    const int64_t va = T.edges[2 * e], vb = T.edges[2 * e + 1];
    for (int a = 0; a < 3; ++a) tvec[3 * g + a] = T.xyz[3 * vb + a] - T.xyz[3 * va + a];
  }
  std::vector<int32_t> row_sub(D.sum_pad());
  for (int32_t i = 0; i < nsub; ++i)
    for (int64_t r = D.loc_off[i]; r < D.loc_off[i + 1]; ++r) row_sub[r] = i;
  std::vector<std::vector<int32_t>> nbl(nsub);
  parallel_for(nsub, [&](int64_t i) {
    std::vector<int32_t> js;
    for (int64_t r = D.loc_off[i]; r < D.loc_off[i] + D.n_pad[i]; ++r) {
      const int32_t g = D.sub_dof[r];
      if (g < 0 || D.D[r] == 0.0) continue;
      for (int64_t k = T.row_ptr[g]; k < T.row_ptr[g + 1]; ++k) {
        const int32_t h = T.col[k];
        for (int64_t q = D.cp_ptr[h]; q < D.cp_ptr[h + 1]; ++q) js.push_back(row_sub[D.cp_row[q]]);
      }
      if (js.size() > (1u << 16)) {
        std::sort(js.begin(), js.end());
        js.erase(std::unique(js.begin(), js.end()), js.end());
      }
    }
    std::sort(js.begin(), js.end());
    js.erase(std::unique(js.begin(), js.end()), js.end());
    nbl[i] = std::move(js);
  });
  std::vector<int64_t> nb_ptr(nsub + 1, 0);
  int max_nb = 0;
  for (int32_t i = 0; i < nsub; ++i) {
    nb_ptr[i + 1] = nb_ptr[i] + (int64_t)nbl[i].size();
    max_nb = std::max(max_nb, (int)nbl[i].size());
  }
  MW_CHECK(max_nb <= kCoarseMaxNb, MW_EINVAL,
           "a subdomain couples to " + std::to_string(max_nb) + " others in the coarse matrix (at most " +
               std::to_string(kCoarseMaxNb) + ")");
  std::vector<int32_t> nb(nb_ptr[nsub]);
  for (int32_t i = 0; i < nsub; ++i) std::copy(nbl[i].begin(), nbl[i].end(), nb.begin() + nb_ptr[i]);
  hipStream_t st = p->stream;
  p->c_tvec = upload(c, st, tvec);
  p->c_row_sub = upload(c, st, row_sub);
  p->c_nb_ptr = upload(c, st, nb_ptr);
  p->c_nb = upload(c, st, nb);
  DeviceCoarse& z = p->cz;
  z.nsub = nsub;
  z.max_nb = max_nb;
  z.tvec = p->c_tvec.as<double>();
  z.row_sub = p->c_row_sub.as<int32_t>();
  z.nb_ptr = p->c_nb_ptr.as<int64_t>();
  z.nb = p->c_nb.as<int32_t>();
  // the coarse matrix as a single dense "subdomain" of the batched
  // factorisation: no structural envelope assumed (every column may be
  // nonzero), all rows needed by the backward solve
  std::vector<int64_t> fac_off{0, (int64_t)ncp * ncp}, loc_off{0, ncp};
  p->ch_n_loc = {nc};
  std::vector<int32_t> n_pad{ncp}, sub_dof(ncp, -1);
  for (int k = 0; k < nc; ++k) sub_dof[k] = k;
  p->ch_row_lo = {0};
  const int stride = ncp / 32;
  p->ch_fenv.assign(stride, 0);
  std::vector<int32_t> fenv_hi(stride, ncp);
  p->ch_env.assign(stride, make_int2(0, 0));
  p->c_fac_off = upload(c, st, fac_off);
  p->c_loc_off = upload(c, st, loc_off);
  p->c_n_loc = upload(c, st, p->ch_n_loc);
  p->c_n_pad = upload(c, st, n_pad);
  p->c_sub_dof = upload(c, st, sub_dof);
  p->c_ipiv = dalloc(c, (int64_t)ncp * 4);
  p->c_ridx = dalloc(c, (int64_t)ncp * 4);
  p->c_info = dalloc(c, 8);
  p->c_amax = dalloc(c, 8);
  p->c_row_lo = upload(c, st, p->ch_row_lo);
  p->c_fenv = upload(c, st, p->ch_fenv);
  p->c_fenvh = upload(c, st, fenv_hi);
  p->c_env = dalloc(c, (int64_t)stride * 8);
  DeviceDecomp& d = p->cdd;
  d = DeviceDecomp{};
  d.nsub = 1;
  d.max_pad = ncp;
  d.sum_pad = ncp;
  d.fac_off = p->c_fac_off.as<int64_t>();
  d.loc_off = p->c_loc_off.as<int64_t>();
  d.n_loc = p->c_n_loc.as<int32_t>();
  d.n_pad = p->c_n_pad.as<int32_t>();
  d.sub_dof = p->c_sub_dof.as<int32_t>();
  d.ipiv = p->c_ipiv.as<int32_t>();
  d.ridx = p->c_ridx.as<int32_t>();
  d.info = p->c_info.as<int32_t>();
  d.amax = p->c_amax.as<double>();
  d.h_n_loc = p->ch_n_loc.data();
  d.row_lo = p->c_row_lo.as<int32_t>();
  d.h_row_lo = p->ch_row_lo.data();
  d.fenv = p->c_fenv.as<int32_t>();
  d.h_fenv = p->ch_fenv.data();
  d.fenv_hi = p->c_fenvh.as<int32_t>();
  d.fenv_stride = stride;
  d.env = p->c_env.as<int2>();
  d.h_env = p->ch_env.data();
  d.env_stride = stride;
  // dense storage of the coarse matrix
  std::vector<int64_t> boff(ncp / 64);
  std::vector<int32_t> blo(ncp / 64, 0), bw(ncp / 64, ncp);
  for (int b = 0; b < ncp / 64; ++b) boff[b] = (int64_t)64 * b * ncp;
  p->c_boff = upload(c, st, boff);
  p->c_blo = upload(c, st, blo);
  p->c_bw = upload(c, st, bw);
  d.boff = p->c_boff.as<int64_t>();
  d.blo = p->c_blo.as<int32_t>();
  d.bw = p->c_bw.as<int32_t>();
  d.bstride = ncp / 64;
  p->coarse_built = true;
}

// E = Z^T A Z assembled and factored (the subdomain factorisation's kind)
template <class C>
void factor_coarse(mw_problem* p, bool sym) {
  hipStream_t st = p->stream;
  const int ncp = p->cdd.max_pad;
  launch_coarse_matrix<C>(p->dm, p->val.as<double2>(), p->dd, p->cz, p->Fc.as<C>(), ncp, st);
  launch_zero_bytes(p->cdd.info, 4, st);
  lu_factor_batched<C>(p->cdd, p->Fc.as<C>(), st, sym);
}

// column 2-norms squared of an n x nc block (device out), deterministic
void colnorm2(mw_problem* p, GmresWork& W, const double2* V, int64_t ld, int nc, double* out) {
  int64_t n = p->T.n();
  int64_t nch = reduce_chunks(n);
  double* part = (double*)W.npart.get(p->ctx, nch * nc * 8);
  launch_colnorm2_partial(V, n, ld, nc, part, W.st);
  launch_sum_chunks(part, nch, nc, out, W.st);
}

// whether GMRES keeps its Krylov basis in complex FP32: with FP32 factors,
// unless an FP64 basis was asked for
bool basis_fp32(mw_problem* p) {
  return p->prec == MW_C64 && (p->basis == MW_BASIS_AUTO || p->basis == MW_BASIS_FP32_LEAN);
}

// device bytes one more right-hand side column costs a GMRES(m) driver:
// basis (m+1), X, B, Z, update, local vectors, reduction partials
int64_t gmres_bytes_per_col(mw_problem* p, int m, bool block) {
  int64_t esz = p->prec == MW_C64 ? 8 : 16;
  const int64_t bsz = (!block && basis_fp32(p)) ? 8 : 16;   // block GMRES keeps an FP64 basis
  int64_t big = (int64_t)(m + 1) * p->T.n() * bsz + 4 * p->T.n() * 16 + p->dd.sum_pad * esz +
                reduce_chunks(p->T.n()) * (2 * m + 3) * 16;
  // FP32 basis: the m preconditioned candidates in FP32 (one, rewritten at
  // every step, when lean), and for the two-level preconditioner an FP64
  // copy of v_j
  if (bsz == 8) {
    big += (p->basis == MW_BASIS_FP32_LEAN ? 1 : (int64_t)m) * 8 * p->T.n();
    if (p->coarse_kind != MW_COARSE_NONE) big += p->T.n() * 16;
  }
  if (p->coarse_kind != MW_COARSE_NONE)   // two-level: Q v and the coarse vector
    big += p->T.n() * 16 + (int64_t)round_up(3 * (int64_t)std::max(p->D.nsub, 1), 64) * esz;
  // Hessenberg (raw and rotated), rotations, g, y, dot sums, provisional
  // column, coefficients, norms, flags
  int64_t small = 2 * (int64_t)(m + 1) * m * 16 + (int64_t)m * 24 + 5 * (int64_t)(m + 1) * 16 + 2 * (int64_t)m * 16 +
                  7 * 8 + 2 * 4 + (int64_t)m * m * 16;
  return big + small + 256;
}

// Z = B - A X (n x nc, ld nc); squared column norms into rn2 (device) and hr2 (host)
void true_residual(mw_problem* p, GmresWork& W, const double2* B, const double2* X, double2* Z, int nc, double* rn2,
                   std::vector<double>& hr2) {
  launch_spmm(p->dm, p->val.as<double2>(), X, nc, Z, nc, nc, B, nc, W.st);
  colnorm2(p, W, Z, nc, nc, rn2);
  hr2.resize(nc);
  MW_HIP(hipMemcpyAsync(hr2.data(), rn2, nc * 8, hipMemcpyDeviceToHost, W.st));
  MW_HIP(hipStreamSynchronize(W.st));
}

// One restart cycle of GMRES(m) right-preconditioned with ORAS (Section 6),
// pseudo-block over the nc columns of X (ld nc).  On entry Z holds the true
// residual r = b - A x and vec = [||b|| | ||r||^2 | scratch x2] (device, nc
// each), rnorm = ||r|| on the host.  Columns with hact[k] = 0 are carried
// along untouched.  The Arnoldi basis is orthogonalised by classical
// Gram-Schmidt applied twice, with the second pass of each new vector
// delayed to the next step so that one sweep of dot products and one sweep of
// updates over the basis serve both passes (k_dgs_step, k_dgs_update): step
// j applies the operator to the once-orthogonalised candidate, finishes its
// second pass and column j-1 of the Hessenberg matrix, then projects the
// operator image.  A column stops when its Givens residual estimate reaches
// tol (relative to ||b||) or its iteration count reaches maxit; the cycle
// ends when every column has stopped or after m steps, then x += M^-1 V y.
// iters[k] counts the Arnoldi steps of column k.
template <class BT>
void gmres_cycle(mw_problem* p, GmresWork& W, double2* X, double2* Z, int nc, const mw_solve_opts& o, double* vec,
                 const std::vector<double>& rnorm, std::vector<int32_t>& hact, std::vector<int32_t>& iters) {
  mw_ctx* c = p->ctx;
  hipStream_t st = W.st;
  const int64_t n = p->T.n();
  const int m = o.restart;
  const int64_t ld = nc;
  const int64_t vstride = n * ld;
  BT* V = (BT*)W.V.get(c, (int64_t)(m + 1) * vstride * (int64_t)sizeof(BT));
  double2* T = (double2*)W.tmp.get(c, vstride * 16);
  double2* H = (double2*)W.H.get(c, (int64_t)(m + 1) * m * nc * 16);
  double2* Hraw = (double2*)W.Hr.get(c, (int64_t)(m + 1) * m * nc * 16);
  double* cs = (double*)W.cs.get(c, (int64_t)m * nc * 8);
  double2* sn = (double2*)W.sn.get(c, (int64_t)m * nc * 16);
  double2* g = (double2*)W.g.get(c, (int64_t)(m + 1) * nc * 16);
  double2* y = (double2*)W.y.get(c, (int64_t)(m + 1) * nc * 16);
  double2* P1 = (double2*)W.h1.get(c, (int64_t)(m + 1) * nc * 16);
  double2* P2 = (double2*)W.h2.get(c, (int64_t)(m + 1) * nc * 16);
  double2* hprov = (double2*)W.hp.get(c, (int64_t)(m + 1) * nc * 16);
  double2* coef = (double2*)W.cf.get(c, (int64_t)2 * m * nc * 16 + 16);
  double* nu = (double*)W.nu.get(c, (int64_t)nc * 8);
  double2* ee = (double2*)W.ee.get(c, (int64_t)nc * 16);
  const int64_t nch = reduce_chunks(n);
  double2* part1 = (double2*)W.part.get(c, nch * 2 * (m + 1) * nc * 16);
  double2* part2 = part1 + nch * (m + 1) * nc;
  double* npart = (double*)W.npart.get(c, nch * nc * 8);
  double* bnorm = vec;        // ||b||
  double* rn2 = vec + nc;     // ||r||^2
  double* hn2 = vec + 2 * nc; // ||u||^2 of the current candidate
  double* resid = vec + 3 * nc;
  int32_t* ivec = (int32_t*)W.ints.get(c, (int64_t)3 * nc * 4);
  int32_t* act = ivec;
  int32_t* kdim = ivec + nc;
  int32_t* done = ivec + 2 * nc;
  // FP32 basis: the operator's inputs are kept (M^-1 of each candidate,
  // FP32, as the SpMM reads it) with the triangular factor Rc relating the
  // candidates to the basis, so that the cycle ends with x += Zc Rc^-1 y
  // instead of one more preconditioner application
  const bool fp32_basis = std::is_same<BT, float2>::value;
  const bool keep_z = fp32_basis && p->basis != MW_BASIS_FP32_LEAN;
  // (lean, one level: one FP32 slot for M^-1 v_j, rewritten every step)
  const bool one_slot = fp32_basis && !keep_z && !p->coarse_active;
  // FP32 basis, one level: the next candidate stays unnormalised in its
  // slot; the three kernels that read it before the next update replaces
  // it (restriction, dot products, update) take it times 1 / ||u||, from
  // the update's partial sums (hn2), instead of a pass that rewrites it
  const bool defer_norm = fp32_basis && !p->coarse_active;
  double* csc_buf = defer_norm ? (double*)W.csc.get(c, (int64_t)nc * 8) : nullptr;
  const double* vj_scale = nullptr;   // 1 / ||u|| per column (csc_buf) from step 1 on: slot j unnormalised
  float2* Zc = keep_z     ? (float2*)W.zc.get(c, (int64_t)m * vstride * 8)
               : one_slot ? (float2*)W.zc.get(c, vstride * 8)
                          : nullptr;
  double2* Rc = keep_z ? (double2*)W.rc.get(c, (int64_t)m * m * nc * 16) : nullptr;
  std::vector<double2> g0((size_t)nc);
  int nact = 0;
  for (int k = 0; k < nc; ++k) {
    g0[k] = make_double2(rnorm[k], 0.0);
    nact += hact[k];
  }
  if (nact == 0) return;
  MW_HIP(hipMemcpyAsync(act, hact.data(), nc * 4, hipMemcpyHostToDevice, st));
  launch_zero_bytes(kdim, nc * 4, st);
  launch_zero(g, (int64_t)(m + 1) * nc, st);
  launch_zero(Hraw, (int64_t)(m + 1) * m * nc, st);
  MW_HIP(hipMemcpyAsync(g, g0.data(), nc * 16, hipMemcpyHostToDevice, st));
  launch_start_cycle(Z, V, n, ld, nc, rn2, act, st);
  std::vector<int32_t> hact_prev(nc), hdone(nc);
  // The step after the one whose trial estimates say every active column is
  // done only finishes the last column (no operator application); if a
  // column then turns out to need more, the step is repeated with the
  // operator, the column already finished.
  bool finish_only = false;
  for (int j = 0; j <= m; ++j) {
    BT* Vj = V + (int64_t)j * vstride;
    bool more = j < m && !finish_only;   // step m only finishes column m-1
    for (int pass = 0; pass < 2; ++pass) {
      if (more) {
        if (keep_z || one_slot) {
          // FP32 basis: M^-1 v_j is rounded to FP32 as well (the product
          // A M^-1 v_j is FP64 either way; the rounding perturbs the Arnoldi
          // relation no more than the basis' own)
          float2* Zf = keep_z ? Zc + (int64_t)j * vstride : Zc;
          MW_CHECK(p->factors_valid, MW_EINVAL, "no valid subdomain factors: call mw_factor_subdomains");
          if (!p->coarse_active) {
            one_level<BT, float2>(p, W, Vj, Zf, nc, ld, vj_scale);
          } else {
            apply_prec(p, W, Vj, Z, nc, ld);
            launch_narrow(Z, Zf, vstride, st);
          }
          launch_spmm(p->dm, p->val.as<double2>(), (const float2*)Zf, ld, T, ld, nc, nullptr, 0, st);
        } else {
          apply_prec(p, W, Vj, Z, nc, ld);
          launch_spmm(p->dm, p->val.as<double2>(), (const double2*)Z, ld, T, ld, nc, nullptr, 0, st);
        }
      }
      launch_dots_partial(V, vstride, j + 1, Vj, more ? T : nullptr, n, ld, nc, act, part1, part2, st, vj_scale);
      launch_sum_chunks_c(part1, nch, (int64_t)(j + 1) * nc, P1, st);
      if (more) launch_sum_chunks_c(part2, nch, (int64_t)(j + 1) * nc, P2, st);
      launch_dgs_step(j, m, pass == 0, nc, P1, more ? P2 : nullptr, hn2, Hraw, H, cs, sn, g, hprov, coef, nu, ee,
                      kdim, act, resid, bnorm, o.tol, Rc, st);
      if (j > 0 && pass == 0) {
        // column j-1 is final: one Arnoldi step for every column active before
        hact_prev = hact;
        MW_HIP(hipMemcpyAsync(hact.data(), act, nc * 4, hipMemcpyDeviceToHost, st));
        MW_HIP(hipStreamSynchronize(st));
        bool changed = false;
        nact = 0;
        for (int k = 0; k < nc; ++k) {
          if (hact_prev[k]) iters[k]++;
          if (hact[k] && iters[k] >= o.maxit) { hact[k] = 0; changed = true; }
          nact += hact[k];
        }
        if (changed) MW_HIP(hipMemcpyAsync(act, hact.data(), nc * 4, hipMemcpyHostToDevice, st));
      }
      if (more || nact == 0 || j == m) break;
      more = true;   // a column continues although its trial estimate said done
    }
    if (nact == 0 || j == m) break;
    launch_dgs_update(V, vstride, j, coef, nu, ee, T, n, ld, nc, act, npart, st, vj_scale);
    launch_sum_chunks(npart, nch, nc, hn2, st);
    if (defer_norm) {
      launch_inv_norms(nc, hn2, csc_buf, st);
      vj_scale = csc_buf;
    } else {
      launch_scale_cols(V + (int64_t)(j + 1) * vstride, n, ld, nc, hn2, act, st);
    }
    finish_only = false;
    if (j + 1 < m) {
      launch_dgs_trial(j, m, nc, hprov, hn2, cs, sn, g, act, bnorm, o.tol, done, st);
      MW_HIP(hipMemcpyAsync(hdone.data(), done, nc * 4, hipMemcpyDeviceToHost, st));
      MW_HIP(hipStreamSynchronize(st));
      finish_only = true;
      for (int k = 0; k < nc; ++k)
        if (hact[k] && !hdone[k] && iters[k] + 1 < o.maxit) finish_only = false;
    }
  }
  // x += M^-1 (V y)
  launch_backsolve(m, nc, H, g, kdim, y, st);
  double2* U = T;
  if (keep_z) {
    // V y = Y Rc^-1 y (Y the candidates), so M^-1 V y = Zc Rc^-1 y
    launch_candsolve(m, nc, Rc, kdim, y, st);
    launch_combine(Zc, vstride, m, y, kdim, U, n, ld, nc, st);
  } else {
    launch_combine(V, vstride, m, y, kdim, Z, n, ld, nc, st);
    apply_prec(p, W, Z, U, nc, ld);
  }
  launch_axpy_cols(X, U, n, ld, nc, st);
}

// whether column k needs another cycle, from its true residual
inline bool column_continues(double bnorm, double relres, int32_t iters, double r, const mw_solve_opts& o) {
  return bnorm > 0 && relres > o.tol && iters < o.maxit && std::isfinite(r);
}

struct ChunkResult {
  int max_iters = 0, cycles = 0;
  bool numeric = false;
};

// Pseudo-block GMRES(m) to convergence on nc columns (one memory chunk of
// mw_solve), true residual recomputed at every restart.
ChunkResult gmres_chunk(mw_problem* p, GmresWork& W, const double2* Bsrc, int64_t ldb_src, double2* Xdst,
                        int64_t ldx_dst, int nc, const mw_solve_opts& o, int32_t* iters_out, double* relres_out) {
  mw_ctx* c = p->ctx;
  hipStream_t st = W.st;
  const int64_t n = p->T.n();
  const int64_t ld = nc;
  const int64_t vstride = n * ld;
  double2* X = (double2*)W.X.get(c, vstride * 16);
  double2* B = (double2*)W.B.get(c, vstride * 16);
  double2* Z = (double2*)W.Z.get(c, vstride * 16);
  double* vec = (double*)W.vec.get(c, (int64_t)4 * nc * 8);
  double* bnorm = vec;
  double* rn2 = vec + nc;

  launch_copy_cols(Bsrc, ldb_src, B, ld, n, nc, st);
  if (o.use_x0) launch_copy_cols(Xdst, ldx_dst, X, ld, n, nc, st);
  else launch_zero(X, vstride, st);
  std::vector<double> hb(nc), hr, hb2(nc);
  colnorm2(p, W, B, ld, nc, rn2);
  MW_HIP(hipMemcpyAsync(hb2.data(), rn2, nc * 8, hipMemcpyDeviceToHost, st));
  MW_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < nc; ++k) hb[k] = std::sqrt(hb2[k]);
  MW_HIP(hipMemcpyAsync(bnorm, hb.data(), nc * 8, hipMemcpyHostToDevice, st));

  ChunkResult res;
  std::vector<int32_t> iters(nc, 0), hact(nc, 0);
  std::vector<double> relres(nc, 0.0), rnorm(nc);
  for (;;) {
    // true residual r = b - A x (iterative refinement point)
    true_residual(p, W, B, X, Z, nc, rn2, hr);
    int nact = 0;
    for (int k = 0; k < nc; ++k) {
      double r = std::sqrt(hr[k]);
      if (!std::isfinite(r)) res.numeric = true;
      relres[k] = hb[k] > 0 ? r / hb[k] : 0.0;
      hact[k] = column_continues(hb[k], relres[k], iters[k], r, o) ? 1 : 0;
      nact += hact[k];
      rnorm[k] = r;
    }
    if (res.numeric || nact == 0) break;
    res.cycles++;
    if (basis_fp32(p)) gmres_cycle<float2>(p, W, X, Z, nc, o, vec, rnorm, hact, iters);
    else gmres_cycle<double2>(p, W, X, Z, nc, o, vec, rnorm, hact, iters);
  }
  launch_copy_cols(X, ld, Xdst, ldx_dst, n, nc, st);
  MW_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < nc; ++k) {
    if (iters_out) iters_out[k] = iters[k];
    if (relres_out) relres_out[k] = relres[k];
    res.max_iters = std::max(res.max_iters, iters[k]);
  }
  return res;
}

// ---------------------------------------------------------------- block GMRES
// Breakdown threshold of the block Cholesky QR: a pivot of the new block's
// factor below this fraction of the largest column norm of A M^-1 V_j (or of
// the starting residual block) counts as rank deficiency.  A Cholesky-based
// QR in FP64 resolves relative pivots down to about the square root of the
// unit roundoff, so the threshold sits above it.
constexpr double BLOCK_DELTA = 1e-7;
// Above this ||R||_F ||R^-1||_F the Cholesky QR of a block is repeated on its
// result (CholQR2), which restores orthogonality to the unit roundoff.
constexpr double BLOCK_COND2 = 2e3;

// device bytes of the block Gram-Schmidt reduction partials for nb blocks
int64_t block_part_bytes(int64_t n, int nb, int m) {
  int64_t best = 0;
  for (int ktot = 1; ktot <= m + 1; ++ktot) {
    int64_t rows, nch;
    bdots_chunks(n, nb, ktot, &rows, &nch);
    best = std::max<int64_t>(best, nch * nb * ktot);
  }
  return best * 1024 * 16;
}

double frob(const zc* A, int q) {
  double s = 0.0;
  for (int e = 0; e < q * q; ++e) s += std::norm(A[e]);
  return std::sqrt(s);
}

// C = A B (q x q, row-major)
void matmul(const zc* A, const zc* B, int q, zc* C) {
  for (int i = 0; i < q; ++i)
    for (int l = 0; l < q; ++l) {
      zc s = 0.0;
      for (int k = 0; k < q; ++k) s += A[i * q + k] * B[k * q + l];
      C[i * q + l] = s;
    }
}

// One cycle of block GMRES(m) right-preconditioned with ORAS on nca columns
// (leading dimension nca) grouped in blocks of BW: block b is columns
// [BW b, min(BW (b+1), nca)).  On entry V_0 (the start of W.V) holds the true
// residuals.  Per block: the starting block is factored by Cholesky QR
// (R0 = V_0 S0); step j applies the operator to V_j, projects the image on
// V_0..V_j twice (block classical Gram-Schmidt, k_bdots / k_bupdate: dots,
// update, dots with the Gram matrix of the projected image, then the second
// update fused with the scaling by R^-1), where R, the Cholesky factor of
// the projected image's Gram matrix, comes from G1 - P2^H P2 (Pythagoras);
// an ill-conditioned R gets a second Cholesky QR pass.  The host appends the
// block column to the least-squares problem and stops the block when every
// one of its columns' estimates reaches atol, after maxsteps[b] steps, or at
// a rank-deficient R (that step still counts: only R^H R enters the least
// squares).  Then U = M^-1 V Y.  steps[b] = steps of block b; 0 for a block
// whose starting residuals are rank deficient (U = 0 there).
void block_cycle(mw_problem* p, GmresWork& W, int nca, int m, const std::vector<double>& atol,
                 const std::vector<int>& maxsteps, double2* U, std::vector<int>& steps) {
  mw_ctx* c = p->ctx;
  hipStream_t st = W.st;
  const int64_t n = p->T.n();
  const int64_t ld = nca;
  const int64_t vstride = n * ld;
  const int nb = (int)ceil_div(nca, BW);
  double2* V = (double2*)W.V.get(c, (int64_t)(m + 1) * vstride * 16);
  double2* T = (double2*)W.tmp.get(c, vstride * 16);
  double2* part = (double2*)W.part.get(c, block_part_bytes(n, nb, m));
  double2* dP1 = (double2*)W.h1.get(c, (int64_t)nb * (m + 1) * 1024 * 16);
  double2* dP2 = (double2*)W.h2.get(c, (int64_t)nb * (m + 2) * 1024 * 16);
  double2* dR = (double2*)W.cf.get(c, (int64_t)nb * 1024 * 16);
  double2* dY = (double2*)W.y.get(c, (int64_t)nb * m * 1024 * 16);
  int32_t* dflag = (int32_t*)W.ints.get(c, (int64_t)3 * nb * 4);
  int32_t* d_dots = dflag;          // 1: block active (dots, first update)
  int32_t* d_upd = dflag + nb;      // 0: skip, 1: compute, 2: write zeros
  int32_t* d_kv = dflag + 2 * nb;   // steps per block (final combination)
  std::vector<int> width(nb);
  for (int b = 0; b < nb; ++b) width[b] = std::min(BW, nca - BW * b);
  steps.assign(nb, 0);
  std::vector<BlockLS> ls(nb);
  std::vector<char> active(nb, 0);
  std::vector<int32_t> f_dots(nb), f_upd(nb), f_kv(nb);
  std::vector<zc> hP1, hP2, hG((size_t)nb * 1024), hR((size_t)nb * 1024);
  std::vector<zc> R1((size_t)nb * 1024), R2((size_t)nb * 1024);
  int64_t nch = 0;
  auto upload_flags = [&](const std::vector<int32_t>& f, int32_t* d) {
    MW_HIP(hipMemcpyAsync(d, f.data(), nb * 4, hipMemcpyHostToDevice, st));
  };
  auto set_identity = [&](zc* A) {
    for (int e = 0; e < 1024; ++e) A[e] = (e % 33 == 0) ? 1.0 : 0.0;
  };
  // Gram matrices (host, nb x 32 x 32) of the blocks of X flagged in f_dots
  auto gram = [&](const double2* X) {
    upload_flags(f_dots, d_dots);
    launch_bdots(V, vstride, 0, X, X, n, ld, nca, nb, d_dots, part, &nch, st);
    launch_sum_chunks_c(part, nch, (int64_t)nb * 1024, dP2, st);
    MW_HIP(hipMemcpyAsync(hG.data(), dP2, (size_t)nb * 1024 * 16, hipMemcpyDeviceToHost, st));
    MW_HIP(hipStreamSynchronize(st));
  };
  // X[:, block b] <- X[:, block b] hR_b for the blocks flagged in f_upd (in place)
  auto scale = [&](double2* X) {
    upload_flags(f_upd, d_upd);
    MW_HIP(hipMemcpyAsync(dR, hR.data(), (size_t)nb * 1024 * 16, hipMemcpyHostToDevice, st));
    launch_bupdate(V, vstride, 0, nullptr, 0, dR, 0, dR, X, X, n, ld, nca, nb, d_upd, st);
  };
  // Cholesky of the Gram matrix of block b (padding columns: identity);
  // returns the number of deficient pivots relative to scale2
  auto chol = [&](const zc* Gb, int b, double scale2, zc* R) {
    std::vector<zc> G(Gb, Gb + 1024);
    for (int q = 0; q < BW; ++q)
      for (int l = 0; l < BW; ++l)
        if (q >= width[b] || l >= width[b]) G[q * BW + l] = (q == l) ? 1.0 : 0.0;
    return chol_upper(G.data(), BW, BLOCK_DELTA * BLOCK_DELTA * scale2, R);
  };
  // second Cholesky QR pass over X for the blocks flagged in f_dots: R_b <- R2 R_b
  auto cholqr2 = [&](double2* X, std::vector<zc>& R) {
    gram(X);
    for (int b = 0; b < nb; ++b) {
      f_upd[b] = 0;
      if (!f_dots[b]) continue;
      zc* r2 = &R2[(size_t)b * 1024];
      if (chol(&hG[(size_t)b * 1024], b, 1.0, r2) > 0) set_identity(r2);
      tri_inv_upper(r2, BW, &hR[(size_t)b * 1024]);
      std::vector<zc> t(1024);
      matmul(r2, &R[(size_t)b * 1024], BW, t.data());
      std::copy(t.begin(), t.end(), R.begin() + (size_t)b * 1024);
      f_upd[b] = 1;
    }
    scale(X);
  };

  // starting block: Gram matrix of the residuals, Cholesky, V_0 = R0 S0^-1
  for (int b = 0; b < nb; ++b) f_dots[b] = 1;
  gram(V);
  int nact = 0;
  bool again = false;
  for (int b = 0; b < nb; ++b) {
    const zc* Gb = &hG[(size_t)b * 1024];
    double s2 = 0.0;
    for (int q = 0; q < width[b]; ++q) s2 = std::max(s2, Gb[q * BW + q].real());
    zc* r1 = &R1[(size_t)b * 1024];
    f_dots[b] = 0;
    f_upd[b] = 2;
    set_identity(&hR[(size_t)b * 1024]);
    if (!(s2 > 0.0) || chol(Gb, b, s2, r1) > 0) continue;
    tri_inv_upper(r1, BW, &hR[(size_t)b * 1024]);
    active[b] = 1;
    f_upd[b] = 1;
    ++nact;
    if (frob(r1, BW) * frob(&hR[(size_t)b * 1024], BW) > BLOCK_COND2) { f_dots[b] = 1; again = true; }
  }
  scale(V);
  if (again) cholqr2(V, R1);
  for (int b = 0; b < nb; ++b)
    if (active[b]) ls[b].start(m, &R1[(size_t)b * 1024], width[b]);
  if (nact == 0) return;

  for (int j = 0; j < m && nact > 0; ++j) {
    double2* Vj = V + (int64_t)j * vstride;
    double2* Vn = V + (int64_t)(j + 1) * vstride;
    const int kv = j + 1;
    for (int b = 0; b < nb; ++b) f_dots[b] = active[b] ? 1 : 0;
    upload_flags(f_dots, d_dots);
    apply_prec(p, W, Vj, U, nca, ld);
    launch_spmm(p->dm, p->val.as<double2>(), U, ld, T, ld, nca, nullptr, 0, st);
    // first pass: P1 = V^H T, T -= V P1
    launch_bdots(V, vstride, kv, nullptr, T, n, ld, nca, nb, d_dots, part, &nch, st);
    launch_sum_chunks_c(part, nch, (int64_t)nb * kv * 1024, dP1, st);
    launch_bupdate(V, vstride, kv, nullptr, kv, dP1, kv, nullptr, T, T, n, ld, nca, nb, d_dots, st);
    // second pass: [P2; G1] = [V T]^H T
    launch_bdots(V, vstride, kv, T, T, n, ld, nca, nb, d_dots, part, &nch, st);
    launch_sum_chunks_c(part, nch, (int64_t)nb * (kv + 1) * 1024, dP2, st);
    hP1.resize((size_t)nb * kv * 1024);
    hP2.resize((size_t)nb * (kv + 1) * 1024);
    MW_HIP(hipMemcpyAsync(hP1.data(), dP1, hP1.size() * 16, hipMemcpyDeviceToHost, st));
    MW_HIP(hipMemcpyAsync(hP2.data(), dP2, hP2.size() * 16, hipMemcpyDeviceToHost, st));
    MW_HIP(hipStreamSynchronize(st));
    // R of every active block; deficient ones end their cycle at this step
    std::vector<int> ndef(nb, 0);
    std::vector<char> cond2(nb, 0);
    parallel_items(nb, [&](int, int64_t bi) {
      const int b = (int)bi;
      if (!active[b]) return;
      const zc* P1 = hP1.data() + (size_t)b * kv * 1024;
      const zc* P2 = hP2.data() + (size_t)b * (kv + 1) * 1024;
      const zc* G1 = P2 + (size_t)kv * 1024;
      // squared column norms of A M^-1 V_j: ||P1 e_c||^2 + ||T e_c||^2
      double s2 = 0.0;
      for (int q = 0; q < width[b]; ++q) {
        double s = G1[q * BW + q].real();
        for (int r = 0; r < kv * BW; ++r) s += std::norm(P1[(size_t)r * BW + q]);
        s2 = std::max(s2, s);
      }
      std::vector<zc> G(1024);
      for (int q = 0; q < BW; ++q)
        for (int l = 0; l < BW; ++l) {
          zc s = G1[q * BW + l];
          for (int r = 0; r < kv * BW; ++r) s -= std::conj(P2[(size_t)r * BW + q]) * P2[(size_t)r * BW + l];
          G[q * BW + l] = s;
        }
      zc* r1 = &R1[(size_t)b * 1024];
      ndef[b] = chol(G.data(), b, s2, r1);
      if (ndef[b] == 0) {
        tri_inv_upper(r1, BW, &hR[(size_t)b * 1024]);
        cond2[b] = frob(r1, BW) * frob(&hR[(size_t)b * 1024], BW) > BLOCK_COND2;
      }
    });
    bool need2 = false;
    for (int b = 0; b < nb; ++b) need2 |= cond2[b] != 0;
    if (need2) {
      // an ill-conditioned factor: form V_{j+1} now and repeat its Cholesky QR
      for (int b = 0; b < nb; ++b) {
        f_upd[b] = (active[b] && ndef[b] == 0) ? 1 : 0;
        f_dots[b] = cond2[b];
      }
      upload_flags(f_upd, d_upd);
      MW_HIP(hipMemcpyAsync(dR, hR.data(), (size_t)nb * 1024 * 16, hipMemcpyHostToDevice, st));
      launch_bupdate(V, vstride, kv, nullptr, kv, dP2, kv + 1, dR, T, Vn, n, ld, nca, nb, d_upd, st);
      cholqr2(Vn, R1);
    }
    // append block column j and test convergence
    std::vector<char> finished(nb, 0);
    parallel_items(nb, [&](int, int64_t bi) {
      const int b = (int)bi;
      if (!active[b]) return;
      const zc* P1 = hP1.data() + (size_t)b * kv * 1024;
      const zc* P2 = hP2.data() + (size_t)b * (kv + 1) * 1024;
      std::vector<zc> Hc((size_t)kv * 1024);
      for (size_t e = 0; e < Hc.size(); ++e) Hc[e] = P1[e] + P2[e];
      ls[b].add(Hc.data(), &R1[(size_t)b * 1024]);
      steps[b] = kv;
      bool done = ndef[b] > 0 || kv >= maxsteps[b];
      if (!done) {
        done = true;
        for (int q = 0; q < width[b]; ++q)
          if (!(ls[b].resid(q) <= atol[(size_t)b * BW + q])) done = false;
      }
      finished[b] = done;
    });
    for (int b = 0; b < nb; ++b)
      if (active[b] && finished[b]) { active[b] = 0; --nact; }
    if (nact == 0 || j + 1 == m) break;
    if (!need2) {
      // V_{j+1} = (T - V P2) R^-1 for the blocks that go on, zero for the others
      for (int b = 0; b < nb; ++b) f_upd[b] = active[b] ? 1 : 2;
      upload_flags(f_upd, d_upd);
      MW_HIP(hipMemcpyAsync(dR, hR.data(), (size_t)nb * 1024 * 16, hipMemcpyHostToDevice, st));
      launch_bupdate(V, vstride, kv, nullptr, kv, dP2, kv + 1, dR, T, Vn, n, ld, nca, nb, d_upd, st);
    } else {
      for (int b = 0; b < nb; ++b) f_upd[b] = active[b] ? 0 : 2;
      upload_flags(f_upd, d_upd);
      launch_bupdate(V, vstride, 0, nullptr, 0, dR, 0, nullptr, nullptr, Vn, n, ld, nca, nb, d_upd, st);
    }
  }
  // U = M^-1 V Y
  int kmax = 0;
  std::vector<zc> Y((size_t)nb * m * 1024, zc(0.0));
  parallel_items(nb, [&](int, int64_t bi) {
    const int b = (int)bi;
    if (steps[b] == 0) return;
    zc* Yb = &Y[(size_t)b * m * 1024];
    ls[b].solve(Yb);
    for (int64_t e = 0; e < (int64_t)steps[b] * 1024; ++e) Yb[e] = -Yb[e];
  });
  for (int b = 0; b < nb; ++b) {
    f_kv[b] = steps[b];
    f_upd[b] = steps[b] > 0 ? 1 : 2;
    kmax = std::max(kmax, steps[b]);
  }
  upload_flags(f_kv, d_kv);
  upload_flags(f_upd, d_upd);
  MW_HIP(hipMemcpyAsync(dY, Y.data(), Y.size() * 16, hipMemcpyHostToDevice, st));
  launch_bupdate(V, vstride, 0, d_kv, kmax, dY, m, nullptr, nullptr, T, n, ld, nca, nb, d_upd, st);
  apply_prec(p, W, T, U, nca, ld);
  // the host vectors read by the asynchronous uploads must outlive them
  MW_HIP(hipStreamSynchronize(st));
}

// Block GMRES(m) to convergence on nc columns (one memory chunk of
// mw_solve): each restart recomputes the true residuals, regroups the
// columns still above tol (in column order) into blocks of BW and runs a
// block cycle on them.  Columns whose starting block is rank deficient are
// finished by the pseudo-block solver from the current iterate.
ChunkResult block_chunk(mw_problem* p, GmresWork& W, const double2* Bsrc, int64_t ldb_src, double2* Xdst,
                        int64_t ldx_dst, int nc, const mw_solve_opts& o, int32_t* iters_out, double* relres_out) {
  mw_ctx* c = p->ctx;
  hipStream_t st = W.st;
  const int64_t n = p->T.n();
  const int64_t ld = nc;
  const int64_t vstride = n * ld;
  const int m = o.restart;
  double2* X = (double2*)W.X.get(c, vstride * 16);
  double2* B = (double2*)W.B.get(c, vstride * 16);
  double2* Z = (double2*)W.Z.get(c, vstride * 16);
  double* vec = (double*)W.vec.get(c, (int64_t)4 * nc * 8);
  double* rn2 = vec + nc;
  int32_t* didx = (int32_t*)W.w_idx.get(c, (int64_t)nc * 4);

  launch_copy_cols(Bsrc, ldb_src, B, ld, n, nc, st);
  if (o.use_x0) launch_copy_cols(Xdst, ldx_dst, X, ld, n, nc, st);
  else launch_zero(X, vstride, st);
  std::vector<double> hb(nc), hr, hb2(nc);
  colnorm2(p, W, B, ld, nc, rn2);
  MW_HIP(hipMemcpyAsync(hb2.data(), rn2, nc * 8, hipMemcpyDeviceToHost, st));
  MW_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < nc; ++k) hb[k] = std::sqrt(hb2[k]);

  ChunkResult res;
  std::vector<int32_t> iters(nc, 0);
  std::vector<double> relres(nc, 0.0);
  std::vector<char> single(nc, 0);
  for (;;) {
    true_residual(p, W, B, X, Z, nc, rn2, hr);
    std::vector<int32_t> act;
    for (int k = 0; k < nc; ++k) {
      double r = std::sqrt(hr[k]);
      if (!std::isfinite(r)) res.numeric = true;
      relres[k] = hb[k] > 0 ? r / hb[k] : 0.0;
      if (column_continues(hb[k], relres[k], iters[k], r, o) && !single[k]) act.push_back(k);
    }
    if (res.numeric || act.empty()) break;
    res.cycles++;
    const int nca = (int)act.size();
    const int nb = (int)ceil_div(nca, BW);
    std::vector<double> atol((size_t)nb * BW, 0.0);
    std::vector<int> maxsteps(nb, m);
    for (int q = 0; q < nca; ++q) {
      atol[q] = o.tol * hb[act[q]];
      maxsteps[q / BW] = std::min(maxsteps[q / BW], o.maxit - iters[act[q]]);
    }
    MW_HIP(hipMemcpyAsync(didx, act.data(), nca * 4, hipMemcpyHostToDevice, st));
    double2* V = (double2*)W.V.get(c, (int64_t)(m + 1) * n * nca * 16);
    launch_gather_cols(Z, ld, didx, V, nca, n, nca, st);
    std::vector<int> steps;
    block_cycle(p, W, nca, m, atol, maxsteps, Z, steps);
    // X[:, act] += U
    double2* T = (double2*)W.tmp.get(c, vstride * 16);
    launch_gather_cols(X, ld, didx, T, nca, n, nca, st);
    launch_axpy_cols(T, Z, n, nca, nca, st);
    launch_scatter_cols(T, nca, didx, X, ld, n, nca, st);
    for (int q = 0; q < nca; ++q) {
      const int s = steps[q / BW];
      if (s == 0) single[act[q]] = 1;
      iters[act[q]] += s;
    }
  }
  launch_copy_cols(X, ld, Xdst, ldx_dst, n, nc, st);
  MW_HIP(hipStreamSynchronize(st));
  // columns left to the pseudo-block solver
  std::vector<int32_t> rest;
  int rest_max_it = 0;
  for (int k = 0; k < nc; ++k)
    if (single[k] && !res.numeric && column_continues(hb[k], relres[k], iters[k], relres[k] * hb[k], o)) {
      rest.push_back(k);
      rest_max_it = std::max(rest_max_it, iters[k]);
    }
  if (!rest.empty()) {
    const int ns = (int)rest.size();
    DevBuf Bs = dalloc(c, n * ns * 16), Xs = dalloc(c, n * ns * 16), ix = dalloc(c, (int64_t)ns * 4);
    MW_HIP(hipMemcpyAsync(ix.p, rest.data(), ns * 4, hipMemcpyHostToDevice, st));
    launch_gather_cols(Bsrc, ldb_src, ix.as<int32_t>(), Bs.as<double2>(), ns, n, ns, st);
    launch_gather_cols(Xdst, ldx_dst, ix.as<int32_t>(), Xs.as<double2>(), ns, n, ns, st);
    mw_solve_opts o2 = o;
    o2.use_x0 = 1;
    o2.maxit = std::max(1, o.maxit - rest_max_it);
    std::vector<int32_t> it2(ns);
    std::vector<double> rr2(ns);
    ChunkResult r2 = gmres_chunk(p, W, Bs.as<double2>(), ns, Xs.as<double2>(), ns, ns, o2, it2.data(), rr2.data());
    launch_scatter_cols(Xs.as<double2>(), ns, ix.as<int32_t>(), Xdst, ldx_dst, n, ns, st);
    MW_HIP(hipStreamSynchronize(st));
    res.numeric |= r2.numeric;
    res.cycles += r2.cycles;
    for (int q = 0; q < ns; ++q) {
      iters[rest[q]] += it2[q];
      relres[rest[q]] = rr2[q];
    }
  }
  for (int k = 0; k < nc; ++k) {
    if (iters_out) iters_out[k] = iters[k];
    if (relres_out) relres_out[k] = relres[k];
    res.max_iters = std::max(res.max_iters, iters[k]);
  }
  return res;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* mw_last_error(void) { return g_last_error.c_str(); }

mw_status mw_create(mw_ctx** out, int device, int64_t hbm_budget_bytes) {
  return guard([&] {
    MW_CHECK(out != nullptr, MW_EINVAL, "out is NULL");
    int ndev = 0;
    MW_HIP(hipGetDeviceCount(&ndev));
    MW_CHECK(device >= 0 && device < ndev, MW_EINVAL, "device ordinal out of range");
    DeviceGuard dg(device);
    size_t fr = 0, tot = 0;
    MW_HIP(hipMemGetInfo(&fr, &tot));
    (void)scratch_for_device(device, true);
    auto* c = new mw_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes > 0 ? hbm_budget_bytes : (int64_t)(0.95 * (double)tot);
    *out = c;
  });
}

mw_status mw_set_stream(mw_ctx* ctx, void* stream) {
  return guard([&] {
    MW_CHECK(ctx != nullptr, MW_EINVAL, "ctx is NULL");
    ctx->stream = (hipStream_t)stream;
  });
}

mw_status mw_destroy(mw_ctx* ctx) {
  return guard([&] {
    if (!ctx) return;
    MW_CHECK(ctx->used.load() == 0, MW_EINVAL, "destroy every problem of the context first");
    delete ctx;
  });
}

mw_status mw_assemble(mw_ctx* ctx, const mw_mesh* mesh, const mw_complex* eps_r, double k0, mw_complex beta_imp,
                      const mw_port* ports, int32_t nports, mw_problem** out) {
  return guard([&] {
    MW_CHECK(ctx && mesh && eps_r && out, MW_EINVAL, "NULL argument");
    MW_CHECK(nports >= 0 && (nports == 0 || ports), MW_EINVAL, "ports");
    MW_CHECK(std::isfinite(k0) && k0 > 0, MW_EINVAL, "k0 must be positive");
    DeviceGuard dg(ctx->device);
    double t0 = now_s();
    auto p = std::make_unique<mw_problem>();
    p->ctx = ctx;
    p->stream = ctx->stream;
    p->k0 = k0;
    p->beta_imp = beta_imp;
    p->ports.assign(ports, ports + nports);
    build_topology(*mesh, p->T);
    Topology& T = p->T;
    for (int32_t f = 0; f < T.nbf; ++f)
      MW_CHECK(T.btag[f] <= nports, MW_EINVAL, "face tag refers to a port beyond nports");
    std::vector<double2> fb(std::max(1, T.nbf), make_double2(0, 0));
    for (int32_t f = 0; f < T.nbf; ++f) {
      if (T.btag[f] == MW_TAG_IMPEDANCE) fb[f] = make_double2(beta_imp.re, beta_imp.im);
      else if (T.btag[f] >= 1) fb[f] = make_double2(ports[T.btag[f] - 1].beta.re, ports[T.btag[f] - 1].beta.im);
    }
    std::vector<double2> e(T.nt);
    for (int32_t t = 0; t < T.nt; ++t) e[t] = make_double2(eps_r[t].re, eps_r[t].im);
    p->xyz = upload(ctx, p->stream, T.xyz);
    p->tet = upload(ctx, p->stream, T.tet);
    p->t2e = upload(ctx, p->stream, T.t2e);
    p->dof = upload(ctx, p->stream, T.dof);
    p->bface = upload(ctx, p->stream, T.bface);
    p->bf2e = upload(ctx, p->stream, T.bf2e);
    p->fbeta = upload(ctx, p->stream, fb);
    p->row_ptr = upload(ctx, p->stream, T.row_ptr);
    const std::vector<int32_t> zrows = zorder_rows(T);
    p->rorder = upload(ctx, p->stream, zrows);
    {
      const SellLayout L = build_sell(T, zrows);
      p->sl_row = upload(ctx, p->stream, L.row);
      p->sl_off = upload(ctx, p->stream, L.off);
      p->sl_col = upload(ctx, p->stream, L.col);
      p->sl_idx = upload(ctx, p->stream, L.idx);
      p->sl_val = dalloc(ctx, (int64_t)L.col.size() * 16);
    }
    p->col = upload(ctx, p->stream, T.col);
    p->rt_ptr = upload(ctx, p->stream, T.rt_ptr);
    p->rt = upload(ctx, p->stream, T.rt);
    p->rf_ptr = upload(ctx, p->stream, T.rf_ptr);
    p->rf = upload(ctx, p->stream, T.rf);
    p->eps = upload(ctx, p->stream, e);
    p->E = dalloc(ctx, (int64_t)T.nt * 21 * 16);
    p->val = dalloc(ctx, (int64_t)T.col.size() * 16);
    DeviceMesh& m = p->dm;
    m.nv = T.nv; m.nt = T.nt; m.n = T.n(); m.nbf = T.nbf; m.nnz = (int64_t)T.col.size();
    m.xyz = p->xyz.as<double>(); m.tet = p->tet.as<int32_t>(); m.t2e = p->t2e.as<int32_t>();
    m.dof = p->dof.as<int32_t>(); m.bface = p->bface.as<int32_t>(); m.bf2e = p->bf2e.as<int32_t>();
    m.fbeta = p->fbeta.as<double2>(); m.row_ptr = p->row_ptr.as<int64_t>(); m.col = p->col.as<int32_t>();
    m.rt_ptr = p->rt_ptr.as<int64_t>(); m.rt = p->rt.as<int32_t>(); m.rf_ptr = p->rf_ptr.as<int64_t>();
    m.rf = p->rf.as<int32_t>();
    m.rorder = p->rorder.as<int32_t>();
    m.sl_slots = (int64_t)(p->sl_row.bytes / 4);
    m.sl_row = p->sl_row.as<int32_t>();
    m.sl_off = p->sl_off.as<int64_t>();
    m.sl_col = p->sl_col.as<int32_t>();
    m.sl_val = p->sl_val.as<double2>();
    m.csr_val = p->val.as<double2>();
    assemble_values(p.get());
    setup_ports(p.get());
    psync(p.get());
    p->t_assemble = now_s() - t0;
    *out = p.release();
  });
}

mw_status mw_set_coarse_space(mw_problem* p, int32_t kind) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(kind == MW_COARSE_NONE || kind == MW_COARSE_CONST, MW_EINVAL, "unknown coarse space");
    if (kind != p->coarse_kind) {
      p->coarse_kind = kind;
      p->coarse_active = false;
      p->factors_valid = false;
      p->state++;
      if (kind == MW_COARSE_NONE) p->Fc.release();
    }
  });
}

mw_status mw_set_factorization(mw_problem* p, int32_t kind) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(kind == MW_FACTOR_AUTO || kind == MW_FACTOR_LU || kind == MW_FACTOR_LDLT, MW_EINVAL,
             "unknown factorisation kind");
    p->factor_kind = kind;
  });
}

mw_status mw_set_krylov_basis(mw_problem* p, int32_t kind) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(kind == MW_BASIS_AUTO || kind == MW_BASIS_FP64 || kind == MW_BASIS_FP32_LEAN, MW_EINVAL,
             "unknown Krylov basis kind");
    p->basis = kind;
  });
}

mw_status mw_set_solve_form(mw_problem* p, int32_t form) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(form == MW_SOLVE_AUTO || form == MW_SOLVE_RECURSIVE || form == MW_SOLVE_ROWS, MW_EINVAL,
             "unknown solve form");
    p->solve_form = form;
  });
}

mw_status mw_update_eps(mw_problem* p, const void* eps_dev) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(eps_dev != nullptr, MW_EINVAL, "eps is NULL");
    DeviceGuard dg(p->ctx->device);
    double t0 = now_s();
    p->state++;
    MW_HIP(hipMemcpyAsync(p->eps.p, eps_dev, (size_t)p->T.nt * 16, hipMemcpyDeviceToDevice, p->stream));
    p->eps_p1 = false;
    assemble_values(p);
    p->factors_valid = false;
    psync(p);
    p->t_assemble = now_s() - t0;
  });
}

mw_status mw_update_eps_vertex(mw_problem* p, const void* eps_vertex_dev) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(eps_vertex_dev != nullptr, MW_EINVAL, "eps is NULL");
    DeviceGuard dg(p->ctx->device);
    double t0 = now_s();
    p->state++;
    if (p->eps_v.p == nullptr) p->eps_v = dalloc(p->ctx, (int64_t)p->T.nv * 16);
    MW_HIP(hipMemcpyAsync(p->eps_v.p, eps_vertex_dev, (size_t)p->T.nv * 16, hipMemcpyDeviceToDevice, p->stream));
    p->eps_p1 = true;
    assemble_values(p);
    p->factors_valid = false;
    psync(p);
    p->t_assemble = now_s() - t0;
  });
}

mw_status mw_gradient_vertex(mw_problem* p, int32_t ntx, const void* U, const void* F, void* grad_vertex) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(ntx >= 1 && U && F && grad_vertex, MW_EINVAL, "NULL argument");
    DeviceGuard dg(p->ctx->device);
    const int64_t nt = p->T.nt, nv = p->T.nv;
    if (p->vt.p == nullptr) {
      // (t*4 + slot) entries of every vertex, ascending t
      std::vector<int64_t> ptr(nv + 1, 0);
      for (int64_t e = 0; e < nt * 4; ++e) ptr[p->T.tet[e] + 1]++;
      for (int64_t v = 0; v < nv; ++v) ptr[v + 1] += ptr[v];
      std::vector<int32_t> lst(nt * 4);
      std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
      for (int64_t e = 0; e < nt * 4; ++e) lst[fill[p->T.tet[e]]++] = (int32_t)e;
      p->vt_ptr = upload(p->ctx, p->stream, ptr);
      p->vt = upload(p->ctx, p->stream, lst);
    }
    DevBuf G = dalloc(p->ctx, nt * 4 * 16);
    launch_gradient_p1(p->dm, (const double2*)U, (const double2*)F, ntx, ntx, p->k0, p->vt_ptr.as<int64_t>(),
                       p->vt.as<int32_t>(), G.as<double2>(), (double2*)grad_vertex, p->stream);
    psync(p);
  });
}

mw_status mw_problem_get_info(mw_problem* p, mw_problem_info* info) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(info != nullptr, MW_EINVAL, "info is NULL");
    std::memset(info, 0, sizeof(*info));
    info->n = p->T.n();
    info->nnz = (int64_t)p->T.col.size();
    info->n_edges = p->T.ne();
    info->nt = p->T.nt;
    info->nports = (int32_t)p->ports.size();
    if (p->has_dec) {
      info->n_sub = p->D.nsub;
      info->sum_ni = std::accumulate(p->D.n_loc.begin(), p->D.n_loc.end(), (int64_t)0);
      info->max_ni = *std::max_element(p->D.n_loc.begin(), p->D.n_loc.end());
    }
    info->precision = p->prec;
    info->factorization = p->factors_valid ? p->factorization : 0;
    info->factor_bytes = (int64_t)p->F.bytes;
    info->t_assemble = p->t_assemble;
    info->t_decompose = p->t_decompose;
    info->t_factor = p->t_factor;
    info->state = p->state;
    info->coarse_size = p->coarse_active ? 3 * p->D.nsub : 0;
  });
}

mw_status mw_dof_edges(mw_problem* p, int32_t* edge_of_dof, int32_t* edge_vertices) {
  return guard([&] {
    check_prob(p);
    if (edge_of_dof) std::copy(p->T.free_edge.begin(), p->T.free_edge.end(), edge_of_dof);
    if (edge_vertices)
      for (size_t k = 0; k < p->T.edges.size(); ++k) edge_vertices[k] = (int32_t)p->T.edges[k];
  });
}

mw_status mw_get_matrix(mw_problem* p, void* row_ptr, void* col, void* val) {
  return guard([&] {
    check_prob(p);
    DeviceGuard dg(p->ctx->device);
    hipStream_t st = p->stream;
    if (row_ptr) MW_HIP(hipMemcpyAsync(row_ptr, p->row_ptr.p, p->row_ptr.bytes, hipMemcpyDeviceToDevice, st));
    if (col) MW_HIP(hipMemcpyAsync(col, p->col.p, p->col.bytes, hipMemcpyDeviceToDevice, st));
    if (val) MW_HIP(hipMemcpyAsync(val, p->val.p, p->val.bytes, hipMemcpyDeviceToDevice, st));
    psync(p);
  });
}

mw_status mw_destroy_problem(mw_problem* p) {
  return guard([&] {
    if (!p) return;
    MW_CHECK(p->live_batches == 0, MW_EINVAL, "destroy the problem's batches first");
    MW_CHECK(p->live_users == 0, MW_EINVAL, "destroy the inversions driving the problem first");
    if (p->ctx) { DeviceGuard dg(p->ctx->device); (void)hipStreamSynchronize(p->stream); delete p; }
    else delete p;
  });
}

mw_status mw_rhs_ports(mw_problem* p, int32_t ntx, const int32_t* tx, void* B) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(ntx >= 0 && (ntx == 0 || (tx && B)), MW_EINVAL, "NULL argument");
    for (int j = 0; j < ntx; ++j) MW_CHECK(tx[j] >= 0 && tx[j] < (int)p->ports.size(), MW_EINVAL, "port index out of range");
    if (ntx == 0) return;
    DeviceGuard dg(p->ctx->device);
    hipStream_t st = p->stream;
    std::vector<int32_t> h(tx, tx + ntx);
    int32_t* d = (int32_t*)p->w_small.get(p->ctx, ntx * 4);
    MW_HIP(hipMemcpyAsync(d, h.data(), ntx * 4, hipMemcpyHostToDevice, st));
    launch_zero((double2*)B, p->T.n() * ntx, st);
    launch_rhs_ports(p->dp, ntx, d, (double2*)B, ntx, st);
    psync(p);
  });
}

mw_status mw_rhs_dipoles(mw_problem* p, int32_t np, const double* xyz, const double* dir, void* B) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(np >= 0 && (np == 0 || (xyz && dir && B)), MW_EINVAL, "NULL argument");
    if (np == 0) return;
    DeviceGuard dg(p->ctx->device);
    hipStream_t st = p->stream;
    char* w = (char*)p->w_small.get(p->ctx, (int64_t)np * (48 + 4));
    double* pts = (double*)w;
    double* dirs = pts + 3 * np;
    int* found = (int*)(dirs + 3 * np);
    std::vector<int> init(np, 0x7fffffff);
    MW_HIP(hipMemcpyAsync(pts, xyz, np * 24, hipMemcpyHostToDevice, st));
    MW_HIP(hipMemcpyAsync(dirs, dir, np * 24, hipMemcpyHostToDevice, st));
    MW_HIP(hipMemcpyAsync(found, init.data(), np * 4, hipMemcpyHostToDevice, st));
    launch_locate(p->dm, pts, np, found, st);
    std::vector<int> hf(np);
    MW_HIP(hipMemcpyAsync(hf.data(), found, np * 4, hipMemcpyDeviceToHost, st));
    psync(p);
    for (int j = 0; j < np; ++j) MW_CHECK(hf[j] != 0x7fffffff, MW_EINVAL, "dipole point outside the mesh");
    launch_zero((double2*)B, p->T.n() * np, st);
    launch_rhs_dipoles(p->dm, pts, dirs, found, np, (double2*)B, np, st);
    psync(p);
  });
}

mw_status mw_factor_subdomains(mw_problem* p, int32_t n_sub, int32_t overlap, mw_precision prec,
                               const int32_t* tet_part) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(prec == MW_C64 || prec == MW_C128, MW_EINVAL, "precision must be MW_C64 or MW_C128");
    mw_ctx* c = p->ctx;
    DeviceGuard dg(c->device);
    double t0 = now_s();
    p->state++;
    uint64_t key = hash_part(tet_part, p->T.nt, n_sub, overlap);
    if (!p->has_dec || key != p->dec_key) {
      p->has_dec = false;
      p->factors_valid = false;
      p->F.release();
      const int32_t* part = tet_part;
      if (part == nullptr) {
        partition_rcb(p->T, n_sub, p->own_part);
        part = p->own_part.data();
      }
      Decomposition D;
      build_decomposition(p->T, part, n_sub, overlap, 64, D);
      p->D = std::move(D);
      p->coarse_built = p->coarse_active = false;
      p->Fc.release();
      upload_decomp(p);
      p->has_dec = true;
      p->dec_key = key;
    }
    double t1 = now_s();
    p->t_decompose = t1 - t0;
    hipStream_t st = p->stream;
    const bool sym = choose_sym(p);
    int64_t esz = prec == MW_C64 ? 8 : 16;
    int64_t need = factor_elems(p->D, sym) * esz;
    p->factors_valid = false;
    if ((int64_t)p->F.bytes != need) {
      p->F.release();
      // solve workspaces are re-created on demand; give their memory to the factors
      p->ws.release();
      p->F = dalloc(c, need);
    }
    set_layout(p, sym);
    p->prec = prec;
    p->factorization = sym ? MW_FACTOR_LDLT : MW_FACTOR_LU;
    p->dd.rows = p->solve_form == MW_SOLVE_ROWS || (p->solve_form == MW_SOLVE_AUTO && p->dd.nsub >= 512);
    launch_zero_bytes(p->dd.info, (int64_t)p->dd.nsub * 4, st);
    if (prec == MW_C64) {
      launch_fill_local<float2>(p->dm, p->dd, p->E.as<double2>(), p->eps.as<double2>(), p->k0, p->F.as<float2>(), st);
      lu_factor_batched<float2>(p->dd, p->F.as<float2>(), st, sym);
    } else {
      launch_fill_local<double2>(p->dm, p->dd, p->E.as<double2>(), p->eps.as<double2>(), p->k0, p->F.as<double2>(), st);
      lu_factor_batched<double2>(p->dd, p->F.as<double2>(), st, sym);
    }
    std::vector<int32_t> info(p->dd.nsub);
    std::vector<double> amax(p->dd.nsub);
    MW_HIP(hipMemcpyAsync(info.data(), p->dd.info, info.size() * 4, hipMemcpyDeviceToHost, st));
    MW_HIP(hipMemcpyAsync(amax.data(), p->dd.amax, amax.size() * 8, hipMemcpyDeviceToHost, st));
    MW_HIP(hipMemcpyAsync(p->h_env.data(), p->dd.env, p->h_env.size() * 8, hipMemcpyDeviceToHost, st));
    psync(p);
    p->t_factor = now_s() - t1;
    for (int i = 0; i < p->dd.nsub; ++i)
      MW_CHECK(std::isfinite(amax[i]), MW_ENUMERIC,
               "NaN or Inf in the local matrix of subdomain " + std::to_string(i) + " (non-finite permittivity?)");
    for (int i = 0; i < p->dd.nsub; ++i)
      MW_CHECK(info[i] == 0, MW_ESINGULAR,
               "(near-)zero pivot in subdomain " + std::to_string(i) + " at column " + std::to_string(info[i] - 1));
    p->coarse_active = false;
    if (p->coarse_kind != MW_COARSE_NONE) {
      if (!p->coarse_built) build_coarse(p);
      const int64_t fcb = (int64_t)p->cdd.max_pad * p->cdd.max_pad * esz;
      if ((int64_t)p->Fc.bytes != fcb) {
        p->Fc.release();
        p->Fc = dalloc(c, fcb);
      }
      if (prec == MW_C64) factor_coarse<float2>(p, sym);
      else factor_coarse<double2>(p, sym);
      int32_t cinfo = 0;
      double camax = 0.0;
      MW_HIP(hipMemcpyAsync(&cinfo, p->cdd.info, 4, hipMemcpyDeviceToHost, st));
      MW_HIP(hipMemcpyAsync(&camax, p->cdd.amax, 8, hipMemcpyDeviceToHost, st));
      MW_HIP(hipMemcpyAsync(p->ch_env.data(), p->cdd.env, p->ch_env.size() * 8, hipMemcpyDeviceToHost, st));
      psync(p);
      MW_CHECK(std::isfinite(camax), MW_ENUMERIC, "NaN or Inf in the coarse matrix");
      MW_CHECK(cinfo == 0, MW_ESINGULAR, "(near-)zero pivot in the coarse matrix at column " + std::to_string(cinfo - 1));
      p->coarse_active = true;
    }
    p->factors_valid = true;
  });
}

mw_status mw_apply_preconditioner(mw_problem* p, int32_t nrhs, const void* V, void* Z) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(nrhs >= 0 && (nrhs == 0 || (V && Z)), MW_EINVAL, "NULL argument");
    if (nrhs == 0) return;
    DeviceGuard dg(p->ctx->device);
    p->ws.st = p->stream;
    apply_prec(p, p->ws, (const double2*)V, (double2*)Z, nrhs, nrhs);
    psync(p);
  });
}

mw_status mw_apply_preconditioner_noalloc(mw_problem* p, int32_t nrhs, const void* V, void* Z) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(nrhs >= 0 && (nrhs == 0 || (V && Z)), MW_EINVAL, "NULL argument");
    MW_CHECK(p->factors_valid, MW_EINVAL, "no valid subdomain factors: call mw_factor_subdomains");
    MW_CHECK(!p->coarse_active, MW_EINVAL,
             "mw_apply_preconditioner_noalloc applies the one-level preconditioner only: the two-level one needs "
             "workspace beyond the fixed buffer (use mw_apply_preconditioner)");
    if (nrhs == 0) return;
    const int64_t esz = p->prec == MW_C64 ? 8 : 16;
    const int64_t need = p->dd.sum_pad * (int64_t)nrhs * esz;
    MW_CHECK(need <= (int64_t)MW_NOALLOC_SCRATCH_BYTES, MW_EINVAL,
             "mw_apply_preconditioner_noalloc: the local vectors need " + std::to_string(need) +
                 " bytes, more than the fixed buffer's " + std::to_string((int64_t)MW_NOALLOC_SCRATCH_BYTES) +
                 " (sum of padded local sizes " + std::to_string(p->dd.sum_pad) + " x " + std::to_string(nrhs) +
                 " columns x " + std::to_string(esz) + " bytes); use fewer columns or mw_apply_preconditioner");
    DeviceGuard dg(p->ctx->device);
    void* Y = scratch_for_device(p->ctx->device, false);
    MW_CHECK(Y != nullptr, MW_EDEVICE, "the fixed buffer of this device was not set up (mw_create)");
    const int64_t n = p->T.n();
    const double2* Vd = (const double2*)V;
    double2* Zd = (double2*)Z;
    // the restriction writes every local row (zeros on the padding), so the
    // buffer needs no clearing between calls
    if (p->prec == MW_C64) {
      launch_restrict<float2>(p->dd, Vd, nrhs, nrhs, (float2*)Y, nrhs, p->stream);
      lu_solve_batched<float2>(p->dd, p->F.as<float2>(), (float2*)Y, nrhs, nrhs, p->stream);
      launch_prolong<float2>(p->dd, n, (const float2*)Y, nrhs, nrhs, Zd, nrhs, p->stream);
    } else {
      launch_restrict<double2>(p->dd, Vd, nrhs, nrhs, (double2*)Y, nrhs, p->stream);
      lu_solve_batched<double2>(p->dd, p->F.as<double2>(), (double2*)Y, nrhs, nrhs, p->stream);
      launch_prolong<double2>(p->dd, n, (const double2*)Y, nrhs, nrhs, Zd, nrhs, p->stream);
    }
    psync(p);
  });
}

static int solve_chunk_cols(mw_problem* p, int nrhs, int m, bool block) {
  mw_ctx* c = p->ctx;
  int64_t per = gmres_bytes_per_col(p, m, block);
  int64_t held = p->ws.held();
  int64_t avail = c->budget - c->used.load() + held;
  // block mode: reduction partials of the block Gram-Schmidt, bounded by
  // about 4096 32x32 products per sweep plus one per block and basis vector
  if (block) avail -= block_part_bytes(p->T.n(), (int)ceil_div(nrhs, BW), m) + (64 << 20);
  int64_t cols = avail / std::max<int64_t>(per, 1);
  // when the columns must be split, use multiples of 32 (the width granule of
  // the triangular-solve tiles) so that no tile runs half empty
  if (cols < nrhs && cols >= 32) cols = (cols / 32) * 32;
  return (int)std::min<int64_t>(nrhs, std::max<int64_t>(cols, 0));
}

mw_status mw_solve(mw_problem* p, int32_t nrhs, const void* B, void* X, const mw_solve_opts* o, mw_solve_info* info) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(nrhs >= 0 && (nrhs == 0 || (B && X)), MW_EINVAL, "NULL argument");
    mw_solve_opts op{1e-8, 30, 1000, 0, 0};
    if (o) op = *o;
    MW_CHECK(op.restart >= 1 && op.maxit >= 1 && op.tol > 0, MW_EINVAL, "invalid solve options");
    MW_CHECK(op.block == 0 || op.block == BW, MW_EINVAL, "block must be 0 (pseudo-block) or 32 (block GMRES)");
    MW_CHECK(p->factors_valid, MW_EINVAL, "no valid subdomain factors: call mw_factor_subdomains");
    if (info) { info->max_iters = 0; info->cycles = 0; info->chunks = 0; info->t_solve = 0; }
    if (nrhs == 0) return;
    DeviceGuard dg(p->ctx->device);
    double t0 = now_s();
    int cols = solve_chunk_cols(p, nrhs, op.restart, op.block != 0);
    MW_CHECK(cols >= 1, MW_ENOMEM, "HBM budget leaves no room for the Krylov basis of one column");
    bool numeric = false, noconv = false;
    int chunks = 0;
    for (int c0 = 0; c0 < nrhs; c0 += cols) {
      int nc = std::min(cols, nrhs - c0);
      std::vector<int32_t> it(nc);
      std::vector<double> rr(nc);
      p->ws.st = p->stream;
      ChunkResult r =
          op.block ? block_chunk(p, p->ws, (const double2*)B + c0, nrhs, (double2*)X + c0, nrhs, nc, op, it.data(),
                                 rr.data())
                   : gmres_chunk(p, p->ws, (const double2*)B + c0, nrhs, (double2*)X + c0, nrhs, nc, op, it.data(),
                                 rr.data());
      chunks++;
      numeric |= r.numeric;
      for (int k = 0; k < nc; ++k) {
        if (info && info->iters) info->iters[c0 + k] = it[k];
        if (info && info->relres) info->relres[c0 + k] = rr[k];
        if (!(rr[k] <= op.tol)) noconv = true;
      }
      if (info) { info->max_iters = std::max(info->max_iters, r.max_iters); info->cycles = std::max(info->cycles, r.cycles); }
    }
    if (info) { info->chunks = chunks; info->t_solve = now_s() - t0; }
    MW_CHECK(!numeric, MW_ENUMERIC, "NaN or Inf in a GMRES residual");
    MW_CHECK(!noconv, MW_ENOCONV, "GMRES did not reach the tolerance within maxit");
  });
}

mw_status mw_s_matrix(mw_problem* p, int32_t nrx, const int32_t* rx, int32_t ntx, const void* U, void* S) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(nrx >= 0 && ntx >= 0, MW_EINVAL, "sizes");
    if (nrx == 0 || ntx == 0) return;
    MW_CHECK(rx && U && S, MW_EINVAL, "NULL argument");
    for (int i = 0; i < nrx; ++i) MW_CHECK(rx[i] >= 0 && rx[i] < (int)p->ports.size(), MW_EINVAL, "port index out of range");
    DeviceGuard dg(p->ctx->device);
    hipStream_t st = p->stream;
    int32_t* d = (int32_t*)p->w_small.get(p->ctx, (int64_t)std::max(nrx, 1) * 4 + 16);
    MW_HIP(hipMemcpyAsync(d, rx, nrx * 4, hipMemcpyHostToDevice, st));
    launch_s_matrix(p->dp, nrx, d, ntx, (const double2*)U, ntx, (double2*)S, st);
    psync(p);
  });
}

mw_status mw_port_norms(mw_problem* p, double* nu) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(nu != nullptr, MW_EINVAL, "nu is NULL");
    if (p->ports.empty()) return;
    DeviceGuard dg(p->ctx->device);
    MW_HIP(hipMemcpyAsync(nu, p->dp.nu, p->ports.size() * 8, hipMemcpyDeviceToHost, p->stream));
    psync(p);
  });
}

mw_status mw_adjoint_rhs(mw_problem* p, int32_t nrx, const int32_t* rx, int32_t ntx, const void* gS, void* Lambda) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(nrx >= 1 && ntx >= 1 && rx && gS && Lambda, MW_EINVAL, "NULL argument or empty port set");
    for (int i = 0; i < nrx; ++i) MW_CHECK(rx[i] >= 0 && rx[i] < (int)p->ports.size(), MW_EINVAL, "port index out of range");
    DeviceGuard dg(p->ctx->device);
    hipStream_t st = p->stream;
    int32_t* d = (int32_t*)p->w_small.get(p->ctx, (int64_t)nrx * 4 + 16);
    MW_HIP(hipMemcpyAsync(d, rx, nrx * 4, hipMemcpyHostToDevice, st));
    launch_zero((double2*)Lambda, p->T.n() * ntx, st);
    launch_adjoint_rhs(p->dp, nrx, d, ntx, (const double2*)gS, (double2*)Lambda, ntx, st);
    psync(p);
  });
}

mw_status mw_gradient(mw_problem* p, int32_t ntx, const void* U, const void* F, void* grad_eps) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(ntx >= 1 && U && F && grad_eps, MW_EINVAL, "NULL argument");
    DeviceGuard dg(p->ctx->device);
    launch_gradient(p->dm, (const double2*)U, (const double2*)F, ntx, ntx, p->k0, (double2*)grad_eps, p->stream);
    psync(p);
  });
}

mw_status mw_misfit(mw_problem* p, int64_t count, const void* S_sim, const void* S_meas, void* gS, double* J) {
  return mw_misfit_weighted(p, count, S_sim, S_meas, nullptr, gS, J);
}

mw_status mw_misfit_weighted(mw_problem* p, int64_t count, const void* S_sim, const void* S_meas, const double* W,
                             void* gS, double* J) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(count >= 1 && S_sim && S_meas && gS && J, MW_EINVAL, "NULL argument");
    DeviceGuard dg(p->ctx->device);
    double* dJ = (double*)p->w_small.get(p->ctx, 16);
    launch_misfit((const double2*)S_sim, (const double2*)S_meas, W, count, (double2*)gS, dJ, p->stream);
    MW_HIP(hipMemcpyAsync(J, dJ, 8, hipMemcpyDeviceToHost, p->stream));
    psync(p);
  });
}

mw_status mw_adjoint_gradient(mw_problem* p, int32_t ntx, const int32_t* tx, int32_t nrx, const int32_t* rx,
                              const void* U, const void* gS, void* grad_eps, const mw_solve_opts* o,
                              mw_solve_info* info) {
  (void)tx;
  mw_status s = guard([&] {
    check_prob(p);
    MW_CHECK(ntx >= 1 && nrx >= 1 && rx && U && gS && grad_eps, MW_EINVAL, "NULL argument or empty port set");
  });
  if (s != MW_OK) return s;
  mw_ctx* c = p->ctx;
  const int64_t n = p->T.n();
  DevBuf lam, F;
  s = guard([&] {
    DeviceGuard dg(c->device);
    lam = dalloc(c, n * ntx * 16);
    F = dalloc(c, n * ntx * 16);
  });
  if (s != MW_OK) return s;
  if ((s = mw_adjoint_rhs(p, nrx, rx, ntx, gS, lam.p)) != MW_OK) return s;
  if ((s = mw_solve(p, ntx, lam.p, F.p, o, info)) != MW_OK) return s;
  return mw_gradient(p, ntx, U, F.p, grad_eps);
}

mw_status mw_misfit_gradient(mw_problem* p, int32_t ntx, const int32_t* tx, int32_t nrx, const int32_t* rx,
                             const void* S_meas, double* J, void* S_sim, void* grad_eps, const mw_solve_opts* o) {
  mw_status s = guard([&] {
    check_prob(p);
    MW_CHECK(ntx >= 1 && nrx >= 1 && tx && rx && S_meas && J && S_sim && grad_eps, MW_EINVAL, "NULL argument");
  });
  if (s != MW_OK) return s;
  mw_ctx* c = p->ctx;
  const int64_t n = p->T.n();
  DevBuf Bb, Ub, gS;
  s = guard([&] {
    DeviceGuard dg(c->device);
    Bb = dalloc(c, n * ntx * 16);
    Ub = dalloc(c, n * ntx * 16);
    gS = dalloc(c, (int64_t)nrx * ntx * 16);
  });
  if (s != MW_OK) return s;
  if ((s = mw_rhs_ports(p, ntx, tx, Bb.p)) != MW_OK) return s;
  if ((s = mw_solve(p, ntx, Bb.p, Ub.p, o, nullptr)) != MW_OK) return s;
  if ((s = mw_s_matrix(p, nrx, rx, ntx, Ub.p, S_sim)) != MW_OK) return s;
  if ((s = mw_misfit(p, (int64_t)nrx * ntx, S_sim, S_meas, gS.p, J)) != MW_OK) return s;
  return mw_adjoint_gradient(p, ntx, tx, nrx, rx, Ub.p, gS.p, grad_eps, o, nullptr);
}

// ---------------------------------------------------------------- serving support
mw_status mw_ctx_get_info(mw_ctx* ctx, int64_t* budget, int64_t* used) {
  return guard([&] {
    MW_CHECK(ctx != nullptr, MW_EINVAL, "ctx is NULL");
    if (budget) *budget = ctx->budget;
    if (used) *used = ctx->used.load();
  });
}

mw_status mw_problem_set_stream(mw_problem* p, void* stream) {
  return guard([&] {
    check_prob(p);
    DeviceGuard dg(p->ctx->device);
    psync(p);
    p->stream = (hipStream_t)stream;
  });
}

mw_status mw_release_factors(mw_problem* p) {
  return guard([&] {
    check_prob(p);
    DeviceGuard dg(p->ctx->device);
    psync(p);
    p->state++;
    p->F.release();
    p->Fc.release();
    p->ws.release();
    p->factors_valid = false;
    p->coarse_active = false;
  });
}

mw_status mw_factor_bytes(mw_problem* p, int32_t n_sub, int32_t overlap, mw_precision prec, const int32_t* tet_part,
                          int64_t* bytes) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(bytes != nullptr, MW_EINVAL, "NULL argument");
    MW_CHECK(prec == MW_C64 || prec == MW_C128, MW_EINVAL, "precision must be MW_C64 or MW_C128");
    int64_t esz = prec == MW_C64 ? 8 : 16;
    uint64_t key = hash_part(tet_part, p->T.nt, n_sub, overlap);
    MW_CHECK(p->has_dec && key == p->dec_key, MW_EINVAL,
             "no decomposition for this partition yet: call mw_factor_subdomains once");
    DeviceGuard dg(p->ctx->device);
    *bytes = factor_elems(p->D, choose_sym(p)) * esz;
  });
}

}  // extern "C"

// Continuous batching of pseudo-block GMRES columns over one problem.  Each
// request owns some column slots of the batch; its columns join the Krylov
// iteration at the next restart cycle and leave it at the restart where
// their true residual meets the tolerance.  Pseudo-block columns never mix,
// so a column's iterates do not depend on its batch-mates.
struct mw_batch {
  mw_problem* p = nullptr;
  mw_solve_opts o{};
  int max_cols = 0;
  DevBuf Bs, Xs, idx;   // slot storage n x max_cols (ld max_cols); device index list [max_cols]
  GmresWork W;          // compact per-cycle workspaces, released when the batch idles
  enum { FREE = 0, ACTIVE = 1, DONE = 2 };
  struct Slot {
    int64_t tag = -1;
    int state = FREE;
    int32_t iters = 0;
    double bnorm = 0, relres = 0;
    bool numeric = false;
  };
  std::vector<Slot> slots;
  struct Req {
    std::vector<int32_t> slots;
    int left = 0;
  };
  std::map<int64_t, Req> reqs;
  std::deque<int64_t> done;
  int64_t cycles = 0;
};

namespace {

void check_batch(mw_batch* b) {
  MW_CHECK(b != nullptr && b->p != nullptr, MW_EINVAL, "batch is NULL");
}

void batch_retire_if_done(mw_batch* b, int slot, int& finished) {
  auto it = b->reqs.find(b->slots[slot].tag);
  if (--it->second.left == 0) {
    b->done.push_back(it->first);
    ++finished;
  }
}

}  // namespace

extern "C" {

mw_status mw_batch_create(mw_problem* p, int32_t max_cols, const mw_solve_opts* o, mw_batch** out) {
  return guard([&] {
    check_prob(p);
    MW_CHECK(out != nullptr && max_cols >= 1, MW_EINVAL, "out is NULL or max_cols < 1");
    mw_solve_opts op{1e-8, 30, 1000, 0, 0};
    if (o) op = *o;
    MW_CHECK(op.restart >= 1 && op.maxit >= 1 && op.tol > 0, MW_EINVAL, "invalid solve options");
    MW_CHECK(!op.use_x0, MW_EINVAL, "batched columns start from x0 = 0");
    MW_CHECK(op.block == 0, MW_EINVAL, "batches run the pseudo-block solver (block must be 0)");
    DeviceGuard dg(p->ctx->device);
    auto b = std::make_unique<mw_batch>();
    b->p = p;
    b->o = op;
    b->max_cols = max_cols;
    const int64_t n = p->T.n();
    b->Bs = dalloc(p->ctx, n * max_cols * 16);
    b->Xs = dalloc(p->ctx, n * max_cols * 16);
    b->idx = dalloc(p->ctx, (int64_t)max_cols * 4);
    b->slots.resize(max_cols);
    p->live_batches++;
    *out = b.release();
  });
}

mw_status mw_batch_join(mw_batch* b, int64_t tag, int32_t ncols, const void* B) {
  return guard([&] {
    check_batch(b);
    MW_CHECK(tag >= 0 && ncols >= 1 && B, MW_EINVAL, "tag < 0, ncols < 1 or B NULL");
    MW_CHECK(b->reqs.find(tag) == b->reqs.end(), MW_EINVAL, "tag already in use in this batch");
    mw_problem* p = b->p;
    std::vector<int32_t> sl;
    for (int k = 0; k < b->max_cols && (int)sl.size() < ncols; ++k)
      if (b->slots[k].state == mw_batch::FREE) sl.push_back(k);
    MW_CHECK((int)sl.size() == ncols, MW_ENOMEM,
             "batch has " + std::to_string(sl.size()) + " free column slots, request needs " + std::to_string(ncols));
    DeviceGuard dg(p->ctx->device);
    hipStream_t st = p->stream;
    const int64_t n = p->T.n();
    MW_HIP(hipMemcpyAsync(b->idx.p, sl.data(), ncols * 4, hipMemcpyHostToDevice, st));
    launch_scatter_cols((const double2*)B, ncols, b->idx.as<int32_t>(), b->Bs.as<double2>(), b->max_cols, n, ncols, st);
    launch_scatter_cols(nullptr, 0, b->idx.as<int32_t>(), b->Xs.as<double2>(), b->max_cols, n, ncols, st);
    b->W.st = p->stream;
    double* nb = (double*)b->W.vec.get(p->ctx, (int64_t)4 * b->max_cols * 8);
    colnorm2(p, b->W, (const double2*)B, ncols, ncols, nb);
    std::vector<double> h(ncols);
    MW_HIP(hipMemcpyAsync(h.data(), nb, ncols * 8, hipMemcpyDeviceToHost, st));
    psync(p);
    mw_batch::Req r;
    r.slots = sl;
    r.left = ncols;
    b->reqs[tag] = r;
    int finished = 0;
    for (int k = 0; k < ncols; ++k) {
      mw_batch::Slot& s = b->slots[sl[k]];
      s.tag = tag;
      s.iters = 0;
      s.bnorm = std::sqrt(h[k]);
      s.relres = 0.0;
      s.numeric = !std::isfinite(s.bnorm);
      s.state = mw_batch::ACTIVE;
      if (!(s.bnorm > 0) || s.numeric) {   // b = 0: x = 0 is exact
        s.state = mw_batch::DONE;
        batch_retire_if_done(b, sl[k], finished);
      }
    }
  });
}

mw_status mw_batch_cycle(mw_batch* b, int32_t* n_active, int32_t* n_finished) {
  return guard([&] {
    check_batch(b);
    mw_problem* p = b->p;
    MW_CHECK(p->factors_valid, MW_EINVAL, "no valid subdomain factors: call mw_factor_subdomains");
    if (n_active) *n_active = 0;
    if (n_finished) *n_finished = 0;
    std::vector<int32_t> act;
    for (int k = 0; k < b->max_cols; ++k)
      if (b->slots[k].state == mw_batch::ACTIVE) act.push_back(k);
    const int na = (int)act.size();
    DeviceGuard dg(p->ctx->device);
    if (na == 0) {
      b->W.release();
      return;
    }
    if (n_active) *n_active = na;
    mw_ctx* c = p->ctx;
    hipStream_t st = p->stream;
    const int64_t n = p->T.n();
    GmresWork& W = b->W;
    W.st = st;
    double2* X = (double2*)W.X.get(c, n * na * 16);
    double2* Bc = (double2*)W.B.get(c, n * na * 16);
    double2* Z = (double2*)W.Z.get(c, n * na * 16);
    double* vec = (double*)W.vec.get(c, (int64_t)4 * b->max_cols * 8);
    std::vector<double> hb(na), hr, rnorm(na), relres(na);
    std::vector<int32_t> iters(na), hact(na);
    for (int k = 0; k < na; ++k) {
      hb[k] = b->slots[act[k]].bnorm;
      iters[k] = b->slots[act[k]].iters;
    }
    MW_HIP(hipMemcpyAsync(b->idx.p, act.data(), na * 4, hipMemcpyHostToDevice, st));
    MW_HIP(hipMemcpyAsync(vec, hb.data(), na * 8, hipMemcpyHostToDevice, st));
    launch_gather_cols(b->Bs.as<double2>(), b->max_cols, b->idx.as<int32_t>(), Bc, na, n, na, st);
    launch_gather_cols(b->Xs.as<double2>(), b->max_cols, b->idx.as<int32_t>(), X, na, n, na, st);
    // residual at the start of the cycle (x of the previous restart, or 0)
    true_residual(p, W, Bc, X, Z, na, vec + na, hr);
    for (int k = 0; k < na; ++k) {
      double r = std::sqrt(hr[k]);
      relres[k] = r / hb[k];
      rnorm[k] = r;
      hact[k] = column_continues(hb[k], relres[k], iters[k], r, b->o) ? 1 : 0;
    }
    if (basis_fp32(p)) gmres_cycle<float2>(p, W, X, Z, na, b->o, vec, rnorm, hact, iters);
    else gmres_cycle<double2>(p, W, X, Z, na, b->o, vec, rnorm, hact, iters);
    b->cycles++;
    // restart point: the true residual decides which columns leave
    true_residual(p, W, Bc, X, Z, na, vec + na, hr);
    launch_scatter_cols(X, na, b->idx.as<int32_t>(), b->Xs.as<double2>(), b->max_cols, n, na, st);
    psync(p);
    int finished = 0, still = 0;
    for (int k = 0; k < na; ++k) {
      mw_batch::Slot& s = b->slots[act[k]];
      double r = std::sqrt(hr[k]);
      s.iters = iters[k];
      s.relres = r / s.bnorm;
      s.numeric = !std::isfinite(r);
      if (column_continues(s.bnorm, s.relres, s.iters, r, b->o)) {
        ++still;
      } else {
        s.state = mw_batch::DONE;
        batch_retire_if_done(b, act[k], finished);
      }
    }
    if (still == 0) W.release();
    if (n_finished) *n_finished = finished;
  });
}

mw_status mw_batch_poll(mw_batch* b, int64_t* tag, int32_t* ncols) {
  return guard([&] {
    check_batch(b);
    MW_CHECK(tag != nullptr, MW_EINVAL, "tag is NULL");
    *tag = -1;
    if (ncols) *ncols = 0;
    if (b->done.empty()) return;
    *tag = b->done.front();
    if (ncols) *ncols = (int32_t)b->reqs[*tag].slots.size();
  });
}

mw_status mw_batch_take(mw_batch* b, int64_t tag, void* X, int32_t* iters, double* relres) {
  bool noconv = false, numeric = false;
  mw_status s = guard([&] {
    check_batch(b);
    MW_CHECK(X != nullptr, MW_EINVAL, "X is NULL");
    auto it = b->reqs.find(tag);
    MW_CHECK(it != b->reqs.end() && it->second.left == 0, MW_EINVAL, "request is unknown or not finished");
    mw_problem* p = b->p;
    DeviceGuard dg(p->ctx->device);
    const std::vector<int32_t>& sl = it->second.slots;
    const int nc = (int)sl.size();
    MW_HIP(hipMemcpyAsync(b->idx.p, sl.data(), nc * 4, hipMemcpyHostToDevice, p->stream));
    launch_gather_cols(b->Xs.as<double2>(), b->max_cols, b->idx.as<int32_t>(), (double2*)X, nc, p->T.n(), nc,
                       p->stream);
    psync(p);
    for (int k = 0; k < nc; ++k) {
      mw_batch::Slot& q = b->slots[sl[k]];
      if (iters) iters[k] = q.iters;
      if (relres) relres[k] = q.relres;
      noconv |= !(q.relres <= b->o.tol);
      numeric |= q.numeric;
      q = mw_batch::Slot();
    }
    b->reqs.erase(it);
    b->done.erase(std::find(b->done.begin(), b->done.end(), tag));
  });
  if (s != MW_OK) return s;
  if (numeric) { g_last_error = "NaN or Inf in a GMRES residual"; return MW_ENUMERIC; }
  if (noconv) { g_last_error = "GMRES did not reach the tolerance within maxit"; return MW_ENOCONV; }
  return MW_OK;
}

mw_status mw_batch_get_info(mw_batch* b, mw_batch_info* info) {
  return guard([&] {
    check_batch(b);
    MW_CHECK(info != nullptr, MW_EINVAL, "info is NULL");
    std::memset(info, 0, sizeof(*info));
    info->max_cols = b->max_cols;
    for (const auto& s : b->slots) {
      if (s.state == mw_batch::FREE) info->free_cols++;
      if (s.state == mw_batch::ACTIVE) info->active_cols++;
    }
    info->requests = (int32_t)b->reqs.size();
    info->finished = (int32_t)b->done.size();
    info->cycles = b->cycles;
    info->slot_bytes = (int64_t)(b->Bs.bytes + b->Xs.bytes + b->idx.bytes);
    info->work_bytes = b->W.held();
    info->bytes_per_col = gmres_bytes_per_col(b->p, b->o.restart, false);
  });
}

mw_status mw_batch_destroy(mw_batch* b) {
  return guard([&] {
    if (!b) return;
    if (b->p) {
      DeviceGuard dg(b->p->ctx->device);
      (void)hipStreamSynchronize(b->p->stream);
      b->p->live_batches--;
    }
    delete b;
  });
}

}  // extern "C"
