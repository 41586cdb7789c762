// Internal helpers shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mw.h"

namespace mw {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  mw_status code;
  Error(mw_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(mw_status c, const std::string& m) { throw Error(c, m); }

#define MW_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      ::mw::fail(MW_EDEVICE, std::string(#call " failed: ") + hipGetErrorString(e_) +     \
                                 " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

#define MW_CHECK(cond, code, msg)        \
  do {                                   \
    if (!(cond)) ::mw::fail(code, (msg)); \
  } while (0)

#define MW_LAUNCH_CHECK() MW_HIP(hipGetLastError())

// ---------------------------------------------------------------- device memory
// Owning device buffer, released on destruction.  Allocation sizes are tracked
// by the context's byte budget (see Context in api.cpp).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  std::atomic<int64_t>* ledger = nullptr;  // running total of the owning context
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; ledger = o.ledger;
      o.p = nullptr; o.bytes = 0; o.ledger = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      (void)hipFree(p);
      if (ledger) ledger->fetch_sub((int64_t)bytes);
    }
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// ---------------------------------------------------------------- complex
// Complex values are (re, im) pairs: float2 for the FP32 path, double2 for FP64.
template <class R> struct cplx;
template <> struct cplx<float> { using t = float2; };
template <> struct cplx<double> { using t = double2; };

template <class C> __host__ __device__ inline C cmk(decltype(C{}.x) r, decltype(C{}.x) i) {
  C z; z.x = r; z.y = i; return z;
}
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// 1 / z by scaling (Smith's method is not needed at these magnitudes; scale
// by the larger component to avoid overflow of |z|^2)
__host__ __device__ inline double2 cinv(double2 z) {
  double s = fabs(z.x) > fabs(z.y) ? fabs(z.x) : fabs(z.y);
  double xr = z.x / s, xi = z.y / s;
  double d = (xr * xr + xi * xi) * s;
  return make_double2(xr / d, -xi / d);
}
__host__ __device__ inline float2 cinv(float2 z) {
  float s = fabsf(z.x) > fabsf(z.y) ? fabsf(z.x) : fabsf(z.y);
  float xr = z.x / s, xi = z.y / s;
  float d = (xr * xr + xi * xi) * s;
  return make_float2(xr / d, -xi / d);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ---------------------------------------------------------------- host mesh data
// Edge topology of the mesh (built on the host, mirrored to the device).
struct Topology {
  int32_t nv = 0, nt = 0, nbf = 0;
  std::vector<double> xyz;          // [nv*3]
  std::vector<int32_t> tet;         // [nt*4] ascending
  std::vector<int64_t> edges;       // [ne*2] (lo, hi), lexicographic
  std::vector<int32_t> t2e;         // [nt*6]
  std::vector<int32_t> bface;       // [nbf*3] ascending
  std::vector<int32_t> btag;        // [nbf]
  std::vector<int32_t> bf_owner;    // [nbf] owning tetrahedron
  std::vector<int32_t> bf2e;        // [nbf*3]
  std::vector<uint8_t> pec;         // [ne]
  std::vector<int32_t> dof;         // [ne] -> free index or -1
  std::vector<int32_t> free_edge;   // [n]  -> edge id
  // CSR pattern of A on free dofs
  std::vector<int64_t> row_ptr;     // [n+1]
  std::vector<int32_t> col;         // [nnz]
  // per-row contributions for the deterministic gather of A's values
  std::vector<int64_t> rt_ptr;      // [n+1]
  std::vector<int32_t> rt;          // tet*6 + p
  std::vector<int64_t> rf_ptr;      // [n+1]
  std::vector<int32_t> rf;          // bface*3 + p (non-PEC boundary faces)
  int64_t ne() const { return (int64_t)edges.size() / 2; }
  int64_t n() const { return (int64_t)free_edge.size(); }
};

void build_topology(const mw_mesh& m, Topology& T);

// Overlapping decomposition (host side of the ORAS preconditioner).
struct Decomposition {
  int32_t nsub = 0, delta = 1;
  std::vector<int32_t> n_loc;       // [nsub] n_i
  std::vector<int32_t> n_pad;       // [nsub] n_i rounded up to the block size
  std::vector<int32_t> n_lead;      // [nsub] leading local unknowns with D = 0
  // [nsub * fenv_stride] per 32-row group of B_i: first column of its rows'
  // envelope (symmetric pattern: also the first row of its columns' envelope)
  std::vector<int32_t> fenv;
  // same layout: one past the last column whose envelope reaches the group's rows
  std::vector<int32_t> fenv_hi;
  int32_t fenv_stride = 0;
  std::vector<int64_t> loc_off;     // [nsub+1] row offset of subdomain i in local vectors
  std::vector<int64_t> fac_off;     // [nsub+1] element offset of subdomain i's dense matrix
  // factor storage per 64-row block k (entry i * bstride + k): offset of the
  // block's first row within the subdomain's storage, first stored column,
  // row width; dense (all n_pad columns) and banded (the block's structural
  // envelope, 64-aligned, reaching at least 64 columns past its diagonal
  // block; what a factorisation without interchanges fills)
  int32_t bstride = 0;
  std::vector<int64_t> boff_dense, boff_band, fac_off_band;
  std::vector<int32_t> blo_dense, blo_band, bw_dense, bw_band;
  std::vector<int32_t> sub_dof;     // [sum n_pad] global dof of each local row (-1 padding);
                                    // reverse Cuthill-McKee order within each subdomain
  std::vector<double> D;            // [sum n_pad] partition-of-unity weight (0 padding)
  // prolongation: copies of every global dof (CSR over dofs, deterministic order)
  std::vector<int64_t> cp_ptr;      // [n+1]
  std::vector<int64_t> cp_row;      // local row index (into sum n_pad)
  // local matrix assembly lists, per subdomain contiguous
  // tets of T_i^delta with the local index of their 6 edges (-1 if PEC)
  std::vector<int64_t> lt_off;      // [nsub+1]
  std::vector<int32_t> lt_tet;      // global tet id
  std::vector<int32_t> lt_loc;      // [6 per entry]
  // faces carrying a boundary/transmission term: 3 sorted vertices, owner tet,
  // kind (-1 interface, else global boundary face index), 3 local dofs
  std::vector<int64_t> lf_off;      // [nsub+1]
  std::vector<int32_t> lf_vert;     // [3 per entry]
  std::vector<int32_t> lf_owner;
  std::vector<int32_t> lf_kind;
  std::vector<int32_t> lf_loc;      // [3 per entry]
  // per local row: contributions (entry*6+p into lt_*, entry*3+p into lf_*)
  std::vector<int64_t> rtl_ptr;     // [sum n_pad + 1]
  std::vector<int32_t> rtl;         // local-tet entry * 6 + p (entry index relative to lt_off[i])
  std::vector<int64_t> rfl_ptr;     // [sum n_pad + 1]
  std::vector<int32_t> rfl;         // local-face entry * 3 + p (relative to lf_off[i])
  int64_t sum_pad() const { return loc_off.empty() ? 0 : loc_off.back(); }
};

void build_decomposition(const Topology& T, const int32_t* tet_part, int32_t nsub, int32_t delta,
                         int32_t block, Decomposition& D);

// Internal non-overlapping partition: recursive coordinate bisection of the
// tetrahedron centroids into nsub parts of floor(nt/nsub) or one more.
void partition_rcb(const Topology& T, int32_t nsub, std::vector<int32_t>& part);

}  // namespace mw
