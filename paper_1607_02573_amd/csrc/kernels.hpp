// Device data views and kernel launchers of the library (all HIP, gfx950).
#pragma once

#include "common.hpp"

namespace mw {

// kernel families timed by ktimer.cpp
enum KFamily { KF_TRSM_GEMM, KF_TRSM_LEAF, KF_LU_GEMM, KF_LU_PANEL, KF_LU_OTHER, KF_SPMM, KF_CGS_DOTS,
               KF_CGS_UPDATE, KF_RESTRICT, KF_PROLONG, KF_VECTOR, KF_BGS_DOTS, KF_BGS_UPDATE, KF_COARSE, KF_COUNT };
bool kt_enabled();
void kt_begin(int family, hipStream_t st);
void kt_end(int family, hipStream_t st, double flops, double bytes);

// Mesh, operator pattern and per-row assembly lists on the device.
struct DeviceMesh {
  int64_t nv = 0, nt = 0, n = 0, nbf = 0, nnz = 0;
  const double* xyz = nullptr;
  const int32_t* tet = nullptr;
  const int32_t* t2e = nullptr;
  const int32_t* dof = nullptr;
  const int32_t* bface = nullptr;
  const int32_t* bf2e = nullptr;
  const double2* fbeta = nullptr;   // i*beta coefficient source per boundary face (beta)
  const int64_t* row_ptr = nullptr;
  const int32_t* col = nullptr;
  const int32_t* rorder = nullptr;   // rows of A in Z-order of their edge midpoints (SpMM locality)
  // A in sliced ELLPACK (SELL-64-512) for products with 1 or 2 columns: the
  // rows in Z order, sorted by length within windows of 512, 64 per slice;
  // slice s holds its rows' nonzeros column-major (entry k of the slice's
  // lane l at sl_off[s] + 64 k + l), each row's in CSR order, padding col -1.
  int64_t sl_slots = 0;                  // 64 x number of slices
  const int32_t* sl_row = nullptr;       // [sl_slots] row of each lane (-1 padding)
  const int64_t* sl_off = nullptr;       // [slices + 1]
  const int32_t* sl_col = nullptr;       // [sl_off[slices]]
  const double2* sl_val = nullptr;       // [sl_off[slices]] values, refreshed with val
  const double2* csr_val = nullptr;      // the CSR values sl_val mirrors
  const int64_t* rt_ptr = nullptr;
  const int32_t* rt = nullptr;
  const int64_t* rf_ptr = nullptr;
  const int32_t* rf = nullptr;
};

struct PortDev {
  double2 beta;
  double radius, theta, width;
  double pol[3];
};

// Sparse port projections: for port k, entries [port_ptr[k], port_ptr[k+1])
// hold distinct unknowns ent_dof[] with values pval[]; each entry sums the
// (face, local edge) contributions ent_fq[ent_ptr[e] .. ent_ptr[e+1]).
struct DevicePorts {
  int nports = 0;
  int64_t nent = 0;
  const PortDev* ports = nullptr;
  const int64_t* port_ptr = nullptr;
  const int32_t* ent_dof = nullptr;
  const int32_t* ent_port = nullptr;
  const int64_t* ent_ptr = nullptr;
  const int32_t* ent_fq = nullptr;
  const int64_t* pf_ptr = nullptr;   // faces of each port
  const int32_t* pf = nullptr;
  double* pval = nullptr;
  double* nu = nullptr;
};

struct DeviceDecomp {
  int nsub = 0;
  int64_t n_glob = 0;           // global unknowns (restriction traffic)
  int max_pad = 0;
  int64_t sum_pad = 0;
  const int64_t* fac_off = nullptr;
  const int64_t* loc_off = nullptr;
  const int32_t* n_loc = nullptr;
  const int32_t* n_pad = nullptr;
  const int64_t* lt_off = nullptr;
  const int32_t* lt_tet = nullptr;
  const int32_t* lt_loc = nullptr;
  const int64_t* lf_off = nullptr;
  const int32_t* lf_vert = nullptr;
  const int32_t* lf_owner = nullptr;
  const int32_t* lf_kind = nullptr;
  const int32_t* lf_loc = nullptr;
  const int64_t* rtl_ptr = nullptr;
  const int32_t* rtl = nullptr;
  const int64_t* rfl_ptr = nullptr;
  const int32_t* rfl = nullptr;
  const int32_t* sub_dof = nullptr;
  const double* D = nullptr;
  const int64_t* cp_ptr = nullptr;
  const int64_t* cp_row = nullptr;
  int32_t* ipiv = nullptr;      // [sum_pad] pivot row of each column (subdomain-relative)
  int32_t* ridx = nullptr;      // [sum_pad] restriction gather index after pivoting (-1 padding)
  int32_t* info = nullptr;      // [nsub] first (near-)zero-pivot column + 1, 0 if none
  double* amax = nullptr;       // [nsub] max |re|+|im| of B_i
  const int32_t* h_n_loc = nullptr;  // host copy of n_loc (launch accounting)
  const int32_t* row_lo = nullptr;   // [nsub] first row (multiple of 64) the backward solve must produce
  const int32_t* h_row_lo = nullptr; // host copy
  const int32_t* order = nullptr;    // [nsub] subdomains by decreasing n_pad (block-row solves)
  bool rows = false;                 // factors in block-row form (scaled off-diagonal rows)
  // envelope of the factors per 32-row group g of every subdomain (entry
  // i * env_stride + g, env_stride = max_pad / 32), written by the
  // factorisation: x = first column left of the group's 64-wide diagonal
  // block holding a nonzero of L (rounded down to 8), y = one past the last
  // column right of it holding a nonzero of U (rounded up to 8)
  const int32_t* fenv = nullptr;     // [nsub * fenv_stride] structural envelope of B_i per 32-row group
  const int32_t* h_fenv = nullptr;   // host copy
  const int32_t* fenv_hi = nullptr;  // [nsub * fenv_stride] one past the last column of B_i reaching the group
  int fenv_stride = 0;
  int2* env = nullptr;
  const int2* h_env = nullptr;       // host copy (launch accounting)
  int env_stride = 0;
  // storage of the factors, per 64-row block k of subdomain i (entry
  // i * bstride + k): element offset of the block's first row within the
  // subdomain's storage, first stored column, row width.  Element (r, c) is
  // at F + fac_off[i] + boff + (r mod 64) * bw + c - blo; only columns
  // [blo, blo + bw) exist.  Dense storage: boff = 64 k n_pad, blo = 0,
  // bw = n_pad (LU with interchanges); banded storage holds each block's
  // structural envelope (L D L^T without interchanges fills nothing outside).
  const int64_t* boff = nullptr;
  const int32_t* blo = nullptr;
  const int32_t* bw = nullptr;
  int bstride = 0;
};

// Row r of a subdomain's factors: P such that P[c] is element (r, c) (the
// block tables of that subdomain).
template <class T>
__device__ inline T* frow(T* Fi, const int64_t* boff, const int32_t* blo, const int32_t* bw, int r) {
  const int k = r >> 6;
  return Fi + boff[k] + (int64_t)(r & 63) * bw[k] - blo[k];
}

// Coarse space of the two-level preconditioner (coarse.hip): three coarse
// unknowns per subdomain (the weighted interpolants of the constant fields).
constexpr int kCoarseMaxNb = 256;   // most neighbours a subdomain may have in E
struct DeviceCoarse {
  int nsub = 0;
  int max_nb = 0;                      // longest neighbour list
  const double* tvec = nullptr;        // [n*3] edge vector x_hi - x_lo of every unknown
  const int32_t* row_sub = nullptr;    // [sum_pad] subdomain of every local row
  const int64_t* nb_ptr = nullptr;     // [nsub+1] neighbour lists of E's block rows
  const int32_t* nb = nullptr;         // ascending subdomain ids, the subdomain itself included
};

// ---- assembly (assemble.hip)
void launch_element_matrices(const DeviceMesh& m, const double2* eps, double k0, double2* E, hipStream_t st);
void launch_gather_csr(const DeviceMesh& m, const double2* E, double2* val, hipStream_t st);
template <class C>
void launch_fill_local(const DeviceMesh& m, const DeviceDecomp& d, const double2* E, const double2* eps,
                       double k0, C* F, hipStream_t st);
void launch_port_setup(const DeviceMesh& m, const DevicePorts& P, hipStream_t st);
void launch_rhs_ports(const DevicePorts& P, int ntx, const int32_t* tx_dev, double2* B, int64_t ldb,
                      hipStream_t st);
void launch_locate(const DeviceMesh& m, const double* pts, int np, int* found, hipStream_t st);
void launch_rhs_dipoles(const DeviceMesh& m, const double* pts, const double* dirs, const int* found, int np,
                        double2* B, int64_t ldb, hipStream_t st);
void launch_s_matrix(const DevicePorts& P, int nrx, const int32_t* rx_dev, int ntx, const double2* U,
                     int64_t ldu, double2* S, hipStream_t st);
void launch_adjoint_rhs(const DevicePorts& P, int nrx, const int32_t* rx_dev, int ntx, const double2* gS,
                        double2* L, int64_t ldl, hipStream_t st);
void launch_gradient(const DeviceMesh& m, const double2* U, const double2* F, int64_t ld, int ncol, double k0,
                     double2* grad, hipStream_t st);

void launch_max_imag(const double2* eps, int64_t nt, double* out, hipStream_t st);
// eps_r linear on every tetrahedron (vertex values): element matrices and tet means;
// vertex gradient (G: nt x 4 scratch; vt_ptr/vt: (t*4 + slot) entries of each vertex)
void launch_element_matrices_p1(const DeviceMesh& m, const double2* eps_v, double k0, double2* E, double2* eps_t,
                                hipStream_t st);
void launch_gradient_p1(const DeviceMesh& m, const double2* U, const double2* F, int64_t ld, int ncol, double k0,
                        const int64_t* vt_ptr, const int32_t* vt, double2* G, double2* grad, hipStream_t st);

// ---- dense subdomain algebra (dense.hip)
// Factor every B_i in place: P_i B_i = L_i U_i (partial pivoting, unit L), or
// with sym B_i = L_i U_i, U_i = D_i L_i^T (no interchanges), then build the
// pivoted restriction index.  C = float2 or double2.
template <class C>
void lu_factor_batched(const DeviceDecomp& d, C* F, hipStream_t st, bool sym);
// Y_i = U_i^-1 L_i^-1 Y_i in place on the local multi-vector (rows
// loc_off[i] .. +n_pad[i], ncols columns, leading dimension ld).
template <class C>
void lu_solve_batched(const DeviceDecomp& d, const C* F, C* Y, int ncols, int64_t ld, hipStream_t st);

// ---- Krylov and vector kernels (krylov.hip)
// values of the sliced ELLPACK copy of A: sl_val[p] = val[sl_idx[p]] (0 for padding)
void launch_sell_values(int64_t total, const int32_t* sl_idx, const double2* val, double2* sl_val, hipStream_t st);
// X complex FP64 or complex FP32 (double2 / float2); products and sums FP64
template <class XT>
void launch_spmm(const DeviceMesh& m, const double2* val, const XT* X, int64_t ldx, double2* Y,
                 int64_t ldy, int ncols, const double2* Bsub, int64_t ldb, hipStream_t st);
// vsc (optional, device, ncols): column c of V is taken times vsc[c]
template <class C, class VT = double2>
void launch_restrict(const DeviceDecomp& d, const VT* V, int64_t ldv, int ncols, C* Y, int64_t ldy,
                     hipStream_t st, const double* vsc = nullptr);
// vsc[c] = 1 / sqrt(n2[c]) where n2[c] > 0, else 1 (device, ncols each)
void launch_inv_norms(int ncols, const double* n2, double* vsc, hipStream_t st);
// Z complex FP64, or complex FP32 (summed in FP64, then rounded)
template <class C, class ZT = double2>
void launch_prolong(const DeviceDecomp& d, int64_t n, const C* Y, int64_t ldy, int ncols, ZT* Z,
                    int64_t ldz, hipStream_t st);
// column sums over rows in fixed-size row chunks, then in chunk order
int64_t reduce_chunks(int64_t n);
void launch_colnorm2_partial(const double2* V, int64_t n, int64_t ld, int ncols, double* part, hipStream_t st);
void launch_sum_chunks(const double* part, int64_t nchunk, int64_t width, double* out, hipStream_t st);
// w1sc (optional, device, ncols): w1 = V_{kcount-1} is a candidate stored
// before its normalisation; both are taken times w1sc[c]
template <class B>
void launch_dots_partial(const B* V, int64_t vstride, int kcount, const B* w1, const double2* w2,
                         int64_t n, int64_t ld, int ncols, const int32_t* act, double2* part1, double2* part2,
                         hipStream_t st, const double* w1sc = nullptr);
void launch_sum_chunks_c(const double2* part, int64_t nchunk, int64_t width, double2* out, hipStream_t st);
void launch_dgs_step(int j, int m, bool fin, int ncols, const double2* P1, const double2* P2, const double* beta2,
                     double2* Hraw, double2* H, double* cs, double2* sn, double2* g, double2* hprov, double2* coef,
                     double* nu, double2* e, int32_t* kdim, int32_t* act, double* resid, const double* bnorm,
                     double tol, double2* Rc, hipStream_t st);
void launch_dgs_trial(int j, int m, int ncols, const double2* hprov, const double* beta2, const double* cs,
                      const double2* sn, const double2* g, const int32_t* act, const double* bnorm, double tol,
                      int32_t* done, hipStream_t st);
// vjsc (optional, device, ncols): V_j is a candidate stored before its
// normalisation, taken times vjsc[c]
template <class B>
void launch_dgs_update(B* V, int64_t vstride, int j, const double2* coef, const double* nu, const double2* e,
                       const double2* T, int64_t n, int64_t ld, int ncols, const int32_t* act, double* norm_part,
                       hipStream_t st, const double* vjsc = nullptr);
template <class B>
void launch_scale_cols(B* w, int64_t n, int64_t ld, int ncols, const double* nrm, const int32_t* act,
                       hipStream_t st);
void launch_backsolve(int m, int ncols, const double2* H, const double2* g, const int32_t* kdim, double2* y,
                      hipStream_t st);
void launch_candsolve(int m, int ncols, const double2* Rc, const int32_t* kdim, double2* y, hipStream_t st);
template <class B>
void launch_combine(const B* V, int64_t vstride, int m, const double2* y, const int32_t* kdim,
                    double2* u, int64_t n, int64_t ld, int ncols, hipStream_t st);
void launch_axpy_cols(double2* x, const double2* z, int64_t n, int64_t ld, int ncols, hipStream_t st);
// dst[i] = src[i] widened to complex FP64
void launch_widen(const float2* src, double2* dst, int64_t count, hipStream_t st);
// dst[i] = src[i] rounded to complex FP32
void launch_narrow(const double2* src, float2* dst, int64_t count, hipStream_t st);
template <class B>
void launch_start_cycle(const double2* r, B* v0, int64_t n, int64_t ld, int ncols, const double* rn2,
                        const int32_t* act, hipStream_t st);
void launch_copy_cols(const double2* src, int64_t lds, double2* dst, int64_t ldd, int64_t n, int ncols,
                      hipStream_t st);
void launch_zero(double2* p, int64_t count, hipStream_t st);
// column moves by an index list idx (device [ncols]) over n rows:
// gather dst[:, k] = src[:, idx[k]]; scatter dst[:, idx[k]] = src[:, k];
// scatter of zeros when src is NULL
void launch_gather_cols(const double2* src, int64_t lds, const int32_t* idx, double2* dst, int64_t ldd, int64_t n,
                        int ncols, hipStream_t st);
void launch_scatter_cols(const double2* src, int64_t lds, const int32_t* idx, double2* dst, int64_t ldd, int64_t n,
                         int ncols, hipStream_t st);
void launch_zero_bytes(void* p, int64_t bytes, hipStream_t st);

// block Gram-Schmidt of block GMRES (block.hip): blocks of 32 columns
void bdots_chunks(int64_t n, int nb, int ktot, int64_t* rows_per_ch, int64_t* nch);
void launch_bdots(const double2* V, int64_t vstride, int kv, const double2* E, const double2* Wr, int64_t n,
                  int64_t ld, int ncols, int nb, const int32_t* blk, double2* part, int64_t* nch_out,
                  hipStream_t st);
void launch_bupdate(const double2* V, int64_t vstride, int kv, const int32_t* kvb, int kv_max, const double2* P,
                    int pk_stride, const double2* Rinv, const double2* Win, double2* Out, int64_t n, int64_t ld,
                    int ncols, int nb, const int32_t* blk, hipStream_t st);
// gS = W (S - Sm), J = 1/2 sum W |S - Sm|^2 (W = NULL: weights 1)
void launch_misfit(const double2* S, const double2* Sm, const double* W, int64_t count, double2* gS, double* J,
                   hipStream_t st);

// two-level ORAS (coarse.hip): E = Z^T A Z into F (ldf x ldf, identity on the
// padding), Y = Z^T V (rows 3 nsub .. ldf zero), Q = Z Y
template <class C>
void launch_coarse_matrix(const DeviceMesh& m, const double2* val, const DeviceDecomp& d, const DeviceCoarse& cz,
                          C* F, int ldf, hipStream_t st);
template <class C>
void launch_coarse_restrict(const DeviceDecomp& d, const DeviceCoarse& cz, const double2* V, int64_t ldv, int ncols,
                            C* Y, int64_t ldy, int ldf, hipStream_t st);
template <class C>
void launch_coarse_prolong(const DeviceDecomp& d, const DeviceCoarse& cz, int64_t n, const C* Y, int64_t ldy,
                           int ncols, double2* Q, int64_t ldq, hipStream_t st);

}  // namespace mw
