// Vector kernels of the preconditioned pseudo-block GMRES (paper Section 6:
// right-preconditioned GMRES, stopped on the unpreconditioned residual; the
// right-hand sides keep their own Krylov spaces and only their arithmetic is
// fused).  All multi-vectors are n x ncols row-major (column index
// contiguous).  Every reduction sums fixed row chunks in a fixed order, so a
// column's result does not depend on how many other columns are present
// (a column solved alone or in a batch gives bitwise the same numbers).
#include "kernels.hpp"

namespace mw {

constexpr int RCHUNK = 2048;   // rows per reduction chunk

int64_t reduce_chunks(int64_t n) { return ceil_div(n, RCHUNK); }

// Multi-vector elements: complex FP64 (double2) or complex FP32 (float2: the
// Krylov basis and the preconditioned vectors of the mixed-precision GMRES);
// every product and sum below is FP64.
__device__ inline double2 bload(const double2& v) { return v; }
__device__ inline double2 bload(const float2& v) { return make_double2(v.x, v.y); }
template <class B> __device__ inline B bstore(double2 v);
template <> __device__ inline double2 bstore<double2>(double2 v) { return v; }
template <> __device__ inline float2 bstore<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }

// acc += a x as four fused multiply-adds, in this order: every form of the
// product A X uses it, so a column's sums are bitwise the same in every form
__device__ inline void cmac(double2& acc, const double2& a, const double2& x) {
  acc.x = fma(a.x, x.x, acc.x);
  acc.x = fma(-a.y, x.y, acc.x);
  acc.y = fma(a.x, x.y, acc.y);
  acc.y = fma(a.y, x.x, acc.y);
}

// ---------------------------------------------------------------- K1 / K12
// Y = A X  (Bsub == nullptr)  or  Y = Bsub - A X, CSR complex128.
// TPR threads per row; each lane walks columns lane, lane+TPR, ...
template <int TPR, class XT>
__global__ void __launch_bounds__(256) k_spmm(int64_t n, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const double2* __restrict__ val,
                                              const XT* __restrict__ X, int64_t ldx, double2* __restrict__ Y,
                                              int64_t ldy, int ncols, const double2* __restrict__ Bs, int64_t ldb) {
  int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / TPR;
  int lane = threadIdx.x % TPR;
  if (r >= n) return;
  int64_t b = row_ptr[r], e = row_ptr[r + 1];
  for (int c0 = 0; c0 < ncols; c0 += TPR) {
    int c = c0 + lane;
    if (c >= ncols) break;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t k = b; k < e; ++k) {
      cmac(acc, val[k], bload(X[(int64_t)col[k] * ldx + c]));
    }
    if (Bs) {
      double2 bb = Bs[r * ldb + c];
      acc = make_double2(bb.x - acc.x, bb.y - acc.y);
    }
    Y[r * ldy + c] = acc;
  }
}

// Wide form for many columns: one wave per row; the row's (column, value)
// pairs are loaded once, 64 at a time (one per lane), and broadcast with
// readlane, so the inner loop issues only the X loads of CPL column groups
// per nonzero.  Per (row, column) the products are summed in the order of
// the row's nonzeros, as in k_spmm.
__device__ inline double bcast(double v, int t) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), t);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), t);
  return __hiloint2double(hi, lo);
}

// nonzeros per gather pass of the wide SpMM forms
template <class XT> constexpr int SPMM_U = sizeof(XT) == 8 ? 4 : 2;

template <int CPL, class XT>
__global__ void __launch_bounds__(256) k_spmm_w(int64_t n, const int64_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col, const double2* __restrict__ val,
                                                const XT* __restrict__ X, int64_t ldx, double2* __restrict__ Y,
                                                int64_t ldy, int ncols, const double2* __restrict__ Bs, int64_t ldb) {
  // workgroups are dealt to the 8 XCDs round-robin: remap so that each XCD
  // takes one contiguous eighth of the rows, whose X rows overlap in its L2
  const int64_t G = gridDim.x;
  const int64_t blk = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int64_t r = (blk * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  const int64_t b = row_ptr[r], e = row_ptr[r + 1];
  for (int c0 = 0; c0 < ncols; c0 += 64 * CPL) {
    double2 acc[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) acc[q] = make_double2(0.0, 0.0);
    // columns past ncols read column ncols - 1 and are never stored, so no
    // load sits behind a per-column branch
    int cq[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) cq[q] = min(c0 + lane + 64 * q, ncols - 1);
    for (int64_t kb = b; kb < e; kb += 64) {
      const int cnt = (int)min((int64_t)64, e - kb);
      int mycol = 0;
      double2 myval = make_double2(0.0, 0.0);
      if (lane < cnt) {
        mycol = col[kb + lane];
        myval = val[kb + lane];
      }
      // SPMM_U nonzeros per pass: all their X rows are requested before the
      // first product, so a wave keeps SPMM_U * CPL loads in flight; the
      // passes past cnt read row mycol of a lane >= cnt (0) or of a lane
      // wrapped round, which is in range, and add nothing
      for (int t = 0; t < cnt; t += SPMM_U<XT>) {
        int64_t cc[SPMM_U<XT>];
        double2 a[SPMM_U<XT>];
#pragma unroll
        for (int u = 0; u < SPMM_U<XT>; ++u) {
          const int s = (t + u) & 63;
          const bool ok = t + u < cnt;   // else a = 0, which adds exactly nothing to a finite sum
          cc[u] = __builtin_amdgcn_readlane(mycol, s);
          a[u].x = ok ? bcast(myval.x, s) : 0.0;
          a[u].y = ok ? bcast(myval.y, s) : 0.0;
        }
        XT x[SPMM_U<XT>][CPL];
#pragma unroll
        for (int u = 0; u < SPMM_U<XT>; ++u)
#pragma unroll
          for (int q = 0; q < CPL; ++q) x[u][q] = X[cc[u] * ldx + cq[q]];
#pragma unroll
        for (int u = 0; u < SPMM_U<XT>; ++u)
#pragma unroll
          for (int q = 0; q < CPL; ++q) cmac(acc[q], a[u], bload(x[u][q]));
      }
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = c0 + lane + 64 * q;
      if (c < ncols) {
        double2 o = acc[q];
        if (Bs) {
          double2 bb = Bs[r * ldb + c];
          o = make_double2(bb.x - o.x, bb.y - o.y);
        }
        Y[r * ldy + c] = o;
      }
    }
  }
}

// Half-wave form: 32 lanes per row (two rows per wave), each lane on CPL
// columns c = lane + 32 q; the row's nonzeros are loaded 32 at a time and
// broadcast within the half-wave.  No idle lanes for 32 * CPL columns.
template <int CPL, class XT>
__global__ void __launch_bounds__(256) k_spmm_h(int64_t n, const int64_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col, const double2* __restrict__ val,
                                                const XT* __restrict__ X, int64_t ldx, double2* __restrict__ Y,
                                                int64_t ldy, int ncols, const double2* __restrict__ Bs, int64_t ldb,
                                                const int32_t* __restrict__ rorder) {
  const int64_t G = gridDim.x;
  const int64_t blk = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int64_t rr = (blk * blockDim.x + threadIdx.x) >> 5;
  const int lane = threadIdx.x & 31;
  const bool live = rr < n;
  const int64_t r = (live && rorder) ? rorder[rr] : rr;
  const int64_t b = live ? row_ptr[r] : 0, e = live ? row_ptr[r + 1] : 0;
  double2 acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = make_double2(0.0, 0.0);
  // both half-waves run the same number of passes (shuffles need every lane)
  const int64_t len = e - b;
  const int64_t len_o = __shfl_xor(len, 32);
  const int64_t len_max = len > len_o ? len : len_o;
  int cq[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) cq[q] = min(lane + 32 * q, ncols - 1);
  for (int64_t kb = 0; kb < len_max; kb += 32) {
    const int cnt = (int)min((int64_t)32, len - kb);
    int mycol = 0;
    double2 myval = make_double2(0.0, 0.0);
    if (lane < cnt) {
      mycol = col[b + kb + lane];
      myval = val[b + kb + lane];
    }
    const int cnt_max = (int)min((int64_t)32, len_max - kb);
    // as in k_spmm_w: SPMM_U nonzeros' X rows requested before their products
    for (int t = 0; t < cnt_max; t += SPMM_U<XT>) {
      int64_t cc[SPMM_U<XT>];
      double2 a[SPMM_U<XT>];
#pragma unroll
      for (int u = 0; u < SPMM_U<XT>; ++u) {
        const int s = (t + u) & 31;
        const bool ok = t + u < cnt;   // else a = 0, which adds exactly nothing to a finite sum
        cc[u] = __shfl(mycol, s, 32);
        const double ax = __shfl(myval.x, s, 32), ay = __shfl(myval.y, s, 32);
        a[u].x = ok ? ax : 0.0;
        a[u].y = ok ? ay : 0.0;
      }
      XT x[SPMM_U<XT>][CPL];
#pragma unroll
      for (int u = 0; u < SPMM_U<XT>; ++u)
#pragma unroll
        for (int q = 0; q < CPL; ++q) x[u][q] = X[cc[u] * ldx + cq[q]];
#pragma unroll
      for (int u = 0; u < SPMM_U<XT>; ++u)
#pragma unroll
        for (int q = 0; q < CPL; ++q) cmac(acc[q], a[u], bload(x[u][q]));
    }
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = lane + 32 * q;
    if (c < ncols) {
      double2 o = acc[q];
      if (Bs) {
        double2 bb = Bs[r * ldb + c];
        o = make_double2(bb.x - o.x, bb.y - o.y);
      }
      Y[r * ldy + c] = o;
    }
  }
}

// SELL form for up to NC columns: lane = one row of a 64-row slice, its
// nonzeros in CSR order along the slice (products summed in the same order
// as the CSR kernels, so a column's result does not depend on the form).
template <int NC, class XT>
__global__ void __launch_bounds__(256) k_spmm_sell(int64_t nslots, const int32_t* __restrict__ sl_row,
                                                   const int64_t* __restrict__ sl_off,
                                                   const int32_t* __restrict__ sl_col,
                                                   const double2* __restrict__ sl_val, const XT* __restrict__ X,
                                                   int64_t ldx, double2* __restrict__ Y, int64_t ldy, int ncols,
                                                   const double2* __restrict__ Bs, int64_t ldb) {
  const int64_t slot = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const int32_t r = sl_row[slot];
  if (r < 0) return;
  const int64_t s = slot >> 6;
  const int lane = (int)(slot & 63);
  const int64_t o0 = sl_off[s], w = (sl_off[s + 1] - o0) >> 6;
  double2 acc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int64_t k = 0; k < w; ++k) {
    const int64_t pos = o0 + 64 * k + lane;
    const int32_t c = sl_col[pos];
    if (c < 0) break;   // the row's entries come first, padding after
    const double2 a = sl_val[pos];
    const XT* xr = X + (int64_t)c * ldx;
#pragma unroll
    for (int q = 0; q < NC; ++q)
      if (q < ncols) {
        cmac(acc[q], a, bload(xr[q]));
      }
  }
#pragma unroll
  for (int q = 0; q < NC; ++q)
    if (q < ncols) {
      double2 o = acc[q];
      if (Bs) {
        const double2 bb = Bs[(int64_t)r * ldb + q];
        o = make_double2(bb.x - o.x, bb.y - o.y);
      }
      Y[(int64_t)r * ldy + q] = o;
    }
}

__global__ void k_sell_values(int64_t total, const int32_t* __restrict__ sl_idx, const double2* __restrict__ val,
                              double2* __restrict__ sl_val) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= total) return;
  const int32_t i = sl_idx[p];
  sl_val[p] = i >= 0 ? val[i] : make_double2(0.0, 0.0);
}
void launch_sell_values(int64_t total, const int32_t* sl_idx, const double2* val, double2* sl_val, hipStream_t st) {
  if (total <= 0) return;
  k_sell_values<<<(unsigned)ceil_div(total, 256), 256, 0, st>>>(total, sl_idx, val, sl_val);
  MW_LAUNCH_CHECK();
}

template <class XT>
void launch_spmm(const DeviceMesh& m, const double2* val, const XT* X, int64_t ldx, double2* Y, int64_t ldy,
                 int ncols, const double2* Bsub, int64_t ldb, hipStream_t st) {
  int64_t n = m.n;
  kt_begin(KF_SPMM, st);
  if (ncols <= 2 && m.sl_val && val == m.csr_val) {
    // one or two columns: one lane per row, the slice's nonzeros read
    // coalesced (the CSR form gives a lane a row whose entries lie apart):
    // 181 against 790 us at one column, 308 against 754 at two on the
    // 1 GHz chamber; from four columns on the CSR forms are faster
#define MW_SELL(NC)                                                                                              \
  k_spmm_sell<NC, XT><<<(unsigned)ceil_div(m.sl_slots, 256), 256, 0, st>>>(m.sl_slots, m.sl_row, m.sl_off, m.sl_col, \
                                                                          m.sl_val, X, ldx, Y, ldy, ncols, Bsub, ldb)
    if (ncols == 1) MW_SELL(1);
    else MW_SELL(2);
#undef MW_SELL
    MW_LAUNCH_CHECK();
    if (kt_enabled())
      kt_end(KF_SPMM, st, 8.0 * m.nnz * ncols,
             (double)m.nnz * 20 + n * 4.0 + n * (double)ncols * (sizeof(XT) + 16.0 * (Bsub ? 2 : 1)));
    return;
  }
#define MW_SPMM(T)                                                                                      \
  k_spmm<T, XT><<<(unsigned)ceil_div(n * T, 256), 256, 0, st>>>(n, m.row_ptr, m.col, val, X, ldx, Y, ldy, \
                                                            ncols, Bsub, ldb)
#define MW_SPMM_W(Q)                                                                                  \
  k_spmm_w<Q, XT><<<(unsigned)round_up(ceil_div(n * 64, 256), 8), 256, 0, st>>>(n, m.row_ptr, m.col, val, X, \
                                                                           ldx, Y, ldy, ncols, Bsub, ldb)
  if (ncols <= 1) MW_SPMM(1);
  else if (ncols <= 2) MW_SPMM(2);
  else if (ncols <= 4) MW_SPMM(4);
  else if (ncols <= 8) MW_SPMM(8);
  else if (ncols <= 16) MW_SPMM(16);
  else if (ncols <= 32)
    // half a wave per row, rows in Z order: 1.31 ms against 1.66 ms for one
    // thread group per row in natural order (32 columns, 1 GHz chamber)
    k_spmm_h<1, XT><<<(unsigned)round_up(ceil_div(n * 32, 256), 8), 256, 0, st>>>(n, m.row_ptr, m.col, val, X, ldx, Y,
                                                                              ldy, ncols, Bsub, ldb, m.rorder);
  else if (ncols <= 64) MW_SPMM_W(1);
  else if (ncols <= 128) MW_SPMM_W(2);
  else if (ncols <= 160)
    k_spmm_h<5, XT><<<(unsigned)round_up(ceil_div(n * 32, 256), 8), 256, 0, st>>>(n, m.row_ptr, m.col, val, X, ldx, Y,
                                                                              ldy, ncols, Bsub, ldb, m.rorder);
  else MW_SPMM_W(3);
#undef MW_SPMM
#undef MW_SPMM_W
  MW_LAUNCH_CHECK();
  if (kt_enabled())
    kt_end(KF_SPMM, st, 8.0 * m.nnz * ncols,
           (double)m.nnz * 20 + (n + 1) * 8.0 + n * (double)ncols * (sizeof(XT) + 16.0 * (Bsub ? 2 : 1)));
}
template void launch_spmm<double2>(const DeviceMesh&, const double2*, const double2*, int64_t, double2*, int64_t, int,
                                   const double2*, int64_t, hipStream_t);
template void launch_spmm<float2>(const DeviceMesh&, const double2*, const float2*, int64_t, double2*, int64_t, int,
                                  const double2*, int64_t, hipStream_t);

// ---------------------------------------------------------------- K4 / K5
// Per-column factors of a GMRES candidate stored before its normalisation:
// vsc[c] = 1 / sqrt(n2[c]) where n2[c] > 0, else 1 (the candidate's readers
// take column c times vsc[c])
__global__ void k_inv_norms(int ncols, const double* __restrict__ n2, double* __restrict__ vsc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const double s2 = n2[c];
  vsc[c] = s2 > 0.0 ? 1.0 / sqrt(s2) : 1.0;
}
void launch_inv_norms(int ncols, const double* n2, double* vsc, hipStream_t st) {
  k_inv_norms<<<(unsigned)ceil_div(ncols, 64), 64, 0, st>>>(ncols, n2, vsc);
  MW_LAUNCH_CHECK();
}
__device__ inline double col_scale(const double* __restrict__ vsc, int c) { return vsc ? vsc[c] : 1.0; }

// restriction: Y[l][c] = V[ridx[l]][c] (cast; times vsc[c] when vsc is
// given), zero on padding rows
template <class C, class VT>
__global__ void k_restrict(int64_t nloc, const int32_t* __restrict__ ridx, const VT* __restrict__ V,
                           int64_t ldv, int ncols, C* __restrict__ Y, int64_t ldy, const double* __restrict__ vsc) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t l = id / ncols;
  int c = (int)(id % ncols);
  if (l >= nloc) return;
  int32_t g = ridx[l];
  C y;
  y.x = 0; y.y = 0;
  if (g >= 0) {
    VT v = V[(int64_t)g * ldv + c];
    if (vsc) {
      const double sc = col_scale(vsc, c);
      y.x = (double)v.x * sc; y.y = (double)v.y * sc;
    } else {
      y.x = v.x; y.y = v.y;
    }
  }
  Y[l * ldy + c] = y;
}

// the same for an even number of columns, two adjacent columns per thread
template <class C, class VT>
__global__ void k_restrict2(int64_t nloc, const int32_t* __restrict__ ridx, const VT* __restrict__ V,
                            int64_t ldv, int npairs, C* __restrict__ Y, int64_t ldy, const double* __restrict__ vsc) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t l = id / npairs;
  int c = 2 * (int)(id % npairs);
  if (l >= nloc) return;
  int32_t g = ridx[l];
  C y0, y1;
  y0.x = 0; y0.y = 0; y1.x = 0; y1.y = 0;
  if (g >= 0) {
    VT v0 = V[(int64_t)g * ldv + c], v1 = V[(int64_t)g * ldv + c + 1];
    if (vsc) {
      const double s0 = col_scale(vsc, c), s1 = col_scale(vsc, c + 1);
      y0.x = (double)v0.x * s0; y0.y = (double)v0.y * s0;
      y1.x = (double)v1.x * s1; y1.y = (double)v1.y * s1;
    } else {
      y0.x = v0.x; y0.y = v0.y;
      y1.x = v1.x; y1.y = v1.y;
    }
  }
  Y[l * ldy + c] = y0;
  Y[l * ldy + c + 1] = y1;
}

template <class C, class VT>
void launch_restrict(const DeviceDecomp& d, const VT* V, int64_t ldv, int ncols, C* Y, int64_t ldy,
                     hipStream_t st, const double* vsc) {
  if (d.sum_pad <= 0 || ncols <= 0) return;
  kt_begin(KF_RESTRICT, st);
  if (ncols % 2 == 0) {
    int64_t tot = d.sum_pad * (ncols / 2);
    k_restrict2<C, VT><<<(unsigned)ceil_div(tot, 256), 256, 0, st>>>(d.sum_pad, d.ridx, V, ldv, ncols / 2, Y, ldy,
                                                                     vsc);
  } else {
    int64_t tot = d.sum_pad * ncols;
    k_restrict<C, VT><<<(unsigned)ceil_div(tot, 256), 256, 0, st>>>(d.sum_pad, d.ridx, V, ldv, ncols, Y, ldy, vsc);
  }
  MW_LAUNCH_CHECK();
  if (kt_enabled()) {
    double sl = 0;
    for (int i = 0; i < d.nsub; ++i) sl += d.h_n_loc[i];
    // algorithmic bytes: every global row read once (n x 16 per column; the
    // copies of a row shared by several subdomains come from L2), the gather
    // index, and every local row written
    kt_end(KF_RESTRICT, st, 0.0,
           sl * 4 + (double)d.n_glob * ncols * (double)sizeof(VT) + sl * ncols * (double)sizeof(C));
  }
}

// weighted prolongation: Z[g][c] = sum over the copies of g of D * Y (FP64 sum,
// ascending subdomain order)
template <class C, class ZT>
__global__ void k_prolong(int64_t n, const int64_t* __restrict__ cp_ptr, const int64_t* __restrict__ cp_row,
                          const double* __restrict__ D, const C* __restrict__ Y, int64_t ldy, int ncols,
                          ZT* __restrict__ Z, int64_t ldz) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t g = id / ncols;
  int c = (int)(id % ncols);
  if (g >= n) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t k = cp_ptr[g]; k < cp_ptr[g + 1]; ++k) {
    int64_t r = cp_row[k];
    C y = Y[r * ldy + c];
    double w = D[r];
    acc.x += w * (double)y.x;
    acc.y += w * (double)y.y;
  }
  Z[g * ldz + c] = bstore<ZT>(acc);
}

// the same for an even number of columns, two adjacent columns per thread
// (each column summed exactly as above)
template <class C, class ZT>
__global__ void k_prolong2(int64_t n, const int64_t* __restrict__ cp_ptr, const int64_t* __restrict__ cp_row,
                           const double* __restrict__ D, const C* __restrict__ Y, int64_t ldy, int npairs,
                           ZT* __restrict__ Z, int64_t ldz) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t g = id / npairs;
  int c = 2 * (int)(id % npairs);
  if (g >= n) return;
  double2 a0 = make_double2(0.0, 0.0), a1 = make_double2(0.0, 0.0);
  for (int64_t k = cp_ptr[g]; k < cp_ptr[g + 1]; ++k) {
    int64_t r = cp_row[k];
    C y0 = Y[r * ldy + c], y1 = Y[r * ldy + c + 1];
    double w = D[r];
    a0.x += w * (double)y0.x;
    a0.y += w * (double)y0.y;
    a1.x += w * (double)y1.x;
    a1.y += w * (double)y1.y;
  }
  Z[g * ldz + c] = bstore<ZT>(a0);
  Z[g * ldz + c + 1] = bstore<ZT>(a1);
}

template <class C, class ZT>
void launch_prolong(const DeviceDecomp& d, int64_t n, const C* Y, int64_t ldy, int ncols, ZT* Z, int64_t ldz,
                    hipStream_t st) {
  if (n <= 0 || ncols <= 0) return;
  kt_begin(KF_PROLONG, st);
  if (ncols % 2 == 0) {
    int64_t tot = n * (ncols / 2);
    k_prolong2<C, ZT><<<(unsigned)ceil_div(tot, 256), 256, 0, st>>>(n, d.cp_ptr, d.cp_row, d.D, Y, ldy, ncols / 2, Z,
                                                                ldz);
  } else {
    int64_t tot = n * ncols;
    k_prolong<C, ZT><<<(unsigned)ceil_div(tot, 256), 256, 0, st>>>(n, d.cp_ptr, d.cp_row, d.D, Y, ldy, ncols, Z, ldz);
  }
  MW_LAUNCH_CHECK();
  if (kt_enabled()) {
    double sl = 0;
    for (int i = 0; i < d.nsub; ++i) sl += d.h_n_loc[i];
    kt_end(KF_PROLONG, st, 4.0 * sl * ncols,
           sl * (16.0 + ncols * sizeof(C)) + (n + 1) * 8.0 + n * ncols * (double)sizeof(ZT));
  }
}

template void launch_restrict<float2, double2>(const DeviceDecomp&, const double2*, int64_t, int, float2*, int64_t,
                                               hipStream_t, const double*);
template void launch_restrict<float2, float2>(const DeviceDecomp&, const float2*, int64_t, int, float2*, int64_t,
                                              hipStream_t, const double*);
template void launch_restrict<double2, double2>(const DeviceDecomp&, const double2*, int64_t, int, double2*,
                                                int64_t, hipStream_t, const double*);
template void launch_prolong<float2, double2>(const DeviceDecomp&, int64_t, const float2*, int64_t, int, double2*,
                                              int64_t, hipStream_t);
template void launch_prolong<float2, float2>(const DeviceDecomp&, int64_t, const float2*, int64_t, int, float2*,
                                             int64_t, hipStream_t);
template void launch_prolong<double2, double2>(const DeviceDecomp&, int64_t, const double2*, int64_t, int, double2*,
                                               int64_t, hipStream_t);

// ---------------------------------------------------------------- reductions
// Workgroup (chunk, column tile of 64): thread (column lane, row lane of 4)
// accumulates rows rl, rl+4, ... of the chunk; the 4 row lanes are combined
// in LDS in a fixed order.
__global__ void __launch_bounds__(256) k_colnorm2_partial(const double2* __restrict__ V, int64_t n, int64_t ld,
                                                          int ncols, double* __restrict__ part) {
  __shared__ double red[4][64];
  int chunk = blockIdx.x;
  int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
  int c = blockIdx.y * 64 + cl;
  int64_t r0 = (int64_t)chunk * RCHUNK, r1 = min(n, r0 + RCHUNK);
  double acc = 0.0;
  if (c < ncols)
    for (int64_t r = r0 + rl; r < r1; r += 4) {
      double2 v = V[r * ld + c];
      acc += v.x * v.x + v.y * v.y;
    }
  red[rl][cl] = acc;
  __syncthreads();
  if (rl == 0 && c < ncols) part[(int64_t)chunk * ncols + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

void launch_colnorm2_partial(const double2* V, int64_t n, int64_t ld, int ncols, double* part, hipStream_t st) {
  dim3 g((unsigned)reduce_chunks(n), (unsigned)ceil_div(ncols, 64));
  k_colnorm2_partial<<<g, 256, 0, st>>>(V, n, ld, ncols, part);
  MW_LAUNCH_CHECK();
}

__global__ void k_sum_chunks(const double* __restrict__ part, int64_t nchunk, int64_t width, double* __restrict__ out) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= width) return;
  double acc = 0.0;
  for (int64_t k = 0; k < nchunk; ++k) acc += part[k * width + c];
  out[c] = acc;
}
void launch_sum_chunks(const double* part, int64_t nchunk, int64_t width, double* out, hipStream_t st) {
  k_sum_chunks<<<(unsigned)ceil_div(width, 128), 128, 0, st>>>(part, nchunk, width, out);
  MW_LAUNCH_CHECK();
}
__global__ void k_sum_chunks_c(const double2* __restrict__ part, int64_t nchunk, int64_t width,
                               double2* __restrict__ out) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= width) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t k = 0; k < nchunk; ++k) acc = cadd(acc, part[k * width + c]);
  out[c] = acc;
}
void launch_sum_chunks_c(const double2* part, int64_t nchunk, int64_t width, double2* out, hipStream_t st) {
  k_sum_chunks_c<<<(unsigned)ceil_div(width, 128), 128, 0, st>>>(part, nchunk, width, out);
  MW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- K6 (CGS2)
// part1[chunk][k][c] = sum_{rows of chunk} conj(V_k[r][c]) w1[r][c] and, if
// w2 is given, part2 likewise with w2, for k < kcount.  A workgroup takes KG
// basis vectors of one row chunk and 64 columns, so w1 and w2 are read once
// per KG vectors; every (k, c) sum runs over the chunk's rows in the same
// order whatever KG and the other columns are.
constexpr int DOTS_KG = 6;
constexpr int CGS_HK = 64;   // coefficients held in LDS up to this many (complex) per column
template <class B, int DOTS_KG = 6>
__global__ void __launch_bounds__(256) k_dots_partial(const B* __restrict__ V, int64_t vstride, int kcount,
                                                      const B* __restrict__ w1, const double2* __restrict__ w2,
                                                      int64_t n, int64_t ld, int ncols,
                                                      const int32_t* __restrict__ act, double2* __restrict__ part1,
                                                      double2* __restrict__ part2, const double* __restrict__ w1sc) {
  __shared__ double2 red[4][64];
  const int kb = blockIdx.x * DOTS_KG;
  const int chunk = blockIdx.y;
  const int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int c = blockIdx.z * 64 + cl;
  const int64_t r0 = (int64_t)chunk * RCHUNK, r1 = min(n, r0 + RCHUNK);
  double2 acc1[DOTS_KG], acc2[DOTS_KG];
#pragma unroll
  for (int q = 0; q < DOTS_KG; ++q) acc1[q] = acc2[q] = make_double2(0.0, 0.0);
  if (c < ncols && act[c]) {
    const B* Vb = V + (int64_t)kb * vstride;
    // RPD rows per pass (r, r + 4, ...): four with an FP32 basis (its loads
    // carry half the bytes; the raw values stay in registers until used),
    // two otherwise; each (k, column) sum still runs over the chunk's rows
    // in ascending order
    constexpr int RPD = sizeof(B) == 8 ? 4 : 2;
    for (int64_t r = r0 + rl; r < r1; r += 4 * RPD) {
      B x[RPD], v[RPD][DOTS_KG];
      double2 y[RPD];
      bool live[RPD];
#pragma unroll
      for (int h = 0; h < RPD; ++h) {
        live[h] = r + 4 * h < r1;
        const int64_t o = (r + 4 * h) * ld + c;
        x[h] = live[h] ? w1[o] : B{};
        y[h] = (live[h] && w2) ? w2[o] : make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < DOTS_KG; ++q) v[h][q] = (live[h] && kb + q < kcount) ? Vb[(int64_t)q * vstride + o] : B{};
      }
#pragma unroll
      for (int h = 0; h < RPD; ++h) {
        if (!live[h]) continue;
        const double2 xh = bload(x[h]);
#pragma unroll
        for (int q = 0; q < DOTS_KG; ++q)
          if (kb + q < kcount) {
            const double2 vq = bload(v[h][q]);
            acc1[q].x += vq.x * xh.x + vq.y * xh.y;
            acc1[q].y += vq.x * xh.y - vq.y * xh.x;
            acc2[q].x += vq.x * y[h].x + vq.y * y[h].y;
            acc2[q].y += vq.x * y[h].y - vq.y * y[h].x;
          }
      }
    }
  }
  if (w1sc && c < ncols) {
    // w1 = V_{kcount-1} stored unnormalised: every sum with w1 taken times
    // its factor, and the sums of V_{kcount-1} itself once more
    const double sc = w1sc[c];
#pragma unroll
    for (int q = 0; q < DOTS_KG; ++q) {
      const double s1 = kb + q == kcount - 1 ? sc * sc : sc, s2 = kb + q == kcount - 1 ? sc : 1.0;
      acc1[q].x *= s1;
      acc1[q].y *= s1;
      acc2[q].x *= s2;
      acc2[q].y *= s2;
    }
  }
#pragma unroll
  for (int q = 0; q < DOTS_KG; ++q) {
    if (kb + q < kcount) {
      red[rl][cl] = acc1[q];
      __syncthreads();
      if (rl == 0 && c < ncols)
        part1[((int64_t)chunk * kcount + kb + q) * ncols + c] =
            cadd(cadd(cadd(red[0][cl], red[1][cl]), red[2][cl]), red[3][cl]);
      __syncthreads();
      if (part2) {
        red[rl][cl] = acc2[q];
        __syncthreads();
        if (rl == 0 && c < ncols)
          part2[((int64_t)chunk * kcount + kb + q) * ncols + c] =
              cadd(cadd(cadd(red[0][cl], red[1][cl]), red[2][cl]), red[3][cl]);
        __syncthreads();
      }
    }
  }
}

template <class B>
void launch_dots_partial(const B* V, int64_t vstride, int kcount, const B* w1, const double2* w2,
                         int64_t n, int64_t ld, int ncols, const int32_t* act, double2* part1, double2* part2,
                         hipStream_t st, const double* w1sc) {
  kt_begin(KF_CGS_DOTS, st);
  // basis vectors per workgroup: 8 for an FP32 basis (the right vectors
  // re-read less often: 279 against 285 ms per 1 GHz step), 6 otherwise
  constexpr int KG = sizeof(B) == 8 ? 8 : DOTS_KG;
  dim3 g((unsigned)ceil_div(kcount, KG), (unsigned)reduce_chunks(n), (unsigned)ceil_div(ncols, 64));
  k_dots_partial<B, KG><<<g, 256, 0, st>>>(V, vstride, kcount, w1, w2, n, ld, ncols, act, part1,
                                           w2 ? part2 : nullptr, w1sc);
  MW_LAUNCH_CHECK();
  if (kt_enabled())
    kt_end(KF_CGS_DOTS, st, (w2 ? 16.0 : 8.0) * kcount * n * ncols,
           ((kcount + 1.0) * sizeof(B) + (w2 ? 16.0 : 0.0)) * n * ncols);
}
template void launch_dots_partial<double2>(const double2*, int64_t, int, const double2*, const double2*, int64_t,
                                           int64_t, int, const int32_t*, double2*, double2*, hipStream_t,
                                           const double*);
template void launch_dots_partial<float2>(const float2*, int64_t, int, const float2*, const double2*, int64_t,
                                          int64_t, int, const int32_t*, double2*, double2*, hipStream_t,
                                          const double*);

// ---------------------------------------------------------------- K6/K7 with delayed reorthogonalisation
// Arnoldi step j of every active column, scalar part (one thread per column).
// Slot j of the basis holds the candidate y (the previous new vector after
// one Gram-Schmidt pass, normalised: its norm before scaling was beta);
// T = A M^-1 y.  From the dot products P1 = [V_0..V_{j-1}, y]^H y and
// P2 = [V_0..V_{j-1}, y]^H T (a = P1[<j], alpha = P1[j], b = P2[<j],
// gamma = P2[j]):
//  * the second pass of y: v_j = (y - V a) / nu, nu = sqrt(alpha - |a|^2)
//    (nu = 1 for j = 0, where y = r0 / |r0| is final);
//  * column j-1 of the Hessenberg matrix becomes final:
//    Hraw[<j][j-1] = hprov + beta a, Hraw[j][j-1] = beta nu; it is rotated
//    by the previous Givens rotations and a new one into H, giving the
//    residual estimate |g_j| and Krylov dimension j (deactivation when
//    |g_j| <= tol |b| or the Krylov space is exhausted);
//  * the first pass of the next vector: with e = (gamma - a^H b) / nu,
//    A M^-1 v_j = (T - [V, v_j] Hraw a) / nu, whose projection on [V, v_j]
//    is hprov = ([b; e] - Hraw[0..j][0..j-1] a) / nu and whose remainder is
//    (T - V b - v_j e) / nu (formed by k_dgs_update).
// Equal in exact arithmetic to classical Gram-Schmidt applied twice; each
// basis vector is read twice per step instead of four times.
__global__ void k_dgs_step(int j, int m, int fin, int ncols, const double2* __restrict__ P1,
                           const double2* __restrict__ P2,
                           const double* __restrict__ beta2, double2* __restrict__ Hraw, double2* __restrict__ H,
                           double* __restrict__ cs, double2* __restrict__ sn, double2* __restrict__ g,
                           double2* __restrict__ hprov, double2* __restrict__ coef, double* __restrict__ nu_out,
                           double2* __restrict__ e_out, int32_t* __restrict__ kdim, int32_t* __restrict__ act,
                           double* __restrict__ resid, const double* __restrict__ bnorm, double tol,
                           double2* __restrict__ Rc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols || !act[c]) return;
  auto at = [&](const double2* X, int i) { return X[(int64_t)i * ncols + c]; };
  auto hr = [&](int i, int k) -> double2& { return Hraw[((int64_t)i * m + k) * ncols + c]; };
  const double alpha = at(P1, j).x;
  double a2 = 0.0;
  for (int k = 0; k < j; ++k) { double2 a = at(P1, k); a2 += a.x * a.x + a.y * a.y; }
  const double nu = j == 0 ? 1.0 : sqrt(fmax(alpha - a2, 0.0));
  if (j > 0 && fin) {
    const double beta = sqrt(beta2[c]);
    const double hn = beta * nu;
    for (int i = 0; i < j; ++i) {
      double2 a = at(P1, i);
      double2 h = at(hprov, i);
      hr(i, j - 1) = make_double2(h.x + beta * a.x, h.y + beta * a.y);
    }
    hr(j, j - 1) = make_double2(hn, 0.0);
    // rotate column j-1 into H
    for (int i = 0; i < j; ++i) H[((int64_t)i * m + j - 1) * ncols + c] = hr(i, j - 1);
    for (int i = 0; i + 1 < j; ++i) {
      double ci = cs[(int64_t)i * ncols + c];
      double2 si = sn[(int64_t)i * ncols + c];
      double2 x = H[((int64_t)i * m + j - 1) * ncols + c];
      double2 y = H[((int64_t)(i + 1) * m + j - 1) * ncols + c];
      H[((int64_t)i * m + j - 1) * ncols + c] = cadd(cscale(x, ci), cmul(si, y));
      H[((int64_t)(i + 1) * m + j - 1) * ncols + c] = csub(cscale(y, ci), cmulc(x, si));
    }
    double2 x = H[((int64_t)(j - 1) * m + j - 1) * ncols + c];
    double xa = hypot(x.x, x.y);
    double rho = hypot(xa, hn);
    double ci;
    double2 si, r;
    if (rho == 0.0) { ci = 1.0; si = make_double2(0.0, 0.0); r = make_double2(0.0, 0.0); }
    else if (xa == 0.0) { ci = 0.0; si = make_double2(1.0, 0.0); r = make_double2(hn, 0.0); }
    else {
      double2 ph = make_double2(x.x / xa, x.y / xa);
      ci = xa / rho;
      si = cscale(ph, hn / rho);
      r = cscale(ph, rho);
    }
    cs[(int64_t)(j - 1) * ncols + c] = ci;
    sn[(int64_t)(j - 1) * ncols + c] = si;
    H[((int64_t)(j - 1) * m + j - 1) * ncols + c] = r;
    double2 gj = g[(int64_t)(j - 1) * ncols + c];
    double2 gj1 = make_double2(-(si.x * gj.x + si.y * gj.y), -(si.x * gj.y - si.y * gj.x));   // -conj(s) g
    g[(int64_t)j * ncols + c] = gj1;
    g[(int64_t)(j - 1) * ncols + c] = cscale(gj, ci);
    kdim[c] = j;
    double res = hypot(gj1.x, gj1.y);
    resid[c] = res;
    if (!(res > tol * bnorm[c]) || !(hn > 0.0)) { act[c] = 0; return; }
  }
  if (j >= m || !P2) return;
  // first pass of the next vector
  double2 e = at(P2, j);
  for (int k = 0; k < j; ++k) {
    double2 a = at(P1, k), b = at(P2, k);
    e.x -= a.x * b.x + a.y * b.y;   // conj(a) b
    e.y -= a.x * b.y - a.y * b.x;
  }
  e = make_double2(e.x / nu, e.y / nu);
  for (int i = 0; i <= j; ++i) {
    double2 d = i < j ? at(P2, i) : e;
    for (int k = 0; k < j; ++k) d = csub(d, cmul(hr(i, k), at(P1, k)));
    hprov[(int64_t)i * ncols + c] = make_double2(d.x / nu, d.y / nu);
  }
  for (int k = 0; k < j; ++k) {
    coef[(int64_t)(2 * k) * ncols + c] = at(P1, k);
    coef[(int64_t)(2 * k + 1) * ncols + c] = at(P2, k);
  }
  nu_out[c] = nu;
  e_out[c] = e;
  if (Rc) {
    // column j of the triangular factor relating the candidates to the basis:
    // y_j = nu v_j + sum_k a_k v_k
    for (int k = 0; k < j; ++k) Rc[((int64_t)k * m + j) * ncols + c] = at(P1, k);
    Rc[((int64_t)j * m + j) * ncols + c] = make_double2(nu, 0.0);
  }
}

void launch_dgs_step(int j, int m, bool fin, int ncols, const double2* P1, const double2* P2, const double* beta2,
                     double2* Hraw, double2* H, double* cs, double2* sn, double2* g, double2* hprov, double2* coef,
                     double* nu, double2* e, int32_t* kdim, int32_t* act, double* resid, const double* bnorm,
                     double tol, double2* Rc, hipStream_t st) {
  k_dgs_step<<<(unsigned)ceil_div(ncols, 64), 64, 0, st>>>(j, m, fin ? 1 : 0, ncols, P1, P2, beta2, Hraw, H, cs, sn,
                                                          g, hprov, coef, nu, e, kdim, act, resid, bnorm, tol, Rc);
  MW_LAUNCH_CHECK();
}

// Residual estimate the next step would give, from the provisional column j
// (its second-pass correction is of the order of the rounding error): the
// column rotated by the rotations so far and a trial rotation.  done[c] = 1
// when the estimate reaches tol |b| or the Krylov space is exhausted, so that
// the next step can finish column j without applying the operator.
__global__ void k_dgs_trial(int j, int m, int ncols, const double2* __restrict__ hprov, const double* __restrict__ beta2,
                            const double* __restrict__ cs, const double2* __restrict__ sn,
                            const double2* __restrict__ g, const int32_t* __restrict__ act,
                            const double* __restrict__ bnorm, double tol, int32_t* __restrict__ done) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  if (!act[c]) { done[c] = 1; return; }
  double2 x = hprov[c], nx = make_double2(0.0, 0.0);
  for (int i = 0; i < j; ++i) {
    nx = hprov[(int64_t)(i + 1) * ncols + c];
    double ci = cs[(int64_t)i * ncols + c];
    double2 si = sn[(int64_t)i * ncols + c];
    x = csub(cscale(nx, ci), cmulc(x, si));   // the lower entry after rotation i
  }
  const double hn = sqrt(beta2[c]);
  const double rho = hypot(hypot(x.x, x.y), hn);
  const double2 gj = g[(int64_t)j * ncols + c];
  const double res = rho > 0.0 ? hypot(gj.x, gj.y) * hn / rho : 0.0;
  done[c] = (!(res > tol * bnorm[c]) || !(hn > 0.0)) ? 1 : 0;
}

void launch_dgs_trial(int j, int m, int ncols, const double2* hprov, const double* beta2, const double* cs,
                      const double2* sn, const double2* g, const int32_t* act, const double* bnorm, double tol,
                      int32_t* done, hipStream_t st) {
  k_dgs_trial<<<(unsigned)ceil_div(ncols, 64), 64, 0, st>>>(j, m, ncols, hprov, beta2, cs, sn, g, act, bnorm, tol,
                                                           done);
  MW_LAUNCH_CHECK();
}

// Vector part of step j: v_j = (y - sum_k V_k a_k) / nu in place of y (slot
// j), and the next candidate u = (T - sum_k V_k b_k - v_j e) / nu into slot
// j+1, with |u|^2 chunk partials; coef holds (a_k, b_k) interleaved.  The
// coefficients sit in LDS when 2j <= CGS_HK.
template <class B, int RPT, bool CF_LDS>
__global__ void __launch_bounds__(256) k_dgs_update(B* __restrict__ V, int64_t vstride, int j,
                                                    const double2* __restrict__ coef, const double* __restrict__ nu,
                                                    const double2* __restrict__ e, const double2* __restrict__ T,
                                                    int64_t n, int64_t ld, int ncols, const int32_t* __restrict__ act,
                                                    double* __restrict__ norm_part, const double* __restrict__ vjsc) {
  __shared__ double red[4][64];
  extern __shared__ double2 cf[];   // [2j][64] when 2j <= CGS_HK
  const int chunk = blockIdx.x;
  const int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int c = blockIdx.y * 64 + cl;
  const int64_t r0 = (int64_t)chunk * RCHUNK, r1 = min(n, r0 + RCHUNK);
  if (CF_LDS) {
    for (int k = rl; k < 2 * j; k += 4) cf[k * 64 + cl] = c < ncols ? coef[(int64_t)k * ncols + c] : make_double2(0.0, 0.0);
    __syncthreads();
  }
  double acc = 0.0;
  if (c < ncols && act[c]) {
    const double inu = nu[c];
    const double2 ec = e[c];
    const double sc = col_scale(vjsc, c);   // v_j stored unnormalised when vjsc is given
    B* Vj = V + (int64_t)j * vstride;
    B* Vn = V + (int64_t)(j + 1) * vstride;
    // RP rows per pass (r, r + 4, ...), sharing each coefficient load; the
    // norm is summed over the rows in ascending order
    constexpr int RP = RPT;
    for (int64_t r = r0 + rl; r < r1; r += 4 * RP) {
      // rows past the chunk read its last row (every load unconditional,
      // so none waits behind a branch) and are neither stored nor summed
      int64_t o[RP];
      bool live[RP];
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        live[q] = r + 4 * q < r1;
        o[q] = (live[q] ? r + 4 * q : r1 - 1) * ld + c;
      }
      B yr[RP];
      double2 u[RP];
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        yr[q] = Vj[o[q]];
        u[q] = T[o[q]];
      }
      // basis vectors two ahead: n0 holds V_k for even k, n1 for odd k,
      // each reloaded with V_{k+2} (clamped to V_{j-1}) right after its use,
      // so that two vectors' loads are in flight while one is applied
      const int jl = j > 0 ? j - 1 : 0;
      B n0[RP], n1[RP];
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        n0[q] = V[o[q]];
        n1[q] = V[(int64_t)min(1, jl) * vstride + o[q]];
      }
      double2 y[RP];
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        y[q] = bload(yr[q]);
        y[q].x *= sc;
        y[q].y *= sc;
      }
      auto apply = [&](int k, B(&cur)[RP]) {
        // (LDS or global by template: a select between the two would make
        // a flat load, which waits for every load in flight)
        double2 ak, bk;
        if constexpr (CF_LDS) {
          ak = cf[(2 * k) * 64 + cl];
          bk = cf[(2 * k + 1) * 64 + cl];
        } else {
          ak = coef[(int64_t)(2 * k) * ncols + c];
          bk = coef[(int64_t)(2 * k + 1) * ncols + c];
        }
#pragma unroll
        for (int q = 0; q < RP; ++q) {
          const double2 v = bload(cur[q]);
          y[q].x -= v.x * ak.x - v.y * ak.y;
          y[q].y -= v.x * ak.y + v.y * ak.x;
          u[q].x -= v.x * bk.x - v.y * bk.y;
          u[q].y -= v.x * bk.y + v.y * bk.x;
        }
        const B* Vk2 = V + (int64_t)min(k + 2, jl) * vstride;
#pragma unroll
        for (int q = 0; q < RP; ++q) cur[q] = Vk2[o[q]];
      };
#pragma unroll 1
      for (int k = 0; k < j; k += 2) {
        apply(k, n0);
        if (k + 1 < j) apply(k + 1, n1);
      }
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        if (!live[q]) continue;
        double2 yy = make_double2(y[q].x / inu, y[q].y / inu);
        double2 uu = u[q];
        uu.x -= yy.x * ec.x - yy.y * ec.y;
        uu.y -= yy.x * ec.y + yy.y * ec.x;
        uu = make_double2(uu.x / inu, uu.y / inu);
        Vj[o[q]] = bstore<B>(yy);
        const B us = bstore<B>(uu);
        Vn[o[q]] = us;
        // the norm of what is stored (the candidate the next step uses)
        const double2 ur = bload(us);
        acc += ur.x * ur.x + ur.y * ur.y;
      }
    }
  }
  red[rl][cl] = acc;
  __syncthreads();
  if (rl == 0 && c < ncols)
    norm_part[(int64_t)chunk * ncols + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

template <class B>
void launch_dgs_update(B* V, int64_t vstride, int j, const double2* coef, const double* nu, const double2* e,
                       const double2* T, int64_t n, int64_t ld, int ncols, const int32_t* act, double* norm_part,
                       hipStream_t st, const double* vjsc) {
  dim3 g((unsigned)reduce_chunks(n), (unsigned)ceil_div(ncols, 64));
  size_t lds = 2 * j <= CGS_HK ? (size_t)(2 * j) * 64 * sizeof(double2) : 0;
  kt_begin(KF_CGS_UPDATE, st);
  // rows per pass: 8 for an FP32 basis (323 against 330 ms per 1 GHz step), 4 otherwise
  if (2 * j <= CGS_HK)
    k_dgs_update<B, sizeof(B) == 8 ? 8 : 4, true><<<g, 256, lds, st>>>(V, vstride, j, coef, nu, e, T, n, ld, ncols,
                                                                     act, norm_part, vjsc);
  else
    k_dgs_update<B, sizeof(B) == 8 ? 8 : 4, false><<<g, 256, 0, st>>>(V, vstride, j, coef, nu, e, T, n, ld, ncols,
                                                                    act, norm_part, vjsc);
  MW_LAUNCH_CHECK();
  // reads V_0..V_j and T, writes v_j and the next candidate
  if (kt_enabled()) kt_end(KF_CGS_UPDATE, st, 16.0 * j * n * ncols, ((j + 3.0) * sizeof(B) + 16.0) * n * ncols);
}
template void launch_dgs_update<double2>(double2*, int64_t, int, const double2*, const double*, const double2*,
                                         const double2*, int64_t, int64_t, int, const int32_t*, double*, hipStream_t,
                                         const double*);
template void launch_dgs_update<float2>(float2*, int64_t, int, const double2*, const double*, const double2*,
                                        const double2*, int64_t, int64_t, int, const int32_t*, double*, hipStream_t,
                                        const double*);

// w[:, c] /= sqrt(nrm2[c]) for active columns with a nonzero norm
template <class B>
__global__ void k_scale_cols(B* __restrict__ w, int64_t n, int64_t ld, int ncols, const double* __restrict__ nrm2,
                             const int32_t* __restrict__ act) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t r = id / ncols;
  int c = (int)(id % ncols);
  if (r >= n || !act[c]) return;
  double s = sqrt(nrm2[c]);
  if (s > 0.0) {
    const double2 v = bload(w[r * ld + c]);
    w[r * ld + c] = bstore<B>(make_double2(v.x / s, v.y / s));
  }
}
template <class B>
void launch_scale_cols(B* w, int64_t n, int64_t ld, int ncols, const double* nrm, const int32_t* act,
                       hipStream_t st) {
  k_scale_cols<B><<<(unsigned)ceil_div(n * ncols, 256), 256, 0, st>>>(w, n, ld, ncols, nrm, act);
  MW_LAUNCH_CHECK();
}
template void launch_scale_cols<double2>(double2*, int64_t, int64_t, int, const double*, const int32_t*, hipStream_t);
template void launch_scale_cols<float2>(float2*, int64_t, int64_t, int, const double*, const int32_t*, hipStream_t);

// ---------------------------------------------------------------- K7
// y = R^-1 g on the Krylov dimension of each column (back substitution)
__global__ void k_backsolve(int m, int ncols, const double2* __restrict__ H, const double2* __restrict__ g,
                            const int32_t* __restrict__ kdim, double2* __restrict__ y) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  int kk = kdim[c];
  for (int i = kk - 1; i >= 0; --i) {
    double2 s = g[(int64_t)i * ncols + c];
    for (int t = i + 1; t < kk; ++t) s = csub(s, cmul(H[((int64_t)i * m + t) * ncols + c], y[(int64_t)t * ncols + c]));
    y[(int64_t)i * ncols + c] = cmul(s, cinv(H[((int64_t)i * m + i) * ncols + c]));
  }
}
void launch_backsolve(int m, int ncols, const double2* H, const double2* g, const int32_t* kdim, double2* y,
                      hipStream_t st) {
  k_backsolve<<<(unsigned)ceil_div(ncols, 64), 64, 0, st>>>(m, ncols, H, g, kdim, y);
  MW_LAUNCH_CHECK();
}

// y <- Rc^-1 y on the Krylov dimension of each column (Rc upper triangular,
// m x m per column, as written by k_dgs_step): the coefficients of the
// combination of the operator's inputs (the candidates) equal to V y
__global__ void k_candsolve(int m, int ncols, const double2* __restrict__ Rc, const int32_t* __restrict__ kdim,
                            double2* __restrict__ y) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  int kk = kdim[c];
  for (int i = kk - 1; i >= 0; --i) {
    double2 s = y[(int64_t)i * ncols + c];
    for (int t = i + 1; t < kk; ++t) s = csub(s, cmul(Rc[((int64_t)i * m + t) * ncols + c], y[(int64_t)t * ncols + c]));
    y[(int64_t)i * ncols + c] = cmul(s, cinv(Rc[((int64_t)i * m + i) * ncols + c]));
  }
}
void launch_candsolve(int m, int ncols, const double2* Rc, const int32_t* kdim, double2* y, hipStream_t st) {
  k_candsolve<<<(unsigned)ceil_div(ncols, 64), 64, 0, st>>>(m, ncols, Rc, kdim, y);
  MW_LAUNCH_CHECK();
}

// u[r][c] = sum_{k < kdim[c]} V_k[r][c] y[k][c]
template <class B>
__global__ void k_combine(const B* __restrict__ V, int64_t vstride, const double2* __restrict__ y,
                          const int32_t* __restrict__ kdim, double2* __restrict__ u, int64_t n, int64_t ld,
                          int ncols) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t r = id / ncols;
  int c = (int)(id % ncols);
  if (r >= n) return;
  double2 acc = make_double2(0.0, 0.0);
  int kk = kdim[c];
  for (int k = 0; k < kk; ++k)
    acc = cadd(acc, cmul(bload(V[(int64_t)k * vstride + r * ld + c]), y[(int64_t)k * ncols + c]));
  u[r * ld + c] = acc;
}
template <class B>
void launch_combine(const B* V, int64_t vstride, int m, const double2* y, const int32_t* kdim, double2* u,
                    int64_t n, int64_t ld, int ncols, hipStream_t st) {
  (void)m;
  k_combine<B><<<(unsigned)ceil_div(n * ncols, 256), 256, 0, st>>>(V, vstride, y, kdim, u, n, ld, ncols);
  MW_LAUNCH_CHECK();
}
template void launch_combine<double2>(const double2*, int64_t, int, const double2*, const int32_t*, double2*,
                                      int64_t, int64_t, int, hipStream_t);
template void launch_combine<float2>(const float2*, int64_t, int, const double2*, const int32_t*, double2*, int64_t,
                                     int64_t, int, hipStream_t);

__global__ void k_axpy_cols(double2* __restrict__ x, const double2* __restrict__ z, int64_t total) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id < total) x[id] = cadd(x[id], z[id]);
}
void launch_axpy_cols(double2* x, const double2* z, int64_t n, int64_t ld, int ncols, hipStream_t st) {
  (void)ncols;
  int64_t tot = n * ld;
  k_axpy_cols<<<(unsigned)ceil_div(tot, 256), 256, 0, st>>>(x, z, tot);
  MW_LAUNCH_CHECK();
}

// v0 = r / ||r|| for active columns, 0 elsewhere
template <class B>
__global__ void k_start_cycle(const double2* __restrict__ r, B* __restrict__ v0, int64_t n, int64_t ld,
                              int ncols, const double* __restrict__ rn2, const int32_t* __restrict__ act) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t row = id / ncols;
  int c = (int)(id % ncols);
  if (row >= n) return;
  double2 v = make_double2(0.0, 0.0);
  if (act[c]) {
    double s = sqrt(rn2[c]);
    double2 x = r[row * ld + c];
    v = make_double2(x.x / s, x.y / s);
  }
  v0[row * ld + c] = bstore<B>(v);
}
template <class B>
void launch_start_cycle(const double2* r, B* v0, int64_t n, int64_t ld, int ncols, const double* rn2,
                        const int32_t* act, hipStream_t st) {
  k_start_cycle<B><<<(unsigned)ceil_div(n * ncols, 256), 256, 0, st>>>(r, v0, n, ld, ncols, rn2, act);
  MW_LAUNCH_CHECK();
}
template void launch_start_cycle<double2>(const double2*, double2*, int64_t, int64_t, int, const double*,
                                          const int32_t*, hipStream_t);
template void launch_start_cycle<float2>(const double2*, float2*, int64_t, int64_t, int, const double*,
                                         const int32_t*, hipStream_t);

__global__ void k_widen(const float2* __restrict__ src, double2* __restrict__ dst, int64_t count) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id < count) dst[id] = make_double2(src[id].x, src[id].y);
}
void launch_widen(const float2* src, double2* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  k_widen<<<(unsigned)ceil_div(count, 256), 256, 0, st>>>(src, dst, count);
  MW_LAUNCH_CHECK();
}
__global__ void k_narrow(const double2* __restrict__ src, float2* __restrict__ dst, int64_t count) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id < count) dst[id] = bstore<float2>(src[id]);
}
void launch_narrow(const double2* src, float2* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  k_narrow<<<(unsigned)ceil_div(count, 256), 256, 0, st>>>(src, dst, count);
  MW_LAUNCH_CHECK();
}

__global__ void k_copy_cols(const double2* __restrict__ src, int64_t lds, double2* __restrict__ dst, int64_t ldd,
                            int64_t n, int ncols) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t r = id / ncols;
  int c = (int)(id % ncols);
  if (r >= n) return;
  dst[r * ldd + c] = src[r * lds + c];
}
void launch_copy_cols(const double2* src, int64_t lds, double2* dst, int64_t ldd, int64_t n, int ncols,
                      hipStream_t st) {
  if (n * ncols == 0) return;
  k_copy_cols<<<(unsigned)ceil_div(n * ncols, 256), 256, 0, st>>>(src, lds, dst, ldd, n, ncols);
  MW_LAUNCH_CHECK();
}

__global__ void k_move_cols(const double2* __restrict__ src, int64_t lds, const int32_t* __restrict__ idx,
                            double2* __restrict__ dst, int64_t ldd, int64_t n, int ncols, int scatter) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t r = id / ncols;
  int k = (int)(id % ncols);
  if (r >= n) return;
  if (scatter) dst[r * ldd + idx[k]] = src ? src[r * lds + k] : make_double2(0.0, 0.0);
  else dst[r * ldd + k] = src[r * lds + idx[k]];
}
void launch_gather_cols(const double2* src, int64_t lds, const int32_t* idx, double2* dst, int64_t ldd, int64_t n,
                        int ncols, hipStream_t st) {
  if (n * ncols == 0) return;
  k_move_cols<<<(unsigned)ceil_div(n * ncols, 256), 256, 0, st>>>(src, lds, idx, dst, ldd, n, ncols, 0);
  MW_LAUNCH_CHECK();
}
void launch_scatter_cols(const double2* src, int64_t lds, const int32_t* idx, double2* dst, int64_t ldd, int64_t n,
                         int ncols, hipStream_t st) {
  if (n * ncols == 0) return;
  k_move_cols<<<(unsigned)ceil_div(n * ncols, 256), 256, 0, st>>>(src, lds, idx, dst, ldd, n, ncols, 1);
  MW_LAUNCH_CHECK();
}

__global__ void k_zero_bytes(uint32_t* __restrict__ p, int64_t words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
void launch_zero_bytes(void* p, int64_t bytes, hipStream_t st) {
  if (bytes <= 0) return;
  MW_CHECK(bytes % 4 == 0, MW_EINVAL, "zero fill of a non-word size");
  int64_t words = bytes / 4;
  unsigned grid = (unsigned)std::min<int64_t>(ceil_div(words, 256), 65536);
  k_zero_bytes<<<grid, 256, 0, st>>>(reinterpret_cast<uint32_t*>(p), words);
  MW_LAUNCH_CHECK();
}
void launch_zero(double2* p, int64_t count, hipStream_t st) { launch_zero_bytes(p, count * 16, st); }

// gS = S - Smes and J = 1/2 sum |gS|^2 (one workgroup, fixed summation order)
__global__ void __launch_bounds__(256) k_misfit(const double2* __restrict__ S, const double2* __restrict__ Sm,
                                                const double* __restrict__ W, int64_t count,
                                                double2* __restrict__ gS, double* __restrict__ J) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < count; k += 256) {
    double2 d = csub(S[k], Sm[k]);
    const double w = W ? W[k] : 1.0;
    gS[k] = make_double2(w * d.x, w * d.y);
    acc += w * (d.x * d.x + d.y * d.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) J[0] = 0.5 * red[0];
}
void launch_misfit(const double2* S, const double2* Sm, const double* W, int64_t count, double2* gS, double* J,
                   hipStream_t st) {
  k_misfit<<<1, 256, 0, st>>>(S, Sm, W, count, gS, J);
  MW_LAUNCH_CHECK();
}

}  // namespace mw
