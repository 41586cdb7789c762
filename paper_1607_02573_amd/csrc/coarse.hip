// Two-level ORAS: the coarse correction added to the one-level
// preconditioner (the paper's conclusion, Section 7, names a coarse space as
// the way to keep the iteration count from growing with the number of
// subdomains, Section 6.1 Table tabscaling).
//
// Coarse space: every subdomain i contributes the partition-of-unity-weighted
// edge interpolants of the three constant fields, Z_i = R_i^T D_i Phi_i with
// Phi_i[l, a] = t_g[a] (t_g = x_hi - x_lo of the edge of unknown g = R_i(l));
// the coarse unknown (i, a) is number 3 i + a.  Coarse operator E = Z^T A Z
// (complex symmetric), factored densely by the subdomain factorisation.
// Correction in the deflated form
//     M2^-1 v = M^-1 (v - A q) + q,   q = Z E^-1 Z^T v.
// The kernels here assemble E, apply Z^T and Z; the factorisation, the coarse
// triangular solves, the SpMM and M^-1 are the one-level kernels.
#include "kernels.hpp"

namespace mw {

namespace {

// first index of `key` in the ascending list a[0..n), -1 if absent
__device__ inline int find_sorted(const int32_t* a, int n, int32_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && a[lo] == key) ? lo : -1;
}

template <class C> __device__ inline C to_c(double re, double im) { C z; z.x = re; z.y = im; return z; }

}  // namespace

// E rows 3i .. 3i+2 (one workgroup per subdomain i), written in full
// (ldf = padded coarse size) in the factor precision:
//   E[(i,a), (j,b)] = sum over the unknowns g of i with D_i(g) > 0, the
//   nonzeros A[g,h], and the copies of h in subdomains j with D_j(h) > 0, of
//   D_i(g) t_g[a] A[g,h] D_j(h) t_h[b].
// The sums over (g, h, j) for one (i, j) pair are accumulated in LDS by
// atomic adds (their order, and so the last bits of E, may differ between
// runs; E is fixed once factored).
template <class C>
__global__ void __launch_bounds__(256) k_coarse_matrix(const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double2* __restrict__ val, DeviceDecomp d,
                                                       DeviceCoarse cz, C* __restrict__ F, int ldf) {
  extern __shared__ double acc[];   // [nnb][9][2]
  __shared__ int32_t nbl[kCoarseMaxNb];
  const int i = blockIdx.x;
  const int64_t nb0 = cz.nb_ptr[i];
  const int nnb = (int)(cz.nb_ptr[i + 1] - nb0);
  for (int k = threadIdx.x; k < nnb; k += blockDim.x) nbl[k] = cz.nb[nb0 + k];
  for (int k = threadIdx.x; k < nnb * 18; k += blockDim.x) acc[k] = 0.0;
  __syncthreads();
  const int64_t r0 = d.loc_off[i], r1 = r0 + d.n_pad[i];
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const int32_t g = d.sub_dof[r];
    const double w = d.D[r];
    if (g < 0 || w == 0.0) continue;
    const double tg0 = w * cz.tvec[3 * (int64_t)g], tg1 = w * cz.tvec[3 * (int64_t)g + 1],
                 tg2 = w * cz.tvec[3 * (int64_t)g + 2];
    for (int64_t k = row_ptr[g]; k < row_ptr[g + 1]; ++k) {
      const int32_t h = col[k];
      const double2 a = val[k];
      const double th0 = cz.tvec[3 * (int64_t)h], th1 = cz.tvec[3 * (int64_t)h + 1], th2 = cz.tvec[3 * (int64_t)h + 2];
      for (int64_t q = d.cp_ptr[h]; q < d.cp_ptr[h + 1]; ++q) {
        const int64_t rr = d.cp_row[q];
        const int s = find_sorted(nbl, nnb, cz.row_sub[rr]);
        if (s < 0) continue;   // cannot happen: the neighbour lists hold every such j
        const double dj = d.D[rr];
        const double tb[3] = {dj * th0, dj * th1, dj * th2};
        const double ta[3] = {tg0, tg1, tg2};
        double* dst = acc + (int64_t)s * 18;
        for (int x = 0; x < 3; ++x)
          for (int y = 0; y < 3; ++y) {
            const double f = ta[x] * tb[y];
            atomicAdd(dst + 2 * (3 * x + y), f * a.x);
            atomicAdd(dst + 2 * (3 * x + y) + 1, f * a.y);
          }
      }
    }
  }
  __syncthreads();
  const int nc = 3 * cz.nsub;
  for (int64_t e = threadIdx.x; e < 3 * (int64_t)ldf; e += blockDim.x) {
    const int x = (int)(e / ldf), c = (int)(e % ldf);
    double re = 0.0, im = 0.0;
    if (c < nc) {
      const int s = find_sorted(nbl, nnb, c / 3);
      if (s >= 0) {
        re = acc[s * 18 + 2 * (3 * x + c % 3)];
        im = acc[s * 18 + 2 * (3 * x + c % 3) + 1];
      }
    }
    F[(int64_t)(3 * i + x) * ldf + c] = to_c<C>(re, im);
  }
}

// rows nc .. ldf-1 of the padded coarse matrix: identity
template <class C>
__global__ void k_coarse_pad(C* F, int nc, int ldf) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t rows = ldf - nc;
  if (e >= rows * ldf) return;
  const int r = nc + (int)(e / ldf), c = (int)(e % ldf);
  F[(int64_t)r * ldf + c] = to_c<C>(r == c ? 1.0 : 0.0, 0.0);
}

// Y[3i+a, c] = sum over the local rows of i of D t_g[a] V[g, c]: one
// workgroup per (subdomain, 8 columns); thread (row lane, column) with 32 row
// lanes, so a column's sum order does not depend on the number of columns
template <class C>
__global__ void __launch_bounds__(256) k_coarse_restrict(DeviceDecomp d, DeviceCoarse cz, const double2* __restrict__ V,
                                                         int64_t ldv, int ncols, C* __restrict__ Y, int64_t ldy) {
  __shared__ double red[256][6];
  const int i = blockIdx.x;
  const int cc = threadIdx.x & 7, lane = threadIdx.x >> 3;
  const int c = blockIdx.y * 8 + cc;
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (c < ncols) {
    const int64_t r0 = d.loc_off[i], r1 = r0 + d.n_pad[i];
    for (int64_t r = r0 + lane; r < r1; r += 32) {
      const int32_t g = d.sub_dof[r];
      const double w = d.D[r];
      if (g < 0 || w == 0.0) continue;
      const double2 v = V[(int64_t)g * ldv + c];
      for (int a = 0; a < 3; ++a) {
        const double t = w * cz.tvec[3 * (int64_t)g + a];
        s[2 * a] += t * v.x;
        s[2 * a + 1] += t * v.y;
      }
    }
  }
  for (int k = 0; k < 6; ++k) red[threadIdx.x][k] = s[k];
  __syncthreads();
  if (threadIdx.x < 48) {
    const int col = threadIdx.x & 7, k = threadIdx.x >> 3;   // k: component 0..5
    double t = 0.0;
    for (int l = 0; l < 32; ++l) t += red[l * 8 + col][k];
    const int cout = blockIdx.y * 8 + col;
    if (cout < ncols) {
      C* y = Y + (int64_t)(3 * i + (k >> 1)) * ldy + cout;
      if (k & 1) y->y = t;
      else y->x = t;
    }
  }
}

// zero rows [r0, r1) of Y (padding of the coarse vector)
template <class C>
__global__ void k_coarse_zero_rows(C* Y, int64_t ldy, int r0, int r1, int ncols) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)(r1 - r0) * ncols) return;
  Y[(int64_t)(r0 + e / ncols) * ldy + e % ncols] = to_c<C>(0.0, 0.0);
}

// Q[g, c] = sum over the copies r of g (ascending subdomain) of
// D(r) t_g . Y[3 sub(r) + (0..2), c]
template <class C>
__global__ void k_coarse_prolong(int64_t n, DeviceDecomp d, DeviceCoarse cz, const C* __restrict__ Y, int64_t ldy,
                                 int ncols, double2* __restrict__ Q, int64_t ldq) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t g = id / ncols;
  const int c = (int)(id % ncols);
  if (g >= n) return;
  const double t0 = cz.tvec[3 * g], t1 = cz.tvec[3 * g + 1], t2 = cz.tvec[3 * g + 2];
  double re = 0.0, im = 0.0;
  for (int64_t k = d.cp_ptr[g]; k < d.cp_ptr[g + 1]; ++k) {
    const int64_t r = d.cp_row[k];
    const double w = d.D[r];
    const int64_t b = 3 * (int64_t)cz.row_sub[r];
    const C y0 = Y[b * ldy + c], y1 = Y[(b + 1) * ldy + c], y2 = Y[(b + 2) * ldy + c];
    re += w * (t0 * (double)y0.x + t1 * (double)y1.x + t2 * (double)y2.x);
    im += w * (t0 * (double)y0.y + t1 * (double)y1.y + t2 * (double)y2.y);
  }
  Q[g * ldq + c] = make_double2(re, im);
}

template <class C>
void launch_coarse_matrix(const DeviceMesh& m, const double2* val, const DeviceDecomp& d, const DeviceCoarse& cz,
                          C* F, int ldf, hipStream_t st) {
  kt_begin(KF_COARSE, st);
  const size_t lds = (size_t)cz.max_nb * 18 * sizeof(double);
  k_coarse_matrix<C><<<cz.nsub, 256, lds, st>>>(m.row_ptr, m.col, val, d, cz, F, ldf);
  MW_LAUNCH_CHECK();
  const int nc = 3 * cz.nsub;
  if (ldf > nc) {
    const int64_t tot = (int64_t)(ldf - nc) * ldf;
    k_coarse_pad<C><<<(unsigned)ceil_div(tot, 256), 256, 0, st>>>(F, nc, ldf);
    MW_LAUNCH_CHECK();
  }
  if (kt_enabled()) {
    double sl = 0;
    for (int i = 0; i < d.nsub; ++i) sl += d.h_n_loc[i];
    // rows of the subdomains (index, weight, edge vector), their A rows read
    // again per copy, and E written
    kt_end(KF_COARSE, st, 0.0, sl * (4 + 8 + 24) + (double)m.nnz * 20 * 3 + (double)ldf * ldf * sizeof(C));
  }
}

template <class C>
void launch_coarse_restrict(const DeviceDecomp& d, const DeviceCoarse& cz, const double2* V, int64_t ldv, int ncols,
                            C* Y, int64_t ldy, int ldf, hipStream_t st) {
  kt_begin(KF_COARSE, st);
  dim3 grid((unsigned)cz.nsub, (unsigned)ceil_div(ncols, 8));
  k_coarse_restrict<C><<<grid, 256, 0, st>>>(d, cz, V, ldv, ncols, Y, ldy);
  MW_LAUNCH_CHECK();
  const int nc = 3 * cz.nsub;
  if (ldf > nc) {
    const int64_t tot = (int64_t)(ldf - nc) * ncols;
    k_coarse_zero_rows<C><<<(unsigned)ceil_div(tot, 256), 256, 0, st>>>(Y, ldy, nc, ldf, ncols);
    MW_LAUNCH_CHECK();
  }
  if (kt_enabled()) {
    double sl = 0;
    for (int i = 0; i < d.nsub; ++i) sl += d.h_n_loc[i];
    kt_end(KF_COARSE, st, 12.0 * sl * ncols, sl * (4 + 8 + 24 + 16.0 * ncols) + (double)ldf * ncols * sizeof(C));
  }
}

template <class C>
void launch_coarse_prolong(const DeviceDecomp& d, const DeviceCoarse& cz, int64_t n, const C* Y, int64_t ldy,
                           int ncols, double2* Q, int64_t ldq, hipStream_t st) {
  kt_begin(KF_COARSE, st);
  const int64_t tot = n * ncols;
  k_coarse_prolong<C><<<(unsigned)ceil_div(tot, 256), 256, 0, st>>>(n, d, cz, Y, ldy, ncols, Q, ldq);
  MW_LAUNCH_CHECK();
  if (kt_enabled()) kt_end(KF_COARSE, st, 0.0, (double)n * (24 + 16.0 * ncols) + 3.0 * cz.nsub * ncols * sizeof(C));
}

template void launch_coarse_matrix<float2>(const DeviceMesh&, const double2*, const DeviceDecomp&, const DeviceCoarse&,
                                           float2*, int, hipStream_t);
template void launch_coarse_matrix<double2>(const DeviceMesh&, const double2*, const DeviceDecomp&,
                                            const DeviceCoarse&, double2*, int, hipStream_t);
template void launch_coarse_restrict<float2>(const DeviceDecomp&, const DeviceCoarse&, const double2*, int64_t, int,
                                             float2*, int64_t, int, hipStream_t);
template void launch_coarse_restrict<double2>(const DeviceDecomp&, const DeviceCoarse&, const double2*, int64_t, int,
                                              double2*, int64_t, int, hipStream_t);
template void launch_coarse_prolong<float2>(const DeviceDecomp&, const DeviceCoarse&, int64_t, const float2*, int64_t,
                                            int, double2*, int64_t, hipStream_t);
template void launch_coarse_prolong<double2>(const DeviceDecomp&, const DeviceCoarse&, int64_t, const double2*,
                                             int64_t, int, double2*, int64_t, hipStream_t);

}  // namespace mw
