// Batched dense complex LU with partial pivoting and triangular solves of the
// ORAS subdomain matrices B_i (paper Section 3: M^-1 = sum R_i^T D_i B_i^-1 R_i,
// each B_i factored once; applying B_i^-1 to many vectors is one forward
// elimination and one backward substitution).
//
// Layout: B_i is row-major with n_pad rows (n_pad a multiple of 64) at
// F + fac_off[i], each 64-row block storing the columns [blo, blo + bw) of
// its rows (block tables of DeviceDecomp; frow() gives a row's base): all
// n_pad columns for LU with interchanges, the structural envelope of the
// block's rows (aligned to 64, plus room for U_kk^-1 beside the diagonal
// block) for L D L^T without interchanges.  The LU kernels that pivot
// (k_lu_panel*, k_laswp, k_trsm_panel, k_gemm_luw without LOWER) address
// dense rows of n_pad; every other kernel goes through the block tables.
// Every kernel is batched over the subdomains (grid.y or grid.x =
// subdomain) and skips the parts beyond each subdomain's size.
//
// LU (right-looking, LAPACK-style row interchanges on the whole row):
//   for each 64-wide panel k:
//     for each 8-wide sub-panel c of it:
//       k_lu_panel: pivot search (max |re|+|im|, lowest row on ties), row
//         swap across the 64-wide panel, scaling, rank-1 updates inside the
//         sub-panel, unit-lower solve of the sub-panel's U rows for the rest
//         of the 64-wide panel;
//       GEMM: trailing rows x rest of the 64-wide panel -= L * U  (K = 8)
//     k_laswp: the panel's interchanges on the columns outside it
//     leaf TRSM: U12 = L11^-1 A12
//     GEMM: A22 -= L21 U12 (K = 64)
// P_i B_i = L_i U_i; P_i is folded into the restriction gather index, so
// the solves need no interchanges.
//
// Complex GEMM on MFMA: with A stored as interleaved (re, im) along K, a real
// 16x16x4 MFMA over two complex K entries gives Re(C) when B's fragment is
// (Re b, -Im b) and Im(C) when it is (Im b, Re b); two MFMAs per 2 complex K,
// no wasted work.  FP32 path: v_mfma_f32_16x16x4f32; FP64: v_mfma_f64_16x16x4f64.
#include "kernels.hpp"

namespace mw {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <class R> struct Mf;
template <> struct Mf<float> {
  using acc = floatx4;
  static __device__ inline acc mfma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element r of lane l sits at row 4*(l/16) + r, column l%16
  static __device__ inline int out_row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mf<double> {
  using acc = doublex4;
  static __device__ inline acc mfma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element r of lane l sits at row (l/16) + 4*r, column l%16
  static __device__ inline int out_row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int TB = 64;    // output tile (complex) per workgroup: TB x TB
constexpr int BK = 16;    // complex K per LDS stage
constexpr int NB = 64;    // LU panel width and TRSM leaf size
constexpr int W0 = 8;     // LU sub-panel width
constexpr int NB2 = 256;  // LU outer block: the trailing update runs once per NB2 columns (K = NB2)

// C[M x N] (ldc) = (OVERWRITE ? 0 : C) - A[M x K] (lda) * B[K x N] (ldb), for the
// output tile (tm, tn); 256 threads = 4 waves, each a 32 x 32 complex quadrant.
template <class R, bool OVERWRITE>
__device__ inline void gemm_tile(const typename cplx<R>::t* __restrict__ A, int64_t lda,
                                 const typename cplx<R>::t* __restrict__ B, int64_t ldb,
                                 typename cplx<R>::t* __restrict__ Cm, int64_t ldc, int M, int N, int K,
                                 int tm, int tn) {
  using C = typename cplx<R>::t;
  using acc_t = typename Mf<R>::acc;
  __shared__ R As[TB][2 * BK + 1];
  __shared__ C Bs[BK][TB + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, kq = lane >> 4;
  const int row0 = tm * TB, col0 = tn * TB;
  acc_t accr[2][2], acci[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) { accr[a][b][r] = 0; acci[a][b][r] = 0; }

  for (int k0 = 0; k0 < K; k0 += BK) {
    // A tile: TB rows x BK complex; consecutive threads -> consecutive k in a row
    for (int e = 0; e < 4; ++e) {
      int idx = tid + e * 256;
      int r = idx >> 4, kc = idx & 15;
      int gr = row0 + r, gk = k0 + kc;
      C v;
      v.x = 0; v.y = 0;
      if (gr < M && gk < K) v = A[(int64_t)gr * lda + gk];
      As[r][2 * kc] = v.x;
      As[r][2 * kc + 1] = v.y;
    }
    // B tile: BK rows x TB complex; consecutive threads -> consecutive columns
    for (int e = 0; e < 4; ++e) {
      int idx = tid + e * 256;
      int r = idx >> 6, c = idx & 63;
      int gk = k0 + r, gc = col0 + c;
      C v;
      v.x = 0; v.y = 0;
      if (gk < K && gc < N) v = B[(int64_t)gk * ldb + gc];
      Bs[r][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      R a[2], br[2], bi[2];
#pragma unroll
      for (int bi_ = 0; bi_ < 2; ++bi_) a[bi_] = As[wm * 32 + bi_ * 16 + li][2 * kk + kq];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        C b = Bs[kk + (kq >> 1)][wn * 32 + bj * 16 + li];
        bool odd = kq & 1;
        br[bj] = odd ? -b.y : b.x;
        bi[bj] = odd ? b.x : b.y;
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          accr[x][y] = Mf<R>::mfma(a[x], br[y], accr[x][y]);
          acci[x][y] = Mf<R>::mfma(a[x], bi[y], acci[x][y]);
        }
    }
    __syncthreads();
  }
  // epilogue
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gr = row0 + wm * 32 + x * 16 + Mf<R>::out_row(lane, r);
        int gc = col0 + wn * 32 + y * 16 + li;
        if (gr < M && gc < N) {
          C* p = Cm + (int64_t)gr * ldc + gc;
          C o;
          if (OVERWRITE) { o.x = -accr[x][y][r]; o.y = -acci[x][y][r]; }
          else { o = *p; o.x -= accr[x][y][r]; o.y -= acci[x][y][r]; }
          *p = o;
        }
      }
}

// LU-internal update of subdomain blockIdx.y:
// F[r0:np, c0:min(c1,np)] -= F[r0:np, k0:k1] * F[k0:k1, c0:min(c1,np)]
// LOWER: only tiles on or below the diagonal (r0 == c0; symmetric factorisation)
// (k0 a multiple of 64 and k1 - k0 <= 64: the K rows lie in one 64-row block)
template <class R, bool LOWER = false>
__global__ void __launch_bounds__(256) k_gemm_lu(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                 const int32_t* __restrict__ n_pad, int r0, int k0, int k1,
                                                 int c0, int c1, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride,
                                                 const int32_t* __restrict__ fenv = nullptr, int fstride = 0) {
  using C = typename cplx<R>::t;
  int i = blockIdx.y;
  int np = n_pad[i];
  int M = np - r0;
  int N = min(c1, np) - c0;
  if (M <= 0 || N <= 0 || k1 > np) return;
  int tiles_n = (N + TB - 1) / TB;
  int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  if (tm * TB >= M) return;
  if (LOWER && r0 + tm * TB + TB <= c0 + tn * TB) return;
  if (fenv) {
    // no interchanges: L[r, k] and U[k, c] vanish for k below the envelope
    // start of row r and of column c (64-row/column tiles lie inside np)
    const int32_t* fe = fenv + (int64_t)i * fstride;
    const int gr = (r0 + tm * TB) / 32, gc = (c0 + tn * TB) / 32;
    if (max(min(fe[gr], fe[gr + 1]), min(fe[gc], fe[gc + 1])) >= k1) return;
  }
  C* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  const int row = r0 + tm * TB, col = c0 + tn * TB;
  C* Ar = frow(Fi, bo, bl, bwi, row);
  gemm_tile<R, false>(Ar + k0, bwi[row >> 6], frow(Fi, bo, bl, bwi, k0) + col, bwi[k0 >> 6], Ar + col,
                      bwi[row >> 6], M - tm * TB, N - tn * TB, k1 - k0, 0, 0);
}

// Wide tile for the triangular-solve updates: C[64 x 32*WC] -= A[64 x K] B[K x 32*WC]
// (or C = A B).  Four waves in a 2 x 2 arrangement, each owning 32 rows x
// 16*WC columns (2 x WC MFMA blocks); every right-hand-side column of the
// tile is in one workgroup, so each factor block (A) is read once per
// launch.  K advances by WBK complex per stage through double-buffered LDS:
// the next stage is fetched into registers while the current one is
// multiplied, then written to the other buffer (one barrier per stage).
// AMODE 0: A as stored; 1: unit lower triangle of A (strict part stored,
// implicit ones); 2: upper triangle of A with its diagonal.  OVERWRITE:
// C = A B (B may alias C: all B rows of the tile are read before the
// epilogue writes).
constexpr int WBK = 8;    // complex K per stage
template <class R, int WC, int AMODE = 0, bool OVERWRITE = false, bool NEG = false>
__device__ __attribute__((always_inline)) inline void gemm_wide(const typename cplx<R>::t* __restrict__ A, int64_t lda,
                                 const typename cplx<R>::t* B, int64_t ldb,
                                 typename cplx<R>::t* Cm, int64_t ldc, int M, int N, int K) {
  using C = typename cplx<R>::t;
  using acc_t = typename Mf<R>::acc;
  constexpr int TM = 64, TN = 32 * WC;
  constexpr int AREG = TM * WBK / 256;
  constexpr int BREG = (WBK * TN + 255) / 256;
  __shared__ R As[2][TM][2 * WBK + 1];
  __shared__ C Bs[2][WBK][TN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, kq = lane >> 4;
  acc_t accr[2][WC], acci[2][WC];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < WC; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) { accr[x][y][r] = 0; acci[x][y][r] = 0; }
  C ra[AREG], rb[BREG];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < AREG; ++e) {
      int idx = tid + e * 256;
      int r = idx / WBK, kc = idx % WBK;
      const int kk = k0 + kc;
      C v;
      v.x = 0; v.y = 0;
      if (r < M && kk < K) {
        if (AMODE == 0 || (AMODE == 1 && kk < r) || (AMODE == 2 && kk >= r)) v = A[(int64_t)r * lda + kk];
        else if (AMODE == 1 && kk == r) v.x = 1;
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < BREG; ++e) {
      int idx = tid + e * 256;
      int r = idx / TN, c = idx % TN;
      C v;
      v.x = 0; v.y = 0;
      if (idx < WBK * TN && k0 + r < K && c < N) v = B[(int64_t)(k0 + r) * ldb + c];
      rb[e] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AREG; ++e) {
      int idx = tid + e * 256;
      int r = idx / WBK, kc = idx % WBK;
      As[buf][r][2 * kc] = ra[e].x;
      As[buf][r][2 * kc + 1] = ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < BREG; ++e) {
      int idx = tid + e * 256;
      if (idx < WBK * TN) Bs[buf][idx / TN][idx % TN] = rb[e];
    }
  };
  fetch(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += WBK) {
    const bool more = k0 + WBK < K;
    if (more) fetch(k0 + WBK);
#pragma unroll
    for (int kk = 0; kk < WBK; kk += 2) {
      R a[2], br[WC], bi[WC];
#pragma unroll
      for (int x = 0; x < 2; ++x) a[x] = As[buf][wm * 32 + x * 16 + li][2 * kk + kq];
#pragma unroll
      for (int y = 0; y < WC; ++y) {
        C b = Bs[buf][kk + (kq >> 1)][wn * 16 * WC + y * 16 + li];
        bool odd = kq & 1;
        br[y] = odd ? -b.y : b.x;
        bi[y] = odd ? b.x : b.y;
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < WC; ++y) {
          accr[x][y] = Mf<R>::mfma(a[x], br[y], accr[x][y]);
          acci[x][y] = Mf<R>::mfma(a[x], bi[y], acci[x][y]);
        }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < WC; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gr = wm * 32 + x * 16 + Mf<R>::out_row(lane, r);
        int gc = wn * 16 * WC + y * 16 + li;
        if (gr < M && gc < N) {
          C* p = Cm + (int64_t)gr * ldc + gc;
          C o;
          if (OVERWRITE && NEG) { o.x = -accr[x][y][r]; o.y = -acci[x][y][r]; }
          else if (OVERWRITE) { o.x = accr[x][y][r]; o.y = acci[x][y][r]; }
          else { o = *p; o.x -= accr[x][y][r]; o.y -= acci[x][y][r]; }
          *p = o;
        }
      }
}

// Complex product by the 3M (Gauss) form: with P1 = Ar Br, P2 = Ai Bi and
// P3 = (Ar + Ai)(Br + Bi) (three real 16x16x4 MFMA products, K = 4 complex per
// instruction), Re = P1 - P2 and Im = P3 - P1 - P2: 3/4 of the real MFMA work of
// the 4M form.  Its rounding error in the imaginary part is bounded by the
// working precision times (|Ar| + |Ai|)(|Br| + |Bi|) instead of |A||B|.  Used
// for the triangular-solve updates (FP32 and FP64) and the FP32 LU trailing
// update; the LU panels keep 4M.
// Tile: 32*RB rows x 32*WC columns, waves 2 x 2 (16*RB rows x 16*WC columns
// each), C -= A B, double-buffered LDS stages of G3K complex.  RB = 2 halves
// the B reads per product at the cost of occupancy (long K pays for it).
// FULL: M, N, K are known to be multiples of the tile (no bounds tests).
constexpr int G3K = 8;
// Rows of B taken from banded factor storage: B row k (0-based) is factor row
// r0 + k, columns c0 + c; entries outside the stored columns of their block
// read as zero.
template <class C>
struct BandRows {
  const C* Fi = nullptr;
  const int64_t* boff = nullptr;
  const int32_t* blo = nullptr;
  const int32_t* bw = nullptr;
  int r0 = 0, c0 = 0;
  // the rows [k, k + 8) of one K stage (r0 + k a multiple of 8) lie in one
  // 64-row block: its base (element (row, c) at base[(row - r0 - k) * w + c0
  // + c]) and stored column range, once per stage
  struct Stage {
    const C* base;
    int lo, w;
  };
  __device__ inline Stage stage(int k) const {
    const int r = r0 + k, b = r >> 6;
    const int lo = blo[b], w = bw[b];
    return {Fi + boff[b] + (int64_t)(r & 63) * w - lo, lo, w};
  }
  __device__ inline C at(const Stage& s, int kk, int c) const {
    const int gc = c0 + c;
    C v;
    v.x = 0;
    v.y = 0;
    if (gc >= s.lo && gc < s.lo + s.w) v = s.base[(int64_t)kk * s.w + gc];
    return v;
  }
};
template <class R, int WC, int RB = 1, bool FULL = false, bool BBAND = false>
__device__ __attribute__((always_inline)) inline void gemm3m(const typename cplx<R>::t* __restrict__ A, int64_t lda,
                                                             const typename cplx<R>::t* B, int64_t ldb,
                                                             typename cplx<R>::t* Cm, int64_t ldc, int M, int N,
                                                             int K,
                                                             BandRows<typename cplx<R>::t> bb = {}) {
  using C = typename cplx<R>::t;
  using acc_t = typename Mf<R>::acc;
  constexpr int TM = 32 * RB, TN = 32 * WC;
  constexpr int AREG = TM * G3K / 256;
  constexpr int BREG = (G3K * TN + 255) / 256;
  // B rows padded by 16 elements: the four K rows a wave reads at once start
  // in different halves of the LDS banks
  __shared__ R As[2][3][TM][G3K + 1];
  __shared__ R Bs[2][3][G3K][TN + 16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, kq = lane >> 4;
  acc_t p1[RB][WC], p2[RB][WC], p3[RB][WC];
#pragma unroll
  for (int x = 0; x < RB; ++x)
#pragma unroll
    for (int y = 0; y < WC; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) { p1[x][y][r] = 0; p2[x][y][r] = 0; p3[x][y][r] = 0; }
  C ra[AREG], rb[BREG];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < AREG; ++e) {
      int idx = tid + e * 256;
      int r = idx / G3K, kc = idx % G3K;
      C v;
      v.x = 0;
      v.y = 0;
      if (FULL || (r < M && k0 + kc < K)) v = A[(int64_t)r * lda + k0 + kc];
      ra[e] = v;
    }
    typename BandRows<C>::Stage bs{};
    if constexpr (BBAND) bs = bb.stage(k0);
#pragma unroll
    for (int e = 0; e < BREG; ++e) {
      int idx = tid + e * 256;
      int r = idx / TN, c = idx % TN;
      C v;
      v.x = 0;
      v.y = 0;
      if (idx < G3K * TN && (FULL || (k0 + r < K && c < N))) {
        if constexpr (BBAND) v = bb.at(bs, r, c);
        else v = B[(int64_t)(k0 + r) * ldb + c];
      }
      rb[e] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AREG; ++e) {
      int idx = tid + e * 256;
      int r = idx / G3K, kc = idx % G3K;
      As[buf][0][r][kc] = ra[e].x;
      As[buf][1][r][kc] = ra[e].y;
      As[buf][2][r][kc] = ra[e].x + ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < BREG; ++e) {
      int idx = tid + e * 256;
      if (idx < G3K * TN) {
        int r = idx / TN, c = idx % TN;
        Bs[buf][0][r][c] = rb[e].x;
        Bs[buf][1][r][c] = rb[e].y;
        Bs[buf][2][r][c] = rb[e].x + rb[e].y;
      }
    }
  };
  fetch(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += G3K) {
    const bool more = k0 + G3K < K;
    if (more) fetch(k0 + G3K);
#pragma unroll
    for (int kk = 0; kk < G3K; kk += 4) {
      R a1[RB], a2[RB], a3[RB];
#pragma unroll
      for (int x = 0; x < RB; ++x) {
        const int row = wm * 16 * RB + x * 16 + li;
        a1[x] = As[buf][0][row][kk + kq];
        a2[x] = As[buf][1][row][kk + kq];
        a3[x] = As[buf][2][row][kk + kq];
      }
#pragma unroll
      for (int y = 0; y < WC; ++y) {
        const int col = wn * 16 * WC + y * 16 + li;
        const R b1 = Bs[buf][0][kk + kq][col], b2 = Bs[buf][1][kk + kq][col], b3 = Bs[buf][2][kk + kq][col];
#pragma unroll
        for (int x = 0; x < RB; ++x) {
          p1[x][y] = Mf<R>::mfma(a1[x], b1, p1[x][y]);
          p2[x][y] = Mf<R>::mfma(a2[x], b2, p2[x][y]);
          p3[x][y] = Mf<R>::mfma(a3[x], b3, p3[x][y]);
        }
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int x = 0; x < RB; ++x)
#pragma unroll
    for (int y = 0; y < WC; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gr = wm * 16 * RB + x * 16 + Mf<R>::out_row(lane, r);
        int gc = wn * 16 * WC + y * 16 + li;
        if (FULL || (gr < M && gc < N)) {
          C* p = Cm + (int64_t)gr * ldc + gc;
          C o = *p;
          o.x -= p1[x][y][r] - p2[x][y][r];
          o.y -= p3[x][y][r] - p1[x][y][r] - p2[x][y][r];
          *p = o;
        }
      }
}

// rows per tile of the triangular-solve updates (3M form)
template <class R, int RB = 1> struct XTile { static constexpr int TM = 32 * RB; };

// Triangular-solve update on the local multi-vector of every subdomain:
// Y[r0:min(r1,np)] -= F[r0:min(r1,np), k0:min(k1,np)] * Y[k0:min(k1,np)].
// 1-D grid of nsub * tiles_per_sub (padded to a multiple of 8) workgroups;
// the linear id is remapped so that the tiles of one subdomain run on one XCD
// (workgroups are dealt to the 8 XCDs round-robin) and share its L2.
template <class R, int WC, int RB, bool FULL = false>
__global__ void __launch_bounds__(256, (sizeof(R) == 8 && WC >= 2) ? 2 : RB) k_gemm_x(const typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                const int32_t* __restrict__ n_pad,
                                                const int64_t* __restrict__ loc_off, typename cplx<R>::t* Y,
                                                int64_t ld, int ncols, int r0, int r1, int k0, int k1,
                                                int tiles_m, int tiles_n, int nsub,
                                                const int32_t* __restrict__ row_lo,
                                                const int2* __restrict__ env, int env_stride, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  using C = typename cplx<R>::t;
  const int per_sub = tiles_m * tiles_n;
  const int G = gridDim.x;
  const int logical = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int i = logical / per_sub;
  if (i >= nsub) return;
  const int t = logical % per_sub;
  const int tm = t / tiles_n, tn = t % tiles_n;
  const int np = n_pad[i];
  const int M = min(r1, np) - r0 - tm * XTile<R, RB>::TM;
  if (M <= 0) return;
  constexpr int TM = XTile<R, RB>::TM;
  const int row = r0 + tm * TM;
  if (row_lo && row + TM <= row_lo[i]) return;   // rows discarded by the weights
  // inner dimension clipped to the envelope of the tile's rows (row < np,
  // both multiples of TM, so the tile's 32-row groups exist)
  int kb = k0, ke = min(k1, np);
  if (env) {
#pragma unroll
    for (int q = 0; q < TM / 32; ++q) {
      const int2 e = env[(int64_t)i * env_stride + row / 32 + q];
      kb = q == 0 ? max(k0, e.x) : min(kb, max(k0, e.x));
      ke = q == 0 ? min(ke, e.y) : max(ke, min(min(k1, np), e.y));
    }
  }
  const int K = ke - kb;
  if (K <= 0) return;
  const int TN = WC * 32;
  const int N = min(ncols - tn * TN, TN);
  const C* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  C* Yi = Y + loc_off[i] * ld;
  // the tile's rows lie in one 64-row block; the clipped inner range lies in
  // the stored columns of that block
  gemm3m<R, WC, RB, FULL>(frow(Fi, bo, bl, bwi, row) + kb, bwi[row >> 6], Yi + (int64_t)kb * ld + tn * TN, ld,
                          Yi + (int64_t)row * ld + tn * TN, ld, M, N, K);
}

// Leaf of the blocked triangular solves: Y[r0:r0+64] = T^-1 Y[r0:r0+64] with the
// inverted diagonal block (AMODE 1: L^-1, 2: U^-1), in place, all columns.
template <class R, int WC, int AMODE>
__global__ void __launch_bounds__(256) k_leaf_x(const typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                const int32_t* __restrict__ n_pad,
                                                const int64_t* __restrict__ loc_off, typename cplx<R>::t* Y,
                                                int64_t ld, int ncols, int r0, int tiles_n, int nsub,
                                                const int32_t* __restrict__ row_lo, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  using C = typename cplx<R>::t;
  const int G = gridDim.x;
  const int logical = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int i = logical / tiles_n;
  if (i >= nsub) return;
  const int tn = logical % tiles_n;
  const int np = n_pad[i];
  if (r0 >= np || (row_lo && r0 < row_lo[i])) return;
  const int TN = WC * 32;
  const int N = min(ncols - tn * TN, TN);
  const C* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  const C* blk = frow(Fi, bo, bl, bwi, r0) + r0;
  C* Yb = Y + (loc_off[i] + r0) * ld + tn * TN;
  gemm_wide<R, WC, AMODE, true>(blk, bwi[r0 >> 6], Yb, ld, Yb, ld, NB, N, NB);
}

// Block-row form of the triangular solves (every batch of more than one
// subdomain).  After the factorisation each 64-row block b keeps, beside its
// inverted diagonal blocks T_L = L_bb^-1 and T_U = U_bb^-1, the scaled
// off-diagonal rows S_L = -T_L L[b, :64b] and S_U = -T_U U[b, 64b+64:]
// (k_scale_offdiag, once per factorisation).  A solve is then one product per
// block and direction, the diagonal solve folded in:
//   forward,  b = 0, 1, ...:  Y_b <- T_L Y_b + S_L Y[lo:64b]
//   backward, b = last, ...:  Y_b <- T_U Y_b + S_U Y[64b+64:hi]
// ([lo, hi) the envelope of the block's rows), each Y_b written once per
// direction.  One workgroup owns a 64-row block and a column tile, so it
// alone reads the old Y_b and writes the new one.

// S_L (UPPER false) or S_U (UPPER true) of block blockIdx.x of subdomain
// blockIdx.y, in place, 64 columns at a time, over the envelope of the
// block's rows (the rest is zero before and after).
template <class R, bool UPPER>
__global__ void __launch_bounds__(256) k_scale_offdiag(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                       const int32_t* __restrict__ n_pad,
                                                       const int2* __restrict__ env, int env_stride,
                                                       const int64_t* __restrict__ boff,
                                                       const int32_t* __restrict__ blo,
                                                       const int32_t* __restrict__ bw, int bstride) {
  const int b = blockIdx.x, i = blockIdx.y;
  const int np = n_pad[i];
  const int r0 = b * NB;
  if (r0 >= np) return;
  const int2 e0 = env[(int64_t)i * env_stride + 2 * b], e1 = env[(int64_t)i * env_stride + 2 * b + 1];
  auto* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  auto* row = frow(Fi, bo, bl, bwi, r0);
  const int ld = bwi[b];
  const auto* T = row + r0;
  if (!UPPER) {
    for (int c = min(e0.x, e1.x) & ~63; c < r0; c += NB)
      gemm_wide<R, 2, 1, true, true>(T, ld, row + c, ld, row + c, ld, NB, NB, NB);
  } else {
    const int hi = min(np, (max(e0.y, e1.y) + 63) & ~63);
    for (int c = r0 + NB; c < hi; c += NB) gemm_wide<R, 2, 2, true, true>(T, ld, row + c, ld, row + c, ld, NB, NB, NB);
  }
}

// The product of one block of the block-row solves, C = A B over a 64-row
// block and up to 32 WC columns, in the 3M form of gemm3m.  A's columns
// [kd, kd + 64) hold the inverted diagonal block, read as unit lower (amode
// 1: strict lower part, ones on the diagonal) or upper with diagonal (amode
// 2).  The operands stay in LDS as complex pairs: one 64-bit (FP32) LDS read
// gives a value's real and imaginary parts, and their sum is formed in
// registers (a third of the LDS reads and writes of gemm3m's three real
// arrays; 3.5 ms less per preconditioner application on the 1 GHz chamber
// at 160 columns).  C aliases B's first or last 64 rows; every B read
// precedes the first C write.
template <class R, int WC, int WNW = 2>
__device__ __attribute__((always_inline)) inline void gemm3m_pairs(const typename cplx<R>::t* __restrict__ A,
                                                                   int64_t lda, const typename cplx<R>::t* B,
                                                                   int64_t ldb, typename cplx<R>::t* Cm, int64_t ldc,
                                                                   int N, int K, int kd, int amode) {
  using C = typename cplx<R>::t;
  using acc_t = typename Mf<R>::acc;
  // WNW waves along N (2: 32-row, 16 WC-column wave tiles; 1: 16-row wave
  // tiles over all TN = 16 WC columns)
  constexpr int WMW = 4 / WNW, RB = 4 / WMW, TM = 64, TN = 16 * WC * WNW, KS = G3K;
  constexpr int AREG = TM * KS / 256;
  constexpr int BREG = (KS * TN + 255) / 256;
  __shared__ C As[2][TM][KS + 1];
  __shared__ C Bs[2][KS][TN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WNW, wn = wave % WNW;
  const int li = lane & 15, kq = lane >> 4;
  const bool lower = amode == 1;
  acc_t p1[RB][WC], p2[RB][WC], p3[RB][WC];
#pragma unroll
  for (int x = 0; x < RB; ++x)
#pragma unroll
    for (int y = 0; y < WC; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) { p1[x][y][r] = 0; p2[x][y][r] = 0; p3[x][y][r] = 0; }
  // Software pipeline: A (the factor rows, streamed from HBM) is requested
  // two stages ahead into two alternating register sets, B (rows of Y,
  // mostly in L2) one stage ahead.  Every load is unconditional (the
  // requests past the last stage repeat its addresses; columns past N read
  // column N - 1), and the diagonal block's masking and the zero columns are
  // applied when the registers are written to LDS, so the only waits are at
  // those writes.
  C ra0[AREG], ra1[AREG], rb[BREG];
  int aoff[AREG], boff[BREG];
#pragma unroll
  for (int e = 0; e < AREG; ++e) {
    const int idx = tid + e * 256;
    aoff[e] = (idx / KS) * (int)lda + idx % KS;
  }
#pragma unroll
  for (int e = 0; e < BREG; ++e) {
    const int idx = min(tid + e * 256, KS * TN - 1);
    boff[e] = (idx / TN) * (int)ldb + min(idx % TN, N - 1);
  }
  auto fetch_a = [&](int k0, C(&dst)[AREG]) {
    const C* Ak = A + k0;
#pragma unroll
    for (int e = 0; e < AREG; ++e) dst[e] = Ak[aoff[e]];
  };
  auto fetch_b = [&](int k0) {
    const C* Bk = B + (int64_t)k0 * ldb;
#pragma unroll
    for (int e = 0; e < BREG; ++e) rb[e] = Bk[boff[e]];
  };
  // LDS buffer buf <- stage k0 (A from src, B from rb)
  auto store = [&](int buf, const C(&src)[AREG], int k0) {
    const bool tstage = k0 + KS > kd && k0 < kd + 64;   // same for the whole workgroup
#pragma unroll
    for (int e = 0; e < AREG; ++e) {
      const int idx = tid + e * 256;
      const int r = idx / KS, kc = idx % KS;
      C v = src[e];
      if (tstage) {
        const int j = k0 + kc - kd;
        if (j >= 0 && j < 64 && !(lower ? j < r : j >= r)) {
          v.x = (lower && j == r) ? 1 : 0;
          v.y = 0;
        }
      }
      As[buf][r][kc] = v;
    }
#pragma unroll
    for (int e = 0; e < BREG; ++e) {
      const int idx = tid + e * 256;
      if ((KS * TN) % 256 != 0 && idx >= KS * TN) break;
      C v = rb[e];
      if (idx % TN >= N) {
        v.x = 0;
        v.y = 0;
      }
      Bs[buf][idx / TN][idx % TN] = v;
    }
  };
  // stage k0 in LDS buffer buf: request B of the next stage and A of the
  // one after (into a_next, whose stage is already in LDS), multiply, then
  // write the next stage (A from a_stage) to the other buffer, which every
  // wave finished reading before the previous barrier
  auto step = [&](int k0, int buf, const C(&a_stage)[AREG], C(&a_next)[AREG]) {
    fetch_b(min(k0 + KS, K - KS));
    fetch_a(min(k0 + 2 * KS, K - KS), a_next);
    // the inverted diagonal block is triangular: its columns on the far
    // side of a wave's rows are zero (unit lower: columns past the wave's
    // last row; upper: columns before its first row), so the wave skips
    // those stages' products and leaves the matrix units to the other
    // workgroups on its SIMD
    constexpr int RW = 16 * RB;   // rows per wave
    const bool zero_t = (lower && k0 >= kd + RW * (wm + 1) && k0 < kd + 64) ||
                        (!lower && k0 >= kd && k0 + KS <= kd + RW * wm);
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      if (zero_t || k0 >= K) break;
      R a1[RB], a2[RB], a3[RB];
#pragma unroll
      for (int x = 0; x < RB; ++x) {
        const C av = As[buf][wm * 16 * RB + x * 16 + li][kk + kq];
        a1[x] = av.x;
        a2[x] = av.y;
        a3[x] = av.x + av.y;
      }
#pragma unroll
      for (int y = 0; y < WC; ++y) {
        const C bv = Bs[buf][kk + kq][wn * 16 * WC + y * 16 + li];
        const R b1 = bv.x, b2 = bv.y, b3 = bv.x + bv.y;
#pragma unroll
        for (int x = 0; x < RB; ++x) {
          p1[x][y] = Mf<R>::mfma(a1[x], b1, p1[x][y]);
          p2[x][y] = Mf<R>::mfma(a2[x], b2, p2[x][y]);
          p3[x][y] = Mf<R>::mfma(a3[x], b3, p3[x][y]);
        }
      }
    }
    store(buf ^ 1, a_stage, k0 + KS);
    __syncthreads();
  };
  // K is a multiple of KS (a difference of multiples of 8), at least 64
  fetch_a(0, ra0);
  fetch_b(0);
  store(0, ra0, 0);
  fetch_a(KS, ra1);
  __syncthreads();
  // stages in pairs, so that each register set keeps its role; with an odd
  // number of stages the last pair's second stage lies past K and only
  // loads (in range, clamped), writes LDS and waits
  for (int k0 = 0; k0 < K; k0 += 2 * KS) {
    step(k0, 0, ra1, ra0);
    step(k0 + KS, 1, ra0, ra1);
  }
#pragma unroll
  for (int x = 0; x < RB; ++x)
#pragma unroll
    for (int y = 0; y < WC; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = wm * 16 * RB + x * 16 + Mf<R>::out_row(lane, r);
        const int gc = wn * 16 * WC + y * 16 + li;
        if (gc < N) {
          C o;
          o.x = p1[x][y][r] - p2[x][y][r];
          o.y = p3[x][y][r] - p1[x][y][r] - p2[x][y][r];
          Cm[(int64_t)gr * ldc + gc] = o;
        }
      }
}

// Both sweeps in one launch: every workgroup takes one (subdomain, column
// tile) and runs its forward blocks, then its backward blocks, reading back
// the rows it has just written (a workgroup barrier between blocks orders
// them).  Subdomains are independent, so no workgroup waits for another; the
// few hundred rows of the moving window stay in the caches between
// consecutive blocks, and the forward sweep's last rows are the backward
// sweep's first.  Workgroup g runs on XCD g mod 8 (round-robin dispatch):
// XCD x takes the subdomains of rank x, x + 8, x + 16, ... in decreasing
// size (order[]), all column tiles of one subdomain on one XCD, so the
// longest sweeps start first and the XCDs get alike shares.
template <class R, int WC, int DIRS, int WNW = 2>
__global__ void __launch_bounds__(256, 2) k_row_sweep(const typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                      const int32_t* __restrict__ n_pad,
                                                      const int64_t* __restrict__ loc_off, typename cplx<R>::t* Y,
                                                      int64_t ld, int ncols, int tiles_n, int nsub,
                                                      const int32_t* __restrict__ order,
                                                      const int32_t* __restrict__ row_lo,
                                                      const int2* __restrict__ env, int env_stride,
                                                      const int64_t* __restrict__ boff,
                                                      const int32_t* __restrict__ blo,
                                                      const int32_t* __restrict__ bw, int bstride) {
  using C = typename cplx<R>::t;
  const int x = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int rank = 8 * (q / tiles_n) + x;
  if (rank >= nsub) return;
  const int i = order[rank];
  const int tn = q % tiles_n;
  const int np = n_pad[i];
  const int nblk = np / NB;
  constexpr int TN = WC * 16 * WNW;
  const int N = min(ncols - tn * TN, TN);
  const C* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  const int2* ei = env + (int64_t)i * env_stride;
  C* Yi = Y + loc_off[i] * ld + tn * TN;
  // blocks of the backward sweep: the last down to the one holding row_lo
  const int nbwd = nblk - (row_lo ? row_lo[i] / NB : 0);
  const int nsteps = ((DIRS & 1) ? nblk : 0) + ((DIRS & 2) ? nbwd : 0);
  // one product per step (one call site, so that both directions share its
  // LDS): forward Y_b <- T_L Y_b + S_L Y[lo:64b], b = 0, 1, ...; backward
  // Y_b <- T_U Y_b + S_U Y[64b+64:hi], b = last, ...
  for (int s = 0; s < nsteps; ++s) {
    const bool fwd = (DIRS & 1) && s < nblk;
    const int b = fwd ? s : nblk - 1 - (s - ((DIRS & 1) ? nblk : 0));
    const int r0 = b * NB;
    const int2 e0 = ei[2 * b], e1 = ei[2 * b + 1];
    const int kb = fwd ? min(min(e0.x, e1.x), r0) : r0;
    const int ke = fwd ? r0 + NB : min(np, max(max(e0.y, e1.y), r0 + NB));
    gemm3m_pairs<R, WC, WNW>(frow(Fi, bo, bl, bwi, r0) + kb, bwi[b], Yi + (int64_t)kb * ld, ld, Yi + (int64_t)r0 * ld,
                        ld, N, ke - kb, r0 - kb, fwd ? 1 : 2);
    __syncthreads();
  }
}

// LU update with wide tiles:
//   F[r0:min(r1,np), c0:min(c1,np)] -= F[r0:min(r1,np), k0:k1] F[k0:k1, c0:min(c1,np)]
// on every subdomain; 1-D XCD-aware grid of nsub * tiles_m * tiles_n.  G3
// selects the three-product complex form (64-row tiles of two row blocks per
// wave).
template <class R, int WC, bool G3>
struct LuwTile { static constexpr int TM = 64; };

template <class R, int WC, bool G3, bool LOWER = false>
__global__ void __launch_bounds__(256, G3 ? 2 : 1) k_gemm_luw(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                  const int32_t* __restrict__ n_pad, int r0, int r1, int k0, int k1,
                                                  int c0, int c1, int tiles_m, int tiles_n, int nsub,
                                                  const int32_t* __restrict__ fenv, int fstride, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  using C = typename cplx<R>::t;
  const int per_sub = tiles_m * tiles_n;
  const int G = gridDim.x;
  const int logical = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int i = logical / per_sub;
  if (i >= nsub) return;
  const int t = logical % per_sub;
  const int tm = t / tiles_n, tn = t % tiles_n;
  const int np = n_pad[i];
  constexpr int TM = LuwTile<R, WC, G3>::TM;
  const int M = min(r1, np) - r0 - tm * TM;
  const int N = min(c1, np) - c0 - tn * 32 * WC;
  if (M <= 0 || N <= 0 || k1 > np) return;
  C* Fi = F + fac_off[i];
  const int row = r0 + tm * TM, col = c0 + tn * 32 * WC;
  if (LOWER && row + TM <= col) return;   // strictly above the diagonal: not needed
  int kb = k0;
  if (fenv) {
    // no interchanges: the products L[r, k] U[k, c] of the tile vanish for k
    // below max(first envelope column of its rows, of its columns)
    const int32_t* fe = fenv + (int64_t)i * fstride;
    int fr = fe[row / 32], fc = fe[col / 32];
#pragma unroll
    for (int q = 1; q < TM / 32; ++q) fr = min(fr, fe[row / 32 + q]);
    for (int q = 1; q < WC && col + 32 * q < min(c1, np); ++q) fc = min(fc, fe[col / 32 + q]);
    kb = max(k0, max(fr, fc) & ~7);
    if (kb >= k1) return;
  }
  if constexpr (LOWER && G3) {
    // factorisation without interchanges, banded storage: the tile's rows
    // lie in one 64-row block whose stored columns hold [kb, k1); the K rows
    // (U part) span several blocks and are read through the block tables;
    // columns of the tile beyond the rows' stored range receive no update
    // (U[k, c] = 0 there for every k of the range)
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
    C* Ar = frow(Fi, bo, bl, bwi, row);
    const int ncol = min(min(N, 32 * WC), bl[row >> 6] + bwi[row >> 6] - col);
    if (ncol <= 0) return;
    BandRows<C> bb;
    bb.Fi = Fi;
    bb.boff = bo;
    bb.blo = bl;
    bb.bw = bwi;
    bb.r0 = kb;
    bb.c0 = col;
    gemm3m<R, WC, 2, false, true>(Ar + kb, bwi[row >> 6], nullptr, 0, Ar + col, bwi[row >> 6], M, ncol, k1 - kb, bb);
  } else if constexpr (G3) {
    gemm3m<R, WC, 2>(Fi + (int64_t)row * np + kb, np, Fi + (int64_t)kb * np + col, np, Fi + (int64_t)row * np + col,
                  np, M, min(N, 32 * WC), k1 - kb);
  } else {
    static_assert(!LOWER, "the factorisation without interchanges uses the three-product tiles");
    gemm_wide<R, WC>(Fi + (int64_t)row * np + kb, np, Fi + (int64_t)kb * np + col, np,
                     Fi + (int64_t)row * np + col, np, M, min(N, 32 * WC), k1 - kb);
  }
}

template <class R, int WC, bool G3 = false, bool LOWER = false>
static void launch_gemm_lu(const DeviceDecomp& d, typename cplx<R>::t* F, int r0, int r1, int k0, int k1, int c0,
                           int c1, int maxp, hipStream_t st) {
  int tiles_m = (int)ceil_div(std::min(r1, maxp) - r0, LuwTile<R, WC, G3>::TM);
  int tiles_n = (int)ceil_div(std::min(c1, maxp) - c0, 32 * WC);
  if (tiles_m <= 0 || tiles_n <= 0 || k1 <= k0) return;
  int64_t G = round_up((int64_t)d.nsub * tiles_m * tiles_n, 8);
  // envelope clipping only for the factorisation without interchanges
  k_gemm_luw<R, WC, G3, LOWER><<<(unsigned)G, 256, 0, st>>>(F, d.fac_off, d.n_pad, r0, r1, k0, k1, c0, c1,
                                                            tiles_m, tiles_n, d.nsub, LOWER ? d.fenv : nullptr,
                                                            d.fenv_stride, d.boff, d.blo, d.bw, d.bstride);
  MW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- pivot reduction
struct Piv { double v; int idx; };
__device__ inline Piv piv_max(Piv a, Piv b) {
  if (b.v > a.v || (b.v == a.v && b.idx < a.idx)) return b;
  return a;
}

// largest |re|+|im| of every B_i (scale of the singular-pivot test; NaN or
// Inf when B_i holds a non-finite entry)
template <class R>
// (only the envelope of B_i is read: every entry outside it is zero)
__global__ void __launch_bounds__(256) k_amax(const typename cplx<R>::t* __restrict__ F,
                                              const int64_t* __restrict__ fac_off, const int32_t* __restrict__ n_pad,
                                              const int32_t* __restrict__ fenv, const int32_t* __restrict__ fenv_hi,
                                              int fstride, double* __restrict__ amax, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  __shared__ double red[4];
  int i = blockIdx.x;
  const int np = n_pad[i];
  const auto* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  double m = 0.0;
  for (int g = 0; 32 * g < np; ++g) {
    const int c0 = fenv[(int64_t)i * fstride + g], w = min(fenv_hi[(int64_t)i * fstride + g], np) - c0;
    const auto* Pg = frow(Fi, bo, bl, bwi, 32 * g) + c0;   // the group's 32 rows: one block
    const int64_t ldg = bwi[g >> 1];
    // wave rows rr, rr + 4, ..., lanes along the row (no index division)
    for (int rr = threadIdx.x >> 6; rr < 32; rr += 4) {
      const auto* pr = Pg + rr * ldg;
#pragma unroll 4
      for (int k = threadIdx.x & 63; k < w; k += 64) {
        const auto v = pr[k];
        const double a = fabs((double)v.x) + fabs((double)v.y);
        m = (a > m || a != a) ? a : m;   // a NaN entry makes the maximum NaN
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(m, off);
    m = (o > m || o != o) ? o : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < 4; ++w) r = (red[w] > r || red[w] != red[w]) ? red[w] : r;
    amax[i] = r;
  }
}

// One workgroup per subdomain: factor columns [c, c+W0) of rows [c, np),
// row interchanges across the 64-wide panel [k, k+NB), then the unit-lower
// solve of rows [c, c+W0) for the panel columns [c+W0, k+NB).
// NOPIV: no interchanges (the diagonal entry is the pivot; symmetric factorisation).
template <class R, bool NOPIV = false>
__global__ void __launch_bounds__(256) k_lu_panel(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                  const int32_t* __restrict__ n_pad,
                                                  const int64_t* __restrict__ loc_off, int32_t* ipiv,
                                                  int32_t* info, const double* __restrict__ amax, double rtol,
                                                  int c, int k) {
  using C = typename cplx<R>::t;
  __shared__ Piv red[4];
  __shared__ C prow[W0];
  int i = blockIdx.x;
  int np = n_pad[i];
  if (c >= np) return;
  int kend = min(k + NB, np);
  C* Fi = F + fac_off[i];
  int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < W0; ++j) {
    int col = c + j;
    Piv best{-1.0, 0x7fffffff};
    if (NOPIV) {
      C v = Fi[(int64_t)col * np + col];
      best.v = fabs((double)v.x) + fabs((double)v.y);
      best.idx = col;
    } else {
      for (int r = col + tid; r < np; r += 256) {
        C v = Fi[(int64_t)r * np + col];
        double a = fabs((double)v.x) + fabs((double)v.y);
        if (a > best.v) { best.v = a; best.idx = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        Piv o;
        o.v = __shfl_xor(best.v, off);
        o.idx = __shfl_xor(best.idx, off);
        best = piv_max(best, o);
      }
      if (lane == 0) red[wave] = best;
      __syncthreads();
      best = piv_max(piv_max(red[0], red[1]), piv_max(red[2], red[3]));
    }
    int p = best.idx;
    // a pivot below rtol * max|B_i| marks B_i numerically singular; an exact
    // zero (or NaN) column is skipped without division
    bool zero = !(best.v > 0.0);
    bool tiny = !(best.v > rtol * amax[i]);
    if (zero) p = col;
    if (tid == 0) {
      ipiv[loc_off[i] + col] = p;
      if (tiny && info[i] == 0) info[i] = col + 1;
    }
    if (p != col)
      for (int cc = k + tid; cc < kend; cc += 256) {
        C t0 = Fi[(int64_t)col * np + cc];
        Fi[(int64_t)col * np + cc] = Fi[(int64_t)p * np + cc];
        Fi[(int64_t)p * np + cc] = t0;
      }
    __syncthreads();
    if (tid < W0) prow[tid] = Fi[(int64_t)col * np + c + tid];
    __syncthreads();
    C pv = prow[j];
    C inv;
    inv.x = 0;
    inv.y = 0;
    if (!zero) inv = cinv(pv);
    for (int r = col + 1 + tid; r < np; r += 256) {
      C* rowp = Fi + (int64_t)r * np;
      C l = cmul(rowp[col], inv);
      rowp[col] = l;
      for (int cc = j + 1; cc < W0; ++cc) rowp[c + cc] = csub(rowp[c + cc], cmul(l, prow[cc]));
    }
    __syncthreads();
  }
  // U rows of the sub-panel for the remaining panel columns (unit lower solve)
  for (int cc = c + W0 + tid; cc < kend; cc += 256) {
    C x[W0];
    for (int r = 0; r < W0; ++r) x[r] = Fi[(int64_t)(c + r) * np + cc];
    for (int r = 1; r < W0; ++r)
      for (int s = 0; s < r; ++s) x[r] = csub(x[r], cmul(Fi[(int64_t)(c + r) * np + c + s], x[s]));
    for (int r = 1; r < W0; ++r) Fi[(int64_t)(c + r) * np + cc] = x[r];
  }
}

// Register-resident form of k_lu_panel (FP32): 1024 threads hold rows
// [c, np) of the sub-panel columns [c, c+W0) in registers (row c + t + 1024 s
// in slot s of thread t, np - c <= 1024 * RPT), so every row is read and
// written once per sub-panel instead of once per column.  Pivot search,
// interchange and rank-1 updates follow k_lu_panel exactly (same pivot rule,
// same order of operations per entry).  One column step per instantiation of
// panel_reg_col, so that every register index is a compile-time constant.
struct PanelRegArgs {
  float2* Fi;
  Piv* red;
  float2 (*prow)[W0];
  int np, c, k, kend, tid;
  int32_t* ipiv_i;   // ipiv + loc_off[i]
  int32_t* info_i;   // info + i
  double thr;        // rtol * max|B_i|
};

template <int J, int RPT, bool NOPIV>
__device__ __forceinline__ void panel_reg_col(float2 (&v)[RPT][W0], const PanelRegArgs& g) {
  const int col = g.c + J, tid = g.tid;
  Piv best{-1.0, 0x7fffffff};
  if (NOPIV) {
    // the diagonal entry (row col: thread J, slot 0) is the pivot
    if (tid == J) g.red[0] = Piv{fabs((double)v[0][J].x) + fabs((double)v[0][J].y), col};
    __syncthreads();
    best = g.red[0];
  } else {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int row = g.c + tid + 1024 * s;
      if (row >= col && row < g.np) {
        const double a = fabs((double)v[s][J].x) + fabs((double)v[s][J].y);
        if (a > best.v) { best.v = a; best.idx = row; }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      Piv o;
      o.v = __shfl_xor(best.v, off);
      o.idx = __shfl_xor(best.idx, off);
      best = piv_max(best, o);
    }
    if ((tid & 63) == 0) g.red[tid >> 6] = best;
    __syncthreads();
    best = g.red[0];
    for (int w = 1; w < 16; ++w) best = piv_max(best, g.red[w]);
  }
  int p = best.idx;
  const bool zero = !(best.v > 0.0);
  const bool tiny = !(best.v > g.thr);
  if (zero) p = col;
  if (tid == 0) {
    g.ipiv_i[col] = p;
    if (tiny && *g.info_i == 0) *g.info_i = col + 1;
  }
  // rows col (thread J, slot 0) and p (thread tp, slot sp) exchange through
  // LDS; prow[0] ends as the pivot row
  const int tp = (p - g.c) & 1023, sp = (p - g.c) >> 10;
#pragma unroll
  for (int s = 0; s < RPT; ++s)
    if (tid == tp && s == sp)
#pragma unroll
      for (int q = 0; q < W0; ++q) g.prow[0][q] = v[s][q];
  if (tid == J && p != col)
#pragma unroll
    for (int q = 0; q < W0; ++q) g.prow[1][q] = v[0][q];
  if (p != col) {
    const int nout = (g.kend - g.k) - W0;   // panel columns outside [c, c+W0)
    for (int e = tid; e < nout; e += 1024) {
      int cc = g.k + e;
      if (cc >= g.c) cc += W0;
      const float2 t0 = g.Fi[(int64_t)col * g.np + cc];
      g.Fi[(int64_t)col * g.np + cc] = g.Fi[(int64_t)p * g.np + cc];
      g.Fi[(int64_t)p * g.np + cc] = t0;
    }
  }
  __syncthreads();
  if (p != col) {
    if (tid == J)
#pragma unroll
      for (int q = 0; q < W0; ++q) v[0][q] = g.prow[0][q];
#pragma unroll
    for (int s = 0; s < RPT; ++s)
      if (tid == tp && s == sp)
#pragma unroll
        for (int q = 0; q < W0; ++q) v[s][q] = g.prow[1][q];
  }
  float2 inv = make_float2(0.f, 0.f);
  if (!zero) inv = cinv(g.prow[0][J]);
  float2 u[W0];
#pragma unroll
  for (int q = J + 1; q < W0; ++q) u[q] = g.prow[0][q];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int row = g.c + tid + 1024 * s;
    if (row > col && row < g.np) {
      const float2 l = cmul(v[s][J], inv);
      v[s][J] = l;
#pragma unroll
      for (int q = J + 1; q < W0; ++q) v[s][q] = csub(v[s][q], cmul(l, u[q]));
    }
  }
  __syncthreads();
}

template <int RPT, bool NOPIV = false>
__global__ void __launch_bounds__(1024) k_lu_panel_reg(float2* F, const int64_t* __restrict__ fac_off,
                                                       const int32_t* __restrict__ n_pad,
                                                       const int64_t* __restrict__ loc_off, int32_t* ipiv,
                                                       int32_t* info, const double* __restrict__ amax, double rtol,
                                                       int c, int k) {
  static_assert(W0 == 8, "column steps are spelled out for W0 = 8");
  __shared__ Piv red[16];
  __shared__ float2 prow[2][W0];
  const int i = blockIdx.x;
  const int np = n_pad[i];
  if (c >= np) return;
  PanelRegArgs g{F + fac_off[i], red, prow, np, c, k, min(k + NB, np), (int)threadIdx.x,
                 ipiv + loc_off[i], info + i, rtol * amax[i]};
  float2 v[RPT][W0];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int row = c + g.tid + 1024 * s;
#pragma unroll
    for (int q = 0; q < W0; ++q) v[s][q] = row < np ? g.Fi[(int64_t)row * np + c + q] : make_float2(0.f, 0.f);
  }
  panel_reg_col<0, RPT, NOPIV>(v, g);
  panel_reg_col<1, RPT, NOPIV>(v, g);
  panel_reg_col<2, RPT, NOPIV>(v, g);
  panel_reg_col<3, RPT, NOPIV>(v, g);
  panel_reg_col<4, RPT, NOPIV>(v, g);
  panel_reg_col<5, RPT, NOPIV>(v, g);
  panel_reg_col<6, RPT, NOPIV>(v, g);
  panel_reg_col<7, RPT, NOPIV>(v, g);
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int row = c + g.tid + 1024 * s;
    if (row < np)
#pragma unroll
      for (int q = 0; q < W0; ++q) g.Fi[(int64_t)row * np + c + q] = v[s][q];
  }
  __syncthreads();
  // U rows of the sub-panel for the remaining panel columns (unit lower solve)
  for (int cc = c + W0 + g.tid; cc < g.kend; cc += 1024) {
    float2 x[W0];
    for (int r = 0; r < W0; ++r) x[r] = g.Fi[(int64_t)(c + r) * np + cc];
    for (int r = 1; r < W0; ++r)
      for (int q = 0; q < r; ++q) x[r] = csub(x[r], cmul(g.Fi[(int64_t)(c + r) * np + c + q], x[q]));
    for (int r = 1; r < W0; ++r) g.Fi[(int64_t)(c + r) * np + cc] = x[r];
  }
}

// interchanges of the panel [k, k+NB) on the columns outside it
template <class R>
__global__ void k_laswp(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                        const int32_t* __restrict__ n_pad, const int64_t* __restrict__ loc_off,
                        const int32_t* __restrict__ ipiv, int k) {
  using C = typename cplx<R>::t;
  int i = blockIdx.y;
  int np = n_pad[i];
  if (k >= np) return;
  int kend = min(k + NB, np);
  int ncol = np - (kend - k);
  int cc = blockIdx.x * blockDim.x + threadIdx.x;
  if (cc >= ncol) return;
  if (cc >= k) cc += kend - k;
  C* Fi = F + fac_off[i];
  const int32_t* pv = ipiv + loc_off[i];
  for (int j = k; j < kend; ++j) {
    int p = pv[j];
    if (p != j) {
      C t0 = Fi[(int64_t)j * np + cc];
      Fi[(int64_t)j * np + cc] = Fi[(int64_t)p * np + cc];
      Fi[(int64_t)p * np + cc] = t0;
    }
  }
}

// ---------------------------------------------------------------- leaf TRSM
// Solve T X = X in place for the NB x NB triangle T (unit lower, or upper with
// its diagonal) and an NB-row block X, columns [c_begin, c_end).  Each
// 16-lane group owns one column at a time and keeps its 64 rows in 4
// registers per lane (row q + 16*sl); solution entries are broadcast by lane
// shuffles.  The triangle is staged in LDS as four 16-row bands, band sl
// holding rows q + 16*sl with a per-band stride, so that every LDS access is
// a per-band base plus a compile-time offset (the loops are fully unrolled).
//   lower band sl: T[q+16sl][r], r in [0, 16sl+16),  stride 16sl+17
//   upper band sl: T[q+16sl][r], r in [16sl, 64),     stride 65-16sl
constexpr int BAND_TOTAL = 16 * (17 + 33 + 49 + 65);
__host__ __device__ constexpr int band_off(int sl, bool upper) {
  return upper ? (sl == 0 ? 0 : sl == 1 ? 16 * 65 : sl == 2 ? 16 * (65 + 49) : 16 * (65 + 49 + 33))
               : (sl == 0 ? 0 : sl == 1 ? 16 * 17 : sl == 2 ? 16 * (17 + 33) : 16 * (17 + 33 + 49));
}
__host__ __device__ constexpr int band_stride(int sl, bool upper) { return upper ? 65 - 16 * sl : 16 * sl + 17; }

template <class C>
__device__ inline C pick4(const C v[4], int sl) {
  C a = sl == 1 ? v[1] : v[0];
  C b = sl == 3 ? v[3] : v[2];
  return sl >= 2 ? b : a;
}

// IDENT: the block X starts as the identity (its old contents are not read);
// WMASK: 0 write every row, 1 only rows below the column (strict lower),
// 2 only rows on or above it (upper with diagonal).
template <class R, bool UPPER, bool IDENT = false, int WMASK = 0>
__device__ inline void trsm_leaf(const typename cplx<R>::t* __restrict__ T, int64_t ldt, typename cplx<R>::t* X,
                                 int64_t ldx, int c_begin, int c_end, typename cplx<R>::t* tri) {
  using C = typename cplx<R>::t;
  const int tid = threadIdx.x;
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    const int w = UPPER ? 64 - 16 * sl : 16 * sl + 16;    // stored columns per band row
    for (int e = tid; e < 16 * w; e += 256) {
      int q = e / w, j = e % w;
      int r = UPPER ? 16 * sl + j : j;
      tri[band_off(sl, UPPER) + q * band_stride(sl, UPPER) + j] = T[(int64_t)(q + 16 * sl) * ldt + r];
    }
  }
  __syncthreads();
  const int q = tid & 15;
  const C* band[4];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) band[sl] = tri + band_off(sl, UPPER) + q * band_stride(sl, UPPER);
  for (int colx = c_begin + (tid >> 4); colx < c_end; colx += 16) {
    C v[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      if (IDENT) { v[sl].x = (q + 16 * sl == colx) ? 1 : 0; v[sl].y = 0; }
      else v[sl] = X[(int64_t)(q + 16 * sl) * ldx + colx];
    }
    if (!UPPER) {
      for (int r = 0; r < NB; ++r) {
        const int owner = r & 15, slot = r >> 4;
        C mine = pick4(v, slot);
        C xr;
        xr.x = __shfl(mine.x, owner, 16);
        xr.y = __shfl(mine.y, owner, 16);
#pragma unroll
        for (int sl = 0; sl < 4; ++sl)
          if (q + 16 * sl > r) v[sl] = csub(v[sl], cmul(band[sl][r], xr));
      }
    } else {
      for (int r = NB - 1; r >= 0; --r) {
        const int owner = r & 15, slot = r >> 4;
        C mine = pick4(v, slot);
        C xr;
        xr.x = __shfl(mine.x, owner, 16);
        xr.y = __shfl(mine.y, owner, 16);
        // diagonal U[r][r]: band `slot`, row `owner`, column r
        C dg = tri[band_off(slot, true) + owner * band_stride(slot, true) + (r - 16 * slot)];
        xr = cmul(xr, cinv(dg));
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
          const int srow = q + 16 * sl;
          if (srow == r) v[sl] = xr;
          else if (srow < r) v[sl] = csub(v[sl], cmul(band[sl][r - 16 * sl], xr));
        }
      }
    }
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      const int srow = q + 16 * sl;
      if (WMASK == 0 || (WMASK == 1 && srow > colx) || (WMASK == 2 && srow <= colx))
        X[(int64_t)srow * ldx + colx] = v[sl];
    }
  }
}

constexpr int PANEL_COLS = 256;   // columns per workgroup of the LU panel solve

// LU: U12 = L11^-1 A12 for the panel k (rows [k, k+NB), columns [k+NB, np))
template <class R>
__global__ void __launch_bounds__(256) k_trsm_panel(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                    const int32_t* __restrict__ n_pad, int k) {
  int i = blockIdx.y;
  int np = n_pad[i];
  int c0 = k + NB;
  int cb = c0 + blockIdx.x * PANEL_COLS;
  if (cb >= np) return;
  auto* Fi = F + fac_off[i];
  __shared__ typename cplx<R>::t tri[BAND_TOTAL];
  trsm_leaf<R, false>(Fi + (int64_t)k * np + k, np, Fi + (int64_t)k * np, np, cb, min(np, cb + PANEL_COLS), tri);
}

// Symmetric factorisation, panel [k, k+NB) without interchanges: with no
// pivot search the panel is a diagonal block and an independent triangular
// solve per row block.  k_sym_diag (one workgroup per subdomain) factors the
// 64 x 64 diagonal block A_kk = L_kk U_kk in LDS (the singular-pivot test of
// the LU panels), writes both triangles back, sets the identity interchanges,
// and leaves U_kk^-1 in the block right of it (rows [k, k+NB), columns
// [k+NB, k+2NB): the future U row, overwritten afterwards by k_sym_row).
template <class R>
__global__ void __launch_bounds__(256) k_sym_diag(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                  const int32_t* __restrict__ n_pad,
                                                  const int64_t* __restrict__ loc_off, int32_t* ipiv,
                                                  int32_t* info, const double* __restrict__ amax, double rtol,
                                                  int k, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  using C = typename cplx<R>::t;
  const int i = blockIdx.x;
  const int np = n_pad[i];
  if (k >= np) return;
  C* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  __shared__ C T[NB][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  C* Pk = frow(Fi, bo, bl, bwi, k) + k;   // rows k .. k+63: one block, row stride bwi[k / 64]
  const int64_t ldk = bwi[k >> 6];
  for (int e = tid; e < NB * NB; e += 256) T[e / NB][e % NB] = Pk[(e / NB) * ldk + e % NB];
  __syncthreads();
  const double thr = rtol * amax[i];
  for (int j = 0; j < NB; ++j) {
    const C pv = T[j][j];
    const double a = fabs((double)pv.x) + fabs((double)pv.y);
    const bool zero = !(a > 0.0);
    if (tid == 0 && !(a > thr) && bad == 0) bad = k + j + 1;
    const C inv = zero ? cmk<C>(0, 0) : cinv(pv);
    // column j of L below the pivot (each thread its own rows), then the
    // rank-1 update of the trailing block
    for (int r = j + 1 + tid; r < NB; r += 256) T[r][j] = cmul(T[r][j], inv);
    __syncthreads();
    const int m = NB - 1 - j;
    for (int e = tid; e < m * m; e += 256) {
      const int r = j + 1 + e / m, c = j + 1 + e % m;
      T[r][c] = csub(T[r][c], cmul(T[r][j], T[j][c]));
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += 256) Pk[(e / NB) * ldk + e % NB] = T[e / NB][e % NB];
  if (tid < NB) ipiv[loc_off[i] + k + tid] = k + tid;
  if (tid == 0 && bad && info[i] == 0) info[i] = bad;
  if (k + 2 * NB > np) return;
  __syncthreads();
  // U_kk^-1 (upper triangular), one column per thread, by back substitution
  __shared__ C X[NB][NB + 1];
  if (tid < NB) {
    const int c = tid;
    for (int r = NB - 1; r >= 0; --r) {
      C v = cmk<C>(0, 0);
      if (r <= c) {
        v = cmk<C>(r == c ? 1 : 0, 0);
        for (int l = r + 1; l <= c; ++l) v = csub(v, cmul(T[r][l], X[l][c]));
        const C d = T[r][r];
        v = (fabs((double)d.x) + fabs((double)d.y) > 0.0) ? cmul(v, cinv(d)) : cmk<C>(0, 0);
      }
      X[r][c] = v;
    }
  }
  __syncthreads();
  // (the stored columns of every block reach at least 64 past its diagonal block)
  for (int e = tid; e < NB * NB; e += 256) Pk[(e / NB) * ldk + NB + e % NB] = X[e / NB][e % NB];
}

// L_rk = A_rk U_kk^-1 for one 64-row block r of the panel below the diagonal
// block (U_kk^-1 read from where k_sym_diag left it).
template <class R>
__global__ void __launch_bounds__(256) k_sym_cols(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                  const int32_t* __restrict__ n_pad, int k,
                                                  const int32_t* __restrict__ fenv, int fstride, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  using C = typename cplx<R>::t;
  const int i = blockIdx.y;
  const int np = n_pad[i];
  const int rb = k + NB + blockIdx.x * NB;
  if (rb >= np) return;
  // rows whose envelope starts right of the panel: A_rk = 0, L_rk stays 0
  const int32_t* fe = fenv + (int64_t)i * fstride;
  if (min(fe[rb / 32], fe[rb / 32 + 1]) >= k + NB) return;
  C* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  __shared__ C A[NB][NB + 1];
  __shared__ C U[NB][NB + 1];
  // (the row block's envelope starts left of k + NB, so its stored columns
  // begin at or before k)
  C* Pr = frow(Fi, bo, bl, bwi, rb) + k;
  const C* Pk = frow(Fi, bo, bl, bwi, k) + k + NB;
  const int64_t ldr = bwi[rb >> 6], ldk = bwi[k >> 6];
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    A[e / NB][e % NB] = Pr[(e / NB) * ldr + e % NB];
    U[e / NB][e % NB] = Pk[(e / NB) * ldk + e % NB];
  }
  __syncthreads();
  const int r = threadIdx.x >> 2, cg = threadIdx.x & 3;
  C acc[NB / 4];
#pragma unroll
  for (int u = 0; u < NB / 4; ++u) acc[u] = cmk<C>(0, 0);
#pragma unroll 4
  for (int l = 0; l < NB; ++l) {
    const C a = A[r][l];
#pragma unroll
    for (int u = 0; u < NB / 4; ++u) acc[u] = cadd(acc[u], cmul(a, U[l][cg + 4 * u]));
  }
  C* out = Pr + r * ldr + cg;
#pragma unroll
  for (int u = 0; u < NB / 4; ++u) out[4 * u] = acc[u];
}

// Symmetric factorisation (B_i = L D L^T, B_i complex symmetric, no
// interchanges): the rows [k, k+NB) of U = D L^T right of the panel are the
// scaled transpose of the panel's L columns, U[r][j] = U[r][r] L[j][r] for
// j >= k+NB, so they are written from the panel instead of being solved for
// (and the trailing updates never need the part above the diagonal).  One
// workgroup per 64 columns j, the 64 x 64 tile transposed through LDS.
template <class R>
__global__ void __launch_bounds__(256) k_sym_row(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                 const int32_t* __restrict__ n_pad, int k,
                                                 const int32_t* __restrict__ fenv, int fstride, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  using C = typename cplx<R>::t;
  const int i = blockIdx.y;
  const int np = n_pad[i];
  const int jb = k + NB + blockIdx.x * NB;
  if (jb >= np) return;
  // columns whose envelope starts below the panel: their U entries are, and
  // stay, zero; the first block always runs (it holds U_kk^-1 until now)
  const int32_t* fe = fenv + (int64_t)i * fstride;
  if (jb > k + NB && min(fe[jb / 32], fe[jb / 32 + 1]) >= k + NB) return;
  C* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  __shared__ C T[NB][NB + 1];
  __shared__ C dg[NB];
  // L[jb + jj, k + rr]: zero left of the stored columns of block jb (the
  // first block runs whatever its envelope); U rows k.. are written where
  // stored (beyond, the scaled zeros are not kept)
  const int jbk = jb >> 6, lo_j = bl[jbk];
  const C* Pj = frow(Fi, bo, bl, bwi, jb);
  const int64_t ldj = bwi[jbk];
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int jj = e / NB, rr = e % NB;
    T[jj][rr] = k + rr >= lo_j ? Pj[jj * ldj + k + rr] : cmk<C>(0, 0);
  }
  C* Pk = frow(Fi, bo, bl, bwi, k);
  const int kk = k >> 6, hi_k = bl[kk] + bwi[kk];
  const int64_t ldk = bwi[kk];
  if (threadIdx.x < NB) dg[threadIdx.x] = Pk[threadIdx.x * ldk + k + threadIdx.x];
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int rr = e / NB, jj = e % NB;
    if (jb + jj < hi_k) Pk[rr * ldk + jb + jj] = cmul(dg[rr], T[jj][rr]);
  }
}

// Every 64 x 64 diagonal block of a factored B_i is replaced by the inverses of
// its two triangles: L_bb^-1 (unit lower, strict part stored) and U_bb^-1
// (upper with diagonal) share the block, so the leaf triangular solves become
// small dense products.  U_bb is staged in LDS before any of its entries is
// overwritten; the L_bb^-1 writes touch only the strict lower part.
template <class R>
__global__ void __launch_bounds__(256) k_invert_diag(typename cplx<R>::t* F, const int64_t* __restrict__ fac_off,
                                                     const int32_t* __restrict__ n_pad, const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  int b = blockIdx.x, i = blockIdx.y;
  int np = n_pad[i];
  if (b * NB >= np) return;
  auto* Fi = F + fac_off[i];
  const int64_t* bo = boff + (int64_t)i * bstride;
  const int32_t* bl = blo + (int64_t)i * bstride;
  const int32_t* bwi = bw + (int64_t)i * bstride;
  auto* blk = frow(Fi, bo, bl, bwi, b * NB) + b * NB;
  const int ldb = bwi[b];
  __shared__ typename cplx<R>::t tri[BAND_TOTAL];
  trsm_leaf<R, false, true, 1>(blk, ldb, blk, ldb, 0, NB, tri);
  __syncthreads();
  trsm_leaf<R, true, true, 2>(blk, ldb, blk, ldb, 0, NB, tri);
}

// restriction gather index with the row interchanges folded in:
// ridx[l] = sub_dof[perm[l]], perm = interchanges applied to the identity
__global__ void __launch_bounds__(256) k_build_perm(const int32_t* __restrict__ n_pad,
                                                    const int64_t* __restrict__ loc_off,
                                                    const int32_t* __restrict__ ipiv,
                                                    const int32_t* __restrict__ sub_dof, int32_t* ridx) {
  __shared__ int32_t perm[8192];
  int i = blockIdx.x;
  int np = n_pad[i];
  int64_t o = loc_off[i];
  for (int l = threadIdx.x; l < np; l += blockDim.x) perm[l] = l;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < np; ++j) {
      int p = ipiv[o + j];
      int t = perm[j];
      perm[j] = perm[p];
      perm[p] = t;
    }
  __syncthreads();
  for (int l = threadIdx.x; l < np; l += blockDim.x) ridx[o + l] = sub_dof[o + perm[l]];
}

// Envelope of the factors: one workgroup per (subdomain, 32-row group g).
// Rows [32g, 32g+32) lie in the diagonal block b = g/2 (columns
// [64b, 64b+64), which holds the inverted diagonal factors and is excluded).
// Every wave takes 8 rows; for each it finds the first nonzero column of L
// left of the block, scanning 64 columns per step from column 0 and
// stopping at the first step with a nonzero (or at the bound already found),
// and the last nonzero column of U right of the block, scanning from the last
// column leftwards in the same way.  Entries
// outside the envelope stay exactly zero through a factorisation without
// interchanges, so skipping them changes no result; with interchanges the
// scan still sees every nonzero.
template <class C>
__global__ void __launch_bounds__(256) k_envelope(const C* __restrict__ F, const int64_t* __restrict__ fac_off,
                                                  const int32_t* __restrict__ n_pad, int stride,
                                                  const int32_t* __restrict__ fenv,
                                                  const int32_t* __restrict__ fenv_hi, int2* __restrict__ env,
                                                  const int64_t* __restrict__ boff, const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  const int i = blockIdx.x / stride, g = blockIdx.x % stride;
  const int np = n_pad[i];
  const int b0 = (g / 2) * 64, b1 = b0 + 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int lo = b0, hi = b1;
  if (32 * g < np) {
    const C* Fi = F + fac_off[i];
    const int64_t* bo = boff + (int64_t)i * bstride;
    const int32_t* bl = blo + (int64_t)i * bstride;
    const int32_t* bwi = bw + (int64_t)i * bstride;
    // without interchanges nothing lies outside the structural envelope of
    // B_i, so the scans may start at its 64-column steps (else at the edges)
    const int l0 = fenv ? min(b0, fenv[blockIdx.x] & ~63) : 0;
    const int u0 = fenv_hi ? max(b1, min(np, (fenv_hi[blockIdx.x] + 63) & ~63)) : np;
    for (int q = 0; q < 8; ++q) {
      const C* row = frow(Fi, bo, bl, bwi, 32 * g + 8 * wave + q);
      for (int c0 = l0; c0 < lo; c0 += 64) {
        const C v = row[c0 + lane];
        const unsigned long long m = __ballot(v.x != 0 || v.y != 0);
        if (m) {
          lo = min(lo, c0 + (int)__builtin_ctzll(m));
          break;
        }
      }
      for (int c0 = u0 - 64; c0 + 64 > hi; c0 -= 64) {
        const C v = row[c0 + lane];
        const unsigned long long m = __ballot(v.x != 0 || v.y != 0);
        if (m) {
          hi = max(hi, c0 + 64 - (int)__builtin_clzll(m));
          break;
        }
      }
    }
  }
  __shared__ int slo[4], shi[4];
  if (lane == 0) {
    slo[wave] = lo;
    shi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = min(lo, slo[w]);
      hi = max(hi, shi[w]);
    }
    env[blockIdx.x] = make_int2(lo & ~7, (hi + 7) & ~7);
  }
}

// Factor entries, clipped inner dimension and rows with work of the
// envelope-restricted update Y[r0:r1] -= F[r0:r1, k0:k1] Y[k0:k1] of
// subdomain i (n unknowns), 32-row groups at a time: the algorithmic work of
// one launch.
static void env_work(const DeviceDecomp& d, int i, int n, int r0, int r1, int k0, int k1, double& fac,
                     double& kspan, double& rows_work) {
  fac = 0;
  rows_work = 0;
  int kmin = k1, kmax = k0;
  r1 = std::min(r1, n);
  k1 = std::min(k1, n);
  for (int g = r0 / 32; 32 * g < r1; ++g) {
    const int2 e = d.h_env[(size_t)i * d.env_stride + g];
    const int rows = std::min(32 * g + 32, r1) - std::max(32 * g, r0);
    const int kb = std::max(k0, e.x), ke = std::min(k1, e.y);
    if (rows > 0 && ke > kb) {
      fac += (double)rows * (ke - kb);
      rows_work += rows;
      kmin = std::min(kmin, kb);
      kmax = std::max(kmax, ke);
    }
  }
  kspan = kmax > kmin ? kmax - kmin : 0;
}

// Algorithmic work of the lower-triangle update
// F[r, c] -= sum_{k in [k0, k1)} L[r, k] U[k, c], r >= r0, c in [c0, c1), c <= r,
// of subdomain i (n unknowns) inside the envelope, 32 x 32 blocks at a time:
// rows and columns with a nonzero product, entries updated, and complex
// multiply-adds.
static void fenv_work(const DeviceDecomp& d, int i, int n, int r0, int k0, int k1, int c0, int c1, double& rows,
                      double& cols, double& entries, double& macs) {
  rows = cols = entries = macs = 0;
  const int32_t* fe = d.h_fenv + (size_t)i * d.fenv_stride;
  c1 = std::min(c1, n);
  k1 = std::min(k1, n);
  if (k1 <= k0) return;
  for (int g = r0 / 32; 32 * g < n; ++g) {
    const int rg = std::min(32 * g + 32, n) - std::max(32 * g, r0);
    if (rg <= 0 || fe[g] >= k1) continue;
    bool any = false;
    for (int h = c0 / 32; 32 * h < c1 && h <= g; ++h) {
      const int ch = std::min(32 * h + 32, c1) - std::max(32 * h, c0);
      const int kb = std::max(k0, std::max(fe[g], fe[h]));
      if (ch <= 0 || kb >= k1) continue;
      const double e = h < g ? (double)rg * ch : (double)rg * (rg + 1) / 2;
      entries += e;
      macs += e * (k1 - kb);
      any = true;
    }
    if (any) rows += rg;
  }
  for (int h = c0 / 32; 32 * h < c1; ++h)
    if (fe[h] < k1) cols += std::min(32 * h + 32, c1) - std::max(32 * h, c0);
}

// Rows in 64-row blocks from r0 on whose envelope starts left of kend (the
// blocks the symmetric panel kernels process; with `first`, the block at r0
// always counts).
static double fenv_rows(const DeviceDecomp& d, int i, int n, int r0, int kend, bool first) {
  const int32_t* fe = d.h_fenv + (size_t)i * d.fenv_stride;
  double rows = 0;
  for (int rb = r0; rb < n; rb += 64)
    if ((first && rb == r0) || std::min(fe[rb / 32], rb + 32 < n ? fe[rb / 32 + 1] : fe[rb / 32]) < kend)
      rows += std::min(64, n - rb);
  return rows;
}

template <class C> struct RealOf;
template <> struct RealOf<float2> { using t = float; };
template <> struct RealOf<double2> { using t = double; };

// ---------------------------------------------------------------- launch accounting
// algorithmic flops / bytes of one batched launch from the true sizes n_i
template <class F>
static void kt_account(const DeviceDecomp& d, int fam, hipStream_t st, F&& per_sub, int esz) {
  if (!kt_enabled()) return;
  double fl = 0, by = 0;
  for (int i = 0; i < d.nsub; ++i) {
    double a = 0, b = 0;
    per_sub(d.h_n_loc[i], a, b);
    fl += a;
    by += b * esz;
  }
  kt_end(fam, st, fl, by);
}
static inline double clampd(double v) { return v > 0 ? v : 0; }

// Block-row solves when the decomposition asks for them (its factors then
// carry the scaled off-diagonal rows), else the recursive solves, whose
// updates spread each matrix over many workgroups (few subdomains, the
// single coarse matrix).
static inline bool row_form(const DeviceDecomp& d) { return d.rows; }

template <class C>
void lu_factor_batched(const DeviceDecomp& d, C* F, hipStream_t st, bool sym) {
  using R = typename RealOf<C>::t;
  MW_CHECK(d.max_pad <= 8192, MW_EINVAL, "subdomain too large for the dense factorisation (n_i > 8192)");
  MW_CHECK(d.boff && d.blo && d.bw && d.bstride >= d.max_pad / 64, MW_EINVAL, "factor storage tables missing");
  const int maxp = d.max_pad;
  k_amax<R><<<d.nsub, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.fenv, d.fenv_hi, d.fenv_stride, d.amax, d.boff, d.blo, d.bw, d.bstride);
  MW_LAUNCH_CHECK();
  const double rtol = sizeof(R) == 4 ? 1e-6 : 1e-14;
  // Right-looking blocked LU in two levels: 64-column panels (8-column
  // sub-panels inside) are factored and applied within an outer block of
  // NB2 columns; the rows of a panel beyond the outer block receive the
  // block's earlier panels just before their triangular solve; the trailing
  // matrix is updated once per outer block with K = NB2.
  // sym (B_i complex symmetric with a definite imaginary part): L D L^T
  // without interchanges in the same storage; the U rows of each panel come
  // from its L columns (k_sym_row) and the updates skip the tiles above the
  // diagonal, about half the work of LU.
  constexpr int WCL = sizeof(R) == 4 ? 5 : 2;
  for (int K0 = 0; K0 < maxp; K0 += NB2) {
    const int Kend = std::min(K0 + NB2, maxp);
    for (int k = K0; k < Kend; k += NB) {
      if (sym) {
        kt_begin(KF_LU_PANEL, st);
        k_sym_diag<R><<<d.nsub, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, d.ipiv, d.info, d.amax, rtol, k,
                                              d.boff, d.blo, d.bw, d.bstride);
        MW_LAUNCH_CHECK();
        if (k + NB < maxp) {
          k_sym_cols<R><<<dim3((unsigned)ceil_div(maxp - k - NB, NB), d.nsub), 256, 0, st>>>(F, d.fac_off, d.n_pad,
                                                                                             k, d.fenv,
                                                                                             d.fenv_stride, d.boff, d.blo, d.bw, d.bstride);
          MW_LAUNCH_CHECK();
        }
        int sub = 0;
        kt_account(d, KF_LU_PANEL, st, [&](int n, double& f, double& b) {
          double rows = fenv_rows(d, sub++, n, k + NB, k + NB, false);
          f = n > k ? 8.0 * (NB * NB * NB / 3.0 + rows * NB * NB / 2.0) : 0;
          b = n > k ? 2.0 * (NB + rows) * NB : 0;
        }, (int)sizeof(C));
      }
      for (int c = k; c < k + NB && !sym; c += W0) {
        kt_begin(KF_LU_PANEL, st);
        if constexpr (sizeof(R) == 4) {
          if (maxp - c <= 4096) {
            if (sym)
              k_lu_panel_reg<4, true><<<d.nsub, 1024, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, d.ipiv, d.info,
                                                              d.amax, rtol, c, k);
            else
              k_lu_panel_reg<4><<<d.nsub, 1024, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, d.ipiv, d.info, d.amax,
                                                        rtol, c, k);
          } else if (sym) {
            k_lu_panel<R, true><<<d.nsub, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, d.ipiv, d.info, d.amax,
                                                        rtol, c, k);
          } else {
            k_lu_panel<R><<<d.nsub, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, d.ipiv, d.info, d.amax, rtol, c,
                                                  k);
          }
        } else if (sym) {
          k_lu_panel<R, true><<<d.nsub, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, d.ipiv, d.info, d.amax, rtol,
                                                      c, k);
        } else {
          k_lu_panel<R><<<d.nsub, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, d.ipiv, d.info, d.amax, rtol, c, k);
        }
        MW_LAUNCH_CHECK();
        kt_account(d, KF_LU_PANEL, st, [&](int n, double& f, double& b) {
          double rows = clampd(n - c);
          f = 8.0 * rows * W0 * W0 / 2;
          b = 2.0 * rows * W0;
        }, (int)sizeof(C));
        int r0 = c + W0, c1 = k + NB;
        if (r0 < c1) {
          kt_begin(KF_LU_GEMM, st);
          launch_gemm_lu<R, 2>(d, F, r0, maxp, c, c + W0, r0, c1, maxp, st);
          kt_account(d, KF_LU_GEMM, st, [&](int n, double& f, double& b) {
            double M = clampd(n - r0), N = clampd(std::min(c1, n) - r0), K = clampd(std::min(c + W0, n) - c);
            f = 8.0 * M * N * K;
            b = M * K + K * N + 2 * M * N;
          }, (int)sizeof(C));
        }
      }
      const int c0 = k + NB;
      if (sym) {
        // no interchanges; the U rows from the L columns; the tiles of the
        // block below the diagonal
        if (c0 >= maxp) continue;
        kt_begin(KF_LU_OTHER, st);
        k_sym_row<R><<<dim3((unsigned)ceil_div(maxp - c0, NB), d.nsub), 256, 0, st>>>(F, d.fac_off, d.n_pad, k,
                                                                                        d.fenv, d.fenv_stride,
                                                                                        d.boff, d.blo, d.bw, d.bstride);
        MW_LAUNCH_CHECK();
        {
          int sub = 0;
          kt_account(d, KF_LU_OTHER, st, [&](int n, double& f, double& b) {
            double N = fenv_rows(d, sub++, n, c0, k + NB, true);
            f = 6.0 * NB * N;
            b = 2.0 * NB * N;
          }, (int)sizeof(C));
        }
        if (c0 < Kend) {
          kt_begin(KF_LU_GEMM, st);
          int M = maxp - c0, N = Kend - c0;
          unsigned tiles = (unsigned)(ceil_div(M, TB) * ceil_div(N, TB));
          k_gemm_lu<R, true><<<dim3(tiles, d.nsub), 256, 0, st>>>(F, d.fac_off, d.n_pad, c0, k, k + NB, c0, Kend,
                                                                  d.boff, d.blo, d.bw, d.bstride, d.fenv, d.fenv_stride);
          MW_LAUNCH_CHECK();
          int sub = 0;
          kt_account(d, KF_LU_GEMM, st, [&](int n, double& f, double& b) {
            double M2, N2, entries, kk;
            fenv_work(d, sub++, n, c0, k, k + NB, c0, Kend, M2, N2, entries, kk);
            f = 8.0 * kk;
            b = M2 * NB + NB * N2 + 2 * entries;
          }, (int)sizeof(C));
        }
        continue;
      }
      int ncol = maxp;  // upper bound of columns outside the panel
      kt_begin(KF_LU_OTHER, st);
      k_laswp<R><<<dim3((unsigned)ceil_div(ncol, 256), d.nsub), 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off,
                                                                               d.ipiv, k);
      MW_LAUNCH_CHECK();
      kt_account(d, KF_LU_OTHER, st, [&](int n, double& f, double& b) { f = 0; b = n > k ? 2.0 * NB * n : 0; },
                 (int)sizeof(C));
      if (c0 >= maxp) continue;
      if (k > K0 && Kend < maxp) {
        // rows [k, k+NB) beyond the outer block: the block's panels [K0, k)
        kt_begin(KF_LU_GEMM, st);
        launch_gemm_lu<R, WCL, true>(d, F, k, k + NB, K0, k, Kend, maxp, maxp, st);
        kt_account(d, KF_LU_GEMM, st, [&](int n, double& f, double& b) {
          double M = clampd(std::min(k + NB, n) - k), N = clampd(n - Kend), K = clampd(std::min(k, n) - K0);
          if (M <= 0) N = 0;
          f = 8.0 * M * N * K;
          b = M * K + K * N + 2 * M * N;
        }, (int)sizeof(C));
      }
      kt_begin(KF_LU_OTHER, st);
      k_trsm_panel<R><<<dim3((unsigned)ceil_div(maxp - c0, PANEL_COLS), d.nsub), 256, 0, st>>>(F, d.fac_off, d.n_pad, k);
      MW_LAUNCH_CHECK();
      kt_account(d, KF_LU_OTHER, st, [&](int n, double& f, double& b) {
        double N = clampd(n - c0);
        f = 4.0 * NB * NB * N;
        b = NB * NB / 2.0 + 2.0 * NB * N;
      }, (int)sizeof(C));
      if (c0 < Kend) {
        // inside the outer block: rows [c0, np), columns [c0, Kend)
        kt_begin(KF_LU_GEMM, st);
        int M = maxp - c0, N = Kend - c0;
        unsigned tiles = (unsigned)(ceil_div(M, TB) * ceil_div(N, TB));
        k_gemm_lu<R><<<dim3(tiles, d.nsub), 256, 0, st>>>(F, d.fac_off, d.n_pad, c0, k, k + NB, c0, Kend, d.boff, d.blo, d.bw, d.bstride);
        MW_LAUNCH_CHECK();
        kt_account(d, KF_LU_GEMM, st, [&](int n, double& f, double& b) {
          double M2 = clampd(n - c0), N2 = clampd(std::min(Kend, n) - c0), K = clampd(std::min(k + NB, n) - k);
          f = 8.0 * M2 * N2 * K;
          b = M2 * K + K * N2 + 2 * M2 * N2;
        }, (int)sizeof(C));
      }
    }
    if (Kend < maxp) {
      // trailing matrix: rows and columns [Kend, np), K = [K0, Kend)
      kt_begin(KF_LU_GEMM, st);
      if (sym) launch_gemm_lu<R, WCL, true, true>(d, F, Kend, maxp, K0, Kend, Kend, maxp, maxp, st);
      else launch_gemm_lu<R, WCL, true>(d, F, Kend, maxp, K0, Kend, Kend, maxp, maxp, st);
      int sub = 0;
      kt_account(d, KF_LU_GEMM, st, [&](int n, double& f, double& b) {
        double M2 = clampd(n - Kend), K = clampd(std::min(Kend, n) - K0);
        if (sym) {
          double R2, C2, entries, kk;
          fenv_work(d, sub++, n, Kend, K0, Kend, Kend, maxp, R2, C2, entries, kk);
          f = 8.0 * kk;
          b = R2 * K + K * C2 + 2 * entries;
        } else {
          f = 8.0 * M2 * M2 * K;
          b = M2 * K + K * M2 + 2 * M2 * M2;
        }
      }, (int)sizeof(C));
    }
  }
  kt_begin(KF_LU_OTHER, st);
  k_invert_diag<R><<<dim3((unsigned)(maxp / NB), d.nsub), 256, 0, st>>>(F, d.fac_off, d.n_pad, d.boff, d.blo, d.bw, d.bstride);
  MW_LAUNCH_CHECK();
  kt_account(d, KF_LU_OTHER, st, [&](int n, double& f, double& b) {
    double nb = std::ceil(n / (double)NB);
    f = nb * 8.0 * NB * NB * NB / 3.0;
    b = nb * 2.0 * NB * NB;
  }, (int)sizeof(C));
  k_build_perm<<<d.nsub, 256, 0, st>>>(d.n_pad, d.loc_off, d.ipiv, d.sub_dof, d.ridx);
  MW_LAUNCH_CHECK();
  k_envelope<C><<<(unsigned)((int64_t)d.nsub * d.env_stride), 256, 0, st>>>(
      F, d.fac_off, d.n_pad, d.env_stride, sym ? d.fenv : nullptr, sym ? d.fenv_hi : nullptr, d.env, d.boff, d.blo, d.bw, d.bstride);
  MW_LAUNCH_CHECK();
  if (row_form(d)) {
    // S_L = -T_L L[b, :64b] and S_U = -T_U U[b, 64b+64:] of every block,
    // over the envelope just found
    kt_begin(KF_LU_OTHER, st);
    const dim3 g((unsigned)(maxp / NB), (unsigned)d.nsub);
    k_scale_offdiag<R, false><<<g, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.env, d.env_stride, d.boff, d.blo, d.bw,
                                                d.bstride);
    MW_LAUNCH_CHECK();
    k_scale_offdiag<R, true><<<g, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.env, d.env_stride, d.boff, d.blo, d.bw,
                                               d.bstride);
    MW_LAUNCH_CHECK();
    int sub = 0;
    kt_account(d, KF_LU_OTHER, st, [&](int n, double& f, double& by) {
      // per 64 x 64 chunk: a triangular 64 x 64 times 64 x 64 product, the
      // chunk read and written, the triangle read once per block; chunks of
      // the structural envelope without interchanges (as many right of the
      // diagonal as left of it: B_i is structurally symmetric), all of them
      // with interchanges
      const int i = sub++;
      double chunks = 0, blocks = 0;
      for (int r0 = 0; r0 < n; r0 += NB) {
        int lo = 0;
        if (sym && d.h_fenv) {
          const int32_t* fe = d.h_fenv + (size_t)i * d.fenv_stride;
          lo = std::min(fe[r0 / 32], fe[r0 / 32 + 1]) & ~63;
        }
        chunks += sym ? 2.0 * ((r0 - std::min(lo, r0)) / NB) : (double)((n + NB - 1) / NB - 1);
        blocks += 1;
      }
      f = chunks * 4.0 * NB * NB * NB;
      by = chunks * 2.0 * NB * NB + blocks * NB * NB;
    }, (int)sizeof(C));
  }
}

// Tile width (columns) for a multi-vector of ncols columns: the narrowest of
// 32, 64, ... that holds it, up to 160 (FP32) or 64 (FP64) per tile (wider
// FP64 tiles drop to one wave per SIMD).
template <class R>
static int pick_wc(int ncols) {
  const int maxwc = sizeof(R) == 4 ? 5 : 2;
  int wc = (int)ceil_div(ncols, 32);
  return wc > maxwc ? maxwc : (wc < 1 ? 1 : wc);
}

// Y[r0:r1] -= F[r0:r1, k0:k1] Y[k0:k1] on every subdomain
template <class R, int WC, int RB = 1, bool FULL = false>
static void launch_gemm_x_wc(const DeviceDecomp& d, const typename cplx<R>::t* F, typename cplx<R>::t* Y,
                             int64_t ld, int ncols, int r0, int r1, int k0, int k1, const int32_t* row_lo,
                             hipStream_t st) {
  int tiles_m = (int)ceil_div(r1 - r0, XTile<R, RB>::TM);
  int tiles_n = (int)ceil_div(ncols, WC * 32);
  int64_t G = round_up((int64_t)d.nsub * tiles_m * tiles_n, 8);
  k_gemm_x<R, WC, RB, FULL><<<(unsigned)G, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, Y, ld, ncols, r0, r1, k0, k1,
                                                   tiles_m, tiles_n, d.nsub, row_lo, d.env, d.env_stride, d.boff, d.blo, d.bw, d.bstride);
  MW_LAUNCH_CHECK();
}
// The updates take 32-row tiles: clipped to the banded envelope their inner
// dimension is a few hundred at most, where more and smaller tiles balance
// better than 64-row tiles with half the B reads per product.
template <class R>
static void launch_gemm_x(const DeviceDecomp& d, const typename cplx<R>::t* F, typename cplx<R>::t* Y, int64_t ld,
                          int ncols, int r0, int r1, int k0, int k1, const int32_t* row_lo, hipStream_t st) {
  switch (pick_wc<R>(ncols)) {
    case 1: launch_gemm_x_wc<R, 1>(d, F, Y, ld, ncols, r0, r1, k0, k1, row_lo, st); break;
    case 2: launch_gemm_x_wc<R, 2>(d, F, Y, ld, ncols, r0, r1, k0, k1, row_lo, st); break;
    case 3: launch_gemm_x_wc<R, sizeof(R) == 4 ? 3 : 2>(d, F, Y, ld, ncols, r0, r1, k0, k1, row_lo, st); break;
    case 4: launch_gemm_x_wc<R, sizeof(R) == 4 ? 4 : 2>(d, F, Y, ld, ncols, r0, r1, k0, k1, row_lo, st); break;
    default:
      // full column tiles: rows and K ranges are multiples of 32 and 8, so
      // only the column count decides between the unchecked and checked forms
      if (sizeof(R) == 4 && ncols % 160 == 0)
        launch_gemm_x_wc<R, 5, 1, true>(d, F, Y, ld, ncols, r0, r1, k0, k1, row_lo, st);
      else
        launch_gemm_x_wc<R, sizeof(R) == 4 ? 5 : 2>(d, F, Y, ld, ncols, r0, r1, k0, k1, row_lo, st);
      break;
  }
}
template <class R, int WC, int AMODE>
static void launch_leaf_x_wc(const DeviceDecomp& d, const typename cplx<R>::t* F, typename cplx<R>::t* Y,
                             int64_t ld, int ncols, int r0, const int32_t* row_lo, hipStream_t st) {
  int tiles_n = (int)ceil_div(ncols, WC * 32);
  int64_t G = round_up((int64_t)d.nsub * tiles_n, 8);
  k_leaf_x<R, WC, AMODE><<<(unsigned)G, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, Y, ld, ncols, r0, tiles_n,
                                                     d.nsub, row_lo, d.boff, d.blo, d.bw, d.bstride);
  MW_LAUNCH_CHECK();
}
// The leaves take 32-column tiles whatever the width: one 64 x 64 block per
// subdomain is too little work per launch, and more, narrower workgroups
// (the inverted block re-read from L2 by each) hide the load latency better.
template <class R, int AMODE>
static void launch_leaf_x(const DeviceDecomp& d, const typename cplx<R>::t* F, typename cplx<R>::t* Y, int64_t ld,
                          int ncols, int r0, const int32_t* row_lo, hipStream_t st) {
  launch_leaf_x_wc<R, 1, AMODE>(d, F, Y, ld, ncols, r0, row_lo, st);
}

template <class R>
static void fwd_rec(const DeviceDecomp& d, const typename cplx<R>::t* F, typename cplx<R>::t* Y, int ncols,
                    int64_t ld, int b0, int b1, hipStream_t st) {
  const int esz = (int)sizeof(typename cplx<R>::t);
  if (b1 - b0 == 1) {
    kt_begin(KF_TRSM_LEAF, st);
    launch_leaf_x<R, 1>(d, F, Y, ld, ncols, b0 * NB, nullptr, st);
    MW_LAUNCH_CHECK();
    kt_account(d, KF_TRSM_LEAF, st, [&](int n, double& f, double& b) {
      double m = clampd(std::min((b0 + 1) * NB, n) - b0 * NB);
      f = 4.0 * m * m * ncols;
      b = m * m / 2 + 2 * m * ncols;
    }, esz);
    return;
  }
  int mid = b0 + (b1 - b0) / 2;
  fwd_rec<R>(d, F, Y, ncols, ld, b0, mid, st);
  kt_begin(KF_TRSM_GEMM, st);
  launch_gemm_x<R>(d, F, Y, ld, ncols, mid * NB, b1 * NB, b0 * NB, mid * NB, nullptr, st);
  MW_LAUNCH_CHECK();
  {
    int sub = 0;
    kt_account(d, KF_TRSM_GEMM, st, [&](int n, double& f, double& b) {
      double fac, kspan, rows;
      env_work(d, sub++, n, mid * NB, b1 * NB, b0 * NB, mid * NB, fac, kspan, rows);
      f = 8.0 * fac * ncols;
      b = fac + kspan * ncols + 2 * rows * ncols;
    }, esz);
  }
  fwd_rec<R>(d, F, Y, ncols, ld, mid, b1, st);
}

template <class R>
static void bwd_rec(const DeviceDecomp& d, const typename cplx<R>::t* F, typename cplx<R>::t* Y, int ncols,
                    int64_t ld, int b0, int b1, hipStream_t st) {
  const int esz = (int)sizeof(typename cplx<R>::t);
  if (b1 - b0 == 1) {
    kt_begin(KF_TRSM_LEAF, st);
    launch_leaf_x<R, 2>(d, F, Y, ld, ncols, b0 * NB, d.row_lo, st);
    MW_LAUNCH_CHECK();
    int sub = 0;
    kt_account(d, KF_TRSM_LEAF, st, [&](int n, double& f, double& b) {
      const int lo = d.h_row_lo[sub++];
      double m = b0 * NB < lo ? 0.0 : clampd(std::min((b0 + 1) * NB, n) - b0 * NB);
      f = 4.0 * m * m * ncols;
      b = m * m / 2 + 2 * m * ncols;
    }, esz);
    return;
  }
  int mid = b0 + (b1 - b0) / 2;
  bwd_rec<R>(d, F, Y, ncols, ld, mid, b1, st);
  kt_begin(KF_TRSM_GEMM, st);
  launch_gemm_x<R>(d, F, Y, ld, ncols, b0 * NB, mid * NB, mid * NB, b1 * NB, d.row_lo, st);
  MW_LAUNCH_CHECK();
  {
    int sub = 0;
    kt_account(d, KF_TRSM_GEMM, st, [&](int n, double& f, double& b) {
      const int i = sub++;
      const int lo = std::max(b0 * NB, d.h_row_lo[i]);
      double fac = 0, kspan = 0, rows = 0;
      if (std::min(mid * NB, n) > lo) env_work(d, i, n, lo, mid * NB, mid * NB, b1 * NB, fac, kspan, rows);
      f = 8.0 * fac * ncols;
      b = fac + kspan * ncols + 2 * rows * ncols;
    }, esz);
  }
  bwd_rec<R>(d, F, Y, ncols, ld, b0, mid, st);
}

template <class R, int WC, int DIRS, int WNW = 2>
static void launch_row_sweep_wc(const DeviceDecomp& d, const typename cplx<R>::t* F, typename cplx<R>::t* Y,
                                int64_t ld, int ncols, hipStream_t st) {
  const int tiles_n = (int)ceil_div(ncols, WC * 16 * WNW);
  const int64_t G = 8 * ceil_div(d.nsub, 8) * (int64_t)tiles_n;
  k_row_sweep<R, WC, DIRS, WNW><<<(unsigned)G, 256, 0, st>>>(F, d.fac_off, d.n_pad, d.loc_off, Y, ld, ncols, tiles_n,
                                                        d.nsub, d.order, d.row_lo, d.env, d.env_stride, d.boff,
                                                        d.blo, d.bw, d.bstride);
  MW_LAUNCH_CHECK();
}
// Both triangular solves of every subdomain, block-row form (DIRS = 3; 1
// forward only, 2 backward only).
template <class R, int DIRS = 3>
static void launch_row_sweep(const DeviceDecomp& d, const typename cplx<R>::t* F, typename cplx<R>::t* Y, int64_t ld,
                             int ncols, hipStream_t st) {
  const int esz = (int)sizeof(typename cplx<R>::t);
  MW_CHECK(d.order != nullptr, MW_EINVAL, "subdomain order missing");
  kt_begin(KF_TRSM_GEMM, st);
  switch (pick_wc<R>(ncols)) {
    case 1: launch_row_sweep_wc<R, 1, DIRS>(d, F, Y, ld, ncols, st); break;
    case 2: launch_row_sweep_wc<R, 2, DIRS>(d, F, Y, ld, ncols, st); break;
    case 3: launch_row_sweep_wc<R, sizeof(R) == 4 ? 3 : 2, DIRS>(d, F, Y, ld, ncols, st); break;
    case 4: launch_row_sweep_wc<R, sizeof(R) == 4 ? 4 : 2, DIRS>(d, F, Y, ld, ncols, st); break;
    default:
      // complex FP32, 129-160 columns: two 80-column tiles of four 16-row
      // wave tiles (127 VGPRs, four workgroups per CU) rather than one
      // 160-column tile of 32-row wave tiles (208 VGPRs, two per CU); the
      // second tile's factor reads mostly hit the XCD's L2 (26.5 against
      // 27.2 ms per application on the 1 GHz chamber)
      if constexpr (sizeof(R) == 4) launch_row_sweep_wc<R, 5, DIRS, 1>(d, F, Y, ld, ncols, st);
      else launch_row_sweep_wc<R, 2, DIRS>(d, F, Y, ld, ncols, st);
      break;
  }
  // algorithmic work per block: the triangular solve with the diagonal
  // block (m rows) and the product with the off-diagonal entries inside the
  // envelope (32-row groups); bytes: those factor entries once, every row of
  // Y read and written once per sweep
  int sub = 0;
  kt_account(d, KF_TRSM_GEMM, st, [&](int n, double& f, double& by) {
    const int i = sub++;
    f = by = 0;
    for (int dir = 1; dir <= 2; ++dir) {
      if (!(DIRS & dir)) continue;
      double rows_y = 0;
      for (int r0 = 0; r0 < n; r0 += NB) {
        const double m = std::min(r0 + NB, n) - r0;
        if (dir == 2 && r0 + NB <= d.h_row_lo[i]) continue;
        double fac, kspan, rows;
        if (dir == 2) env_work(d, i, n, r0, r0 + NB, r0 + NB, n, fac, kspan, rows);
        else env_work(d, i, n, r0, r0 + NB, 0, r0, fac, kspan, rows);
        f += 8.0 * fac * ncols + 4.0 * m * m * ncols;
        by += fac + m * m / 2;
        rows_y += m;
      }
      by += 2.0 * rows_y * ncols;
    }
  }, esz);
}

template <class C>
void lu_solve_batched(const DeviceDecomp& d, const C* F, C* Y, int ncols, int64_t ld, hipStream_t st) {
  using R = typename RealOf<C>::t;
  int nblk = d.max_pad / NB;
  if (row_form(d)) {
    launch_row_sweep<R>(d, F, Y, ld, ncols, st);
    return;
  }
  fwd_rec<R>(d, F, Y, ncols, ld, 0, nblk, st);
  bwd_rec<R>(d, F, Y, ncols, ld, 0, nblk, st);
}

template void lu_factor_batched<float2>(const DeviceDecomp&, float2*, hipStream_t, bool);
template void lu_factor_batched<double2>(const DeviceDecomp&, double2*, hipStream_t, bool);
template void lu_solve_batched<float2>(const DeviceDecomp&, const float2*, float2*, int, int64_t, hipStream_t);
template void lu_solve_batched<double2>(const DeviceDecomp&, const double2*, double2*, int, int64_t, hipStream_t);

}  // namespace mw
