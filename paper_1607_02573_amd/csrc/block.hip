// Block Gram-Schmidt kernels of block GMRES (the block Krylov method named in
// the paper's conclusion, Section 7, as a way to solve many right-hand sides
// together at higher arithmetic intensity).  The right-hand-side columns of a
// solve are grouped into blocks of BW = 32 consecutive columns (the last one
// may be narrower); block b of a multi-vector is columns [32 b, 32 b + w_b)
// of an n x ncols row-major array (column index contiguous, leading dimension
// ncols), so the Krylov basis keeps the layout of the pseudo-block solver:
// V_k = V + k * vstride.
//
// Both kernels are complex FP64 products on the matrix cores in the 3M
// (Gauss) form: three real 16x16x4 MFMA products per complex product, with
// Re = P1 - P2 and Im = P3 - P1 - P2.  With 32 right-hand sides per block a
// basis vector element is used 32 times, about 12 flops per byte, so these
// sweeps are bound by the FP64 matrix rate rather than by HBM.
#include "kernels.hpp"

namespace mw {

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ inline doublex4 mf64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// output element r of lane l of a 16x16x4 FP64 product: row (l/16) + 4r, column l%16
__device__ inline int orow(int lane, int r) { return (lane >> 4) + 4 * r; }

// logical workgroup index with consecutive indices on one XCD (workgroups are
// dealt to the 8 XCDs round robin); G must be a multiple of 8
__device__ inline int xcd_remap(int bid, int G) { return (bid & 7) * (G >> 3) + (bid >> 3); }

}  // namespace

// ---------------------------------------------------------------- dots
// part[u][c1][c2] (u = (chunk * nb + b) * ktot + k, 32 x 32 complex each) =
//   sum over the rows of `chunk` of conj(L_k[r][32b + c1]) * Wr[r][32b + c2],
// L_k = V_k for k < kv and L_kv = E when E is given (ktot = kv + (E != 0)).
// One wave per unit u; a workgroup holds four consecutive units.  Columns
// beyond the block's width read as zero, so their entries are zero.  Blocks
// with blk[b] == 0 write zeros.
__global__ void __launch_bounds__(256, 2)
    k_bdots(const double2* __restrict__ V, int64_t vstride, int kv, const double2* __restrict__ E,
            const double2* __restrict__ Wr, int64_t n, int64_t ld, int ncols, int nb,
            const int32_t* __restrict__ blk, int64_t rows_per_ch, int64_t units, double2* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t u = L * 4 + wave;
  if (u >= units) return;
  const int ktot = kv + (E ? 1 : 0);
  const int k = (int)(u % ktot);
  const int64_t t = u / ktot;
  const int b = (int)(t % nb);
  const int64_t ch = t / nb;
  double2* out = part + u * 1024;
  const int li = lane & 15, kq = lane >> 4;
  if (blk && !blk[b]) {
    for (int e = lane; e < 1024; e += 64) out[e] = make_double2(0.0, 0.0);
    return;
  }
  const double2* Lk = k < kv ? V + (int64_t)k * vstride : E;
  const int cb = 32 * b;
  const bool okc[2] = {cb + li < ncols, cb + 16 + li < ncols};
  const int64_t r0 = ch * rows_per_ch;
  const int64_t r1 = min(n, r0 + rows_per_ch);
  doublex4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) { p1[x][y][r] = 0; p2[x][y][r] = 0; p3[x][y][r] = 0; }
  for (int64_t i = r0; i < r1; i += 16) {
    double2 a[4][2], w[4][2];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t row = i + 4 * s + kq;
      const bool okr = row < r1;
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int64_t off = row * ld + cb + 16 * x + li;
        a[s][x] = (okr && okc[x]) ? Lk[off] : make_double2(0.0, 0.0);
        w[s][x] = (okr && okc[x]) ? Wr[off] : make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // conj(a) = (ar, -ai): P1 = ar wr, P2 = (-ai) wi, P3 = (ar - ai)(wr + wi)
      double a1[2], a2[2], a3[2], b1[2], b2[2], b3[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a1[x] = a[s][x].x;
        a2[x] = -a[s][x].y;
        a3[x] = a[s][x].x - a[s][x].y;
        b1[x] = w[s][x].x;
        b2[x] = w[s][x].y;
        b3[x] = w[s][x].x + w[s][x].y;
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          p1[x][y] = mf64(a1[x], b1[y], p1[x][y]);
          p2[x][y] = mf64(a2[x], b2[y], p2[x][y]);
          p3[x][y] = mf64(a3[x], b3[y], p3[x][y]);
        }
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c1 = 16 * x + orow(lane, r), c2 = 16 * y + li;
        out[c1 * 32 + c2] = make_double2(p1[x][y][r] - p2[x][y][r], p3[x][y][r] - p1[x][y][r] - p2[x][y][r]);
      }
}

// rows per chunk and chunk count of k_bdots for ktot left operands
void bdots_chunks(int64_t n, int nb, int ktot, int64_t* rows_per_ch, int64_t* nch) {
  const int64_t target_units = 4096;
  int64_t c = std::max<int64_t>(1, target_units / std::max<int64_t>(1, (int64_t)nb * ktot));
  c = std::min<int64_t>(c, ceil_div(std::max<int64_t>(n, 1), 16));
  int64_t rows = round_up(ceil_div(std::max<int64_t>(n, 1), c), 16);
  *rows_per_ch = rows;
  *nch = ceil_div(std::max<int64_t>(n, 1), rows);
}

void launch_bdots(const double2* V, int64_t vstride, int kv, const double2* E, const double2* Wr, int64_t n,
                  int64_t ld, int ncols, int nb, const int32_t* blk, double2* part, int64_t* nch_out,
                  hipStream_t st) {
  const int ktot = kv + (E ? 1 : 0);
  int64_t rows, nch;
  bdots_chunks(n, nb, ktot, &rows, &nch);
  *nch_out = nch;
  if (ktot == 0 || nb == 0) return;
  const int64_t units = nch * nb * ktot;
  const int64_t G = round_up(ceil_div(units, 4), 8);
  kt_begin(KF_BGS_DOTS, st);
  k_bdots<<<(unsigned)G, 256, 0, st>>>(V, vstride, kv, E, Wr, n, ld, ncols, nb, blk, rows, units, part);
  MW_LAUNCH_CHECK();
  // algorithmic work: every left operand and the right operand read once;
  // 32 x 32 complex multiply-adds (8 flops each) per row, block and operand
  const double elems = (double)n * ncols;
  kt_end(KF_BGS_DOTS, st, 8.0 * 32.0 * elems * ktot, 16.0 * elems * (ktot + 1));
}

// ---------------------------------------------------------------- update
// For every block b with blk[b] != 0 (blk == 0: all blocks):
//   T = (Win ? Win : 0) - sum_{k < kv_b} V_k[:, block b] P_b,k,
//   Out[:, block b] = Rinv ? T Rinv_b : T,
// where P_b,k = P + (b * pk_stride + k) * 1024 is 32 x 32 (row c1 = the basis
// column, column c2 = the output column) and Rinv_b = Rinv + b * 1024 is
// 32 x 32; kv_b = kvb[b] if kvb is given, else kv.  blk[b] == 2 writes zeros
// to the block instead.  Tile: 64 rows x the 32 columns of one block, four
// waves in a 2 x 2 arrangement, the K dimension (basis vector, column) staged
// through double-buffered LDS 8 complex at a time.  Out may equal Win.
constexpr int UK = 8;
__global__ void __launch_bounds__(256, 2)
    k_bupdate(const double2* __restrict__ V, int64_t vstride, int kv, const int32_t* __restrict__ kvb,
              const double2* __restrict__ P, int pk_stride, const double2* __restrict__ Rinv,
              const double2* Win, double2* Out, int64_t n, int64_t ld, int ncols, int nb,
              const int32_t* __restrict__ blk, int64_t tiles) {
  constexpr int TM = 64;
  constexpr int A_BYTES = 2 * 3 * TM * (UK + 1) * 8;
  constexpr int B_BYTES = 2 * 3 * UK * 48 * 8;
  constexpr int T_BYTES = TM * 33 * 16 + 32 * 33 * 16;
  constexpr int SMEM = (A_BYTES + B_BYTES) > T_BYTES ? (A_BYTES + B_BYTES) : T_BYTES;
  __shared__ __attribute__((aligned(16))) char smem[SMEM];
  auto As = reinterpret_cast<double(*)[3][TM][UK + 1]>(smem);
  auto Bs = reinterpret_cast<double(*)[3][UK][48]>(smem + A_BYTES);
  const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
  if (L >= tiles) return;
  const int b = (int)(L % nb);
  const int64_t row0 = (L / nb) * TM;
  const int mode = blk ? blk[b] : 1;
  if (mode == 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, kq = lane >> 4;
  const int cb = 32 * b;
  const int width = min(32, ncols - cb);
  if (mode == 2) {
    for (int e = tid; e < TM * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      if (row0 + r < n && c < width) Out[(row0 + r) * ld + cb + c] = make_double2(0.0, 0.0);
    }
    return;
  }
  const int K = 32 * (kvb ? kvb[b] : kv);
  doublex4 p1[2], p2[2], p3[2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) { p1[x][r] = 0; p2[x][r] = 0; p3[x][r] = 0; }
  const double2* Pb = P + (int64_t)b * pk_stride * 1024;
  double2 ra[2], rb;
  // stage k0 (multiple of 8): basis vector k0 / 32, columns k0 % 32 .. + 8
  auto fetch = [&](int k0) {
    const double2* Vk = V + (int64_t)(k0 >> 5) * vstride + cb + (k0 & 31);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = tid + e * 256;
      const int r = idx >> 3, kc = idx & 7;
      const bool ok = row0 + r < n && (k0 & 31) + kc < width;
      ra[e] = ok ? Vk[(row0 + r) * ld + kc] : make_double2(0.0, 0.0);
    }
    const int r = tid >> 5, c = tid & 31;
    rb = Pb[(int64_t)(k0 + r) * 32 + c];
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = tid + e * 256;
      const int r = idx >> 3, kc = idx & 7;
      As[buf][0][r][kc] = ra[e].x;
      As[buf][1][r][kc] = ra[e].y;
      As[buf][2][r][kc] = ra[e].x + ra[e].y;
    }
    const int r = tid >> 5, c = tid & 31;
    Bs[buf][0][r][c] = rb.x;
    Bs[buf][1][r][c] = rb.y;
    Bs[buf][2][r][c] = rb.x + rb.y;
  };
  if (K > 0) {
    fetch(0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += UK) {
      const bool more = k0 + UK < K;
      if (more) fetch(k0 + UK);
#pragma unroll
      for (int kk = 0; kk < UK; kk += 4) {
        const int col = wn * 16 + li;
        const double b1 = Bs[buf][0][kk + kq][col], b2 = Bs[buf][1][kk + kq][col], b3 = Bs[buf][2][kk + kq][col];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const int row = wm * 32 + x * 16 + li;
          p1[x] = mf64(As[buf][0][row][kk + kq], b1, p1[x]);
          p2[x] = mf64(As[buf][1][row][kk + kq], b2, p2[x]);
          p3[x] = mf64(As[buf][2][row][kk + kq], b3, p3[x]);
        }
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  if (!Rinv) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gr = row0 + wm * 32 + x * 16 + orow(lane, r);
        const int gc = wn * 16 + li;
        if (gr < n && gc < width) {
          const int64_t off = gr * ld + cb + gc;
          double2 o = Win ? Win[off] : make_double2(0.0, 0.0);
          o.x -= p1[x][r] - p2[x][r];
          o.y -= p3[x][r] - p1[x][r] - p2[x][r];
          Out[off] = o;
        }
      }
    return;
  }
  // T (64 x 32) through LDS, then Out = T Rinv_b row by row
  auto Ts = reinterpret_cast<double2(*)[33]>(smem);
  auto Rs = reinterpret_cast<double2(*)[33]>(smem + TM * 33 * 16);
  __syncthreads();   // every wave is done with As/Bs (no-op ordering when K == 0)
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = wm * 32 + x * 16 + orow(lane, r);
      const int gc = wn * 16 + li;
      const int64_t gr = row0 + lr;
      double2 o = make_double2(0.0, 0.0);
      if (gr < n && gc < width) {
        if (Win) o = Win[gr * ld + cb + gc];
        o.x -= p1[x][r] - p2[x][r];
        o.y -= p3[x][r] - p1[x][r] - p2[x][r];
      }
      Ts[lr][gc] = o;
    }
  const double2* Rb = Rinv + (int64_t)b * 1024;
  for (int e = tid; e < 1024; e += 256) Rs[e >> 5][e & 31] = Rb[e];
  __syncthreads();
  const int r = tid >> 2, cg = tid & 3;
  double2 acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = make_double2(0.0, 0.0);
#pragma unroll 2
  for (int c1 = 0; c1 < 32; ++c1) {
    const double2 tv = Ts[r][c1];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double2 rv = Rs[c1][cg + 4 * u];
      acc[u].x += tv.x * rv.x - tv.y * rv.y;
      acc[u].y += tv.x * rv.y + tv.y * rv.x;
    }
  }
  if (row0 + r < n) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = cg + 4 * u;
      if (c < width) Out[(row0 + r) * ld + cb + c] = acc[u];
    }
  }
}

void launch_bupdate(const double2* V, int64_t vstride, int kv, const int32_t* kvb, int kv_max, const double2* P,
                    int pk_stride, const double2* Rinv, const double2* Win, double2* Out, int64_t n, int64_t ld,
                    int ncols, int nb, const int32_t* blk, hipStream_t st) {
  if (n == 0 || nb == 0) return;
  const int64_t tiles = ceil_div(n, 64) * nb;
  const int64_t G = round_up(tiles, 8);
  kt_begin(KF_BGS_UPDATE, st);
  k_bupdate<<<(unsigned)G, 256, 0, st>>>(V, vstride, kv, kvb, P, pk_stride, Rinv, Win, Out, n, ld, ncols, nb, blk,
                                         tiles);
  MW_LAUNCH_CHECK();
  const int kk = kvb ? kv_max : kv;
  const double elems = (double)n * ncols;
  kt_end(KF_BGS_UPDATE, st, 8.0 * 32.0 * elems * (kk + (Rinv ? 1 : 0)), 16.0 * elems * (kk + (Win ? 2 : 1)));
}

}  // namespace mw
