// Host-side small dense algebra of block GMRES; see blockls.hpp.
#include "blockls.hpp"

#include <cmath>
#include <cstdint>

namespace mw {

int chol_upper(const zc* G, int q, double thr2, zc* R) {
  int deficient = 0;
  for (int i = 0; i < q * q; ++i) R[i] = 0.0;
  for (int k = 0; k < q; ++k) {
    double d = G[k * q + k].real();
    for (int i = 0; i < k; ++i) d -= std::norm(R[i * q + k]);
    if (!(d > thr2)) {   // also catches NaN
      ++deficient;
      continue;
    }
    const double rkk = std::sqrt(d);
    R[k * q + k] = rkk;
    for (int l = k + 1; l < q; ++l) {
      zc s = G[k * q + l];
      for (int i = 0; i < k; ++i) s -= std::conj(R[i * q + k]) * R[i * q + l];
      R[k * q + l] = s / rkk;
    }
  }
  return deficient;
}

void tri_inv_upper(const zc* R, int q, zc* Rinv) {
  for (int i = 0; i < q * q; ++i) Rinv[i] = 0.0;
  for (int c = 0; c < q; ++c) {
    // R x = e_c by back substitution; x is zero below row c
    for (int i = c; i >= 0; --i) {
      zc s = (i == c) ? zc(1.0) : zc(0.0);
      for (int l = i + 1; l <= c; ++l) s -= R[i * q + l] * Rinv[l * q + c];
      Rinv[i * q + c] = s / R[i * q + i];
    }
  }
}

void BlockLS::start(int m, const zc* S0, int width) {
  m_ = m;
  j_ = 0;
  width_ = width;
  ldr_ = (int64_t)(m + 1) * BW;
  R_.assign((size_t)ldr_ * m * BW, zc(0.0));
  v_.assign((size_t)m * BW * (BW + 1), zc(0.0));
  h_.assign((size_t)m * BW, 0.0);
  g_.assign((size_t)ldr_ * BW, zc(0.0));
  c_.assign((size_t)ldr_ * BW, zc(0.0));
  for (int r = 0; r < BW; ++r)
    for (int c = 0; c < width; ++c) g_[(size_t)r * BW + c] = S0[r * BW + c];
}

void BlockLS::add(const zc* Hc, const zc* R) {
  const int j = j_;
  const int64_t rows = (int64_t)(j + 2) * BW;
  // new block column, column-major with ldr_ rows
  for (int t = 0; t < BW; ++t) {
    zc* col = &c_[(size_t)t * ldr_];
    for (int64_t r = 0; r < (int64_t)(j + 1) * BW; ++r) col[r] = Hc[r * BW + t];
    for (int r = 0; r < BW; ++r) col[(int64_t)(j + 1) * BW + r] = R[r * BW + t];
  }
  // reflectors of the earlier columns
  for (int64_t k = 0; k < (int64_t)j * BW; ++k) {
    const double h = h_[k];
    if (h == 0.0) continue;
    const zc* v = &v_[(size_t)k * (BW + 1)];
    for (int t = 0; t < BW; ++t) {
      zc* y = &c_[(size_t)t * ldr_ + k];
      zc s = 0.0;
      for (int r = 0; r <= BW; ++r) s += std::conj(v[r]) * y[r];
      s *= h;
      for (int r = 0; r <= BW; ++r) y[r] -= s * v[r];
    }
  }
  // a reflector for each new column: x -> beta e_0, beta = -phase(x_0) ||x||
  for (int t = 0; t < BW; ++t) {
    const int64_t k = (int64_t)j * BW + t;
    zc* x = &c_[(size_t)t * ldr_ + k];
    zc* v = &v_[(size_t)k * (BW + 1)];
    double nrm2 = 0.0;
    for (int r = 0; r <= BW; ++r) nrm2 += std::norm(x[r]);
    const double nrm = std::sqrt(nrm2);
    double h = 0.0;
    if (nrm > 0.0) {
      const double ax = std::abs(x[0]);
      const zc ph = ax > 0.0 ? x[0] / ax : zc(1.0);
      for (int r = 0; r <= BW; ++r) v[r] = x[r];
      v[0] += ph * nrm;
      double vv = 0.0;
      for (int r = 0; r <= BW; ++r) vv += std::norm(v[r]);
      h = 2.0 / vv;
      // apply to this and the later columns of the block, and to g
      for (int t2 = t; t2 < BW; ++t2) {
        zc* y = &c_[(size_t)t2 * ldr_ + k];
        zc s = 0.0;
        for (int r = 0; r <= BW; ++r) s += std::conj(v[r]) * y[r];
        s *= h;
        for (int r = 0; r <= BW; ++r) y[r] -= s * v[r];
      }
      for (int c = 0; c < BW; ++c) {
        zc s = 0.0;
        for (int r = 0; r <= BW; ++r) s += std::conj(v[r]) * g_[(size_t)(k + r) * BW + c];
        s *= h;
        for (int r = 0; r <= BW; ++r) g_[(size_t)(k + r) * BW + c] -= s * v[r];
      }
    }
    h_[k] = h;
  }
  // keep the triangular part (rows <= k of column k)
  for (int t = 0; t < BW; ++t) {
    const int64_t k = (int64_t)j * BW + t;
    for (int64_t r = 0; r <= k; ++r) R_[(size_t)k * ldr_ + r] = c_[(size_t)t * ldr_ + r];
  }
  (void)rows;
  j_ = j + 1;
}

double BlockLS::resid(int c) const {
  double s = 0.0;
  for (int r = 0; r < BW; ++r) s += std::norm(g_[(size_t)((int64_t)j_ * BW + r) * BW + c]);
  return std::sqrt(s);
}

void BlockLS::solve(zc* Y) const {
  const int64_t K = (int64_t)j_ * BW;
  for (int c = 0; c < BW; ++c) {
    for (int64_t i = K - 1; i >= 0; --i) {
      zc s = c < width_ ? g_[(size_t)i * BW + c] : zc(0.0);
      for (int64_t l = i + 1; l < K; ++l) s -= R_[(size_t)l * ldr_ + i] * Y[l * BW + c];
      const zc d = R_[(size_t)i * ldr_ + i];
      Y[i * BW + c] = d != zc(0.0) ? s / d : zc(0.0);
    }
  }
}

}  // namespace mw
