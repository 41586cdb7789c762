// Host-side small dense algebra of block GMRES (block Arnoldi with block
// classical Gram-Schmidt and a Cholesky QR of each new block; Saad, Iterative
// Methods for Sparse Linear Systems, 2nd ed., Section 6.12): the Cholesky
// factor of a block's Gram matrix and its inverse, and the per-column least-
// squares problems of the block Hessenberg matrix, kept in factored form by
// Householder reflections added one block column at a time.  Blocks are
// BW = 32 columns wide; a narrower block pads its trailing columns (identity
// in the Gram matrix, zero right-hand sides), which keeps them decoupled.
#pragma once

#include <complex>
#include <vector>

namespace mw {

using zc = std::complex<double>;
constexpr int BW = 32;

// R (q x q, row-major, upper triangular) with R^H R = G (Hermitian, row-major).
// A pivot whose square is <= thr2 is taken as zero: its row of R is zero.
// Returns the number of such pivots.
int chol_upper(const zc* G, int q, double thr2, zc* R);

// Rinv = R^-1 for an upper triangular R (q x q, row-major) with non-zero diagonal.
void tri_inv_upper(const zc* R, int q, zc* Rinv);

// Least squares min ||E_1 S0 - Hbar_j Y|| for the BW right-hand sides of one
// block, with Hbar_j the (j+2)BW x (j+1)BW block upper Hessenberg matrix
// whose sub-diagonal blocks are upper triangular.  Column k of Hbar has
// non-zeros in rows <= k + BW only, so one reflector of length BW + 1 per
// column reduces it to triangular form.
class BlockLS {
 public:
  // S0: BW x BW (row-major) upper triangular; columns >= width are padding.
  void start(int m, const zc* S0, int width);
  // Appends block column j = steps(): Hc ((j+1)BW x BW, row-major; row
  // k*BW + c1 is basis column c1 of V_k) and the sub-diagonal block R.
  void add(const zc* Hc, const zc* R);
  int steps() const { return j_; }
  // least-squares residual norm of right-hand side c after steps() columns
  double resid(int c) const;
  // Y (steps()*BW x BW, row-major) of the least-squares solution
  void solve(zc* Y) const;

 private:
  int m_ = 0, j_ = 0, width_ = BW;
  int64_t ldr_ = 0;               // rows of the stored factor, (m+1)BW
  std::vector<zc> R_;             // triangular factor, column-major, ldr_ rows
  std::vector<zc> v_;             // reflector of column k: v_[k*(BW+1) .. +BW]
  std::vector<double> h_;         // 2 / (v^H v) per column (0: identity)
  std::vector<zc> g_;             // transformed right-hand sides, row-major ((m+1)BW x BW)
  std::vector<zc> c_;             // scratch: the new block column, column-major
};

}  // namespace mw
