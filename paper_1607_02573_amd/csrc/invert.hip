// The outer inversion loop of Section 5: L-BFGS on the normalised,
// regularised misfit (equation (defJ2)) over a permittivity given at the mesh
// vertices (Section 6 discretises kappa = k0^2 eps_r with P1 elements).
//
// One evaluation at the vertex field e:
//   A(e): the tetrahedron means of e (or, with p1, e integrated exactly in
//         the mass term), the subdomain factors;
//   U = A^-1 B for the transmitting ports, S (equation (sij));
//   J_d = 1/2 sum_ij w_ij |S_ij - Smes_ij|^2, w_ij = 1 / |Sempty_ij|^2;
//   F = A^-1 Lambda with the adjoint data of the weighted residual
//       (problem (pbadj)), the per-tetrahedron gradient, mapped to the
//       vertices by the transpose of the averaging (or the exact P1 form);
//   the Tikhonov term alpha/2 int |grad e|^2, exact for the P1 field through
//       the P1 stiffness matrix K1 (applied to Re e and Im e): alpha/2
//       Re(e^H K1 e) and its gradient alpha K1 e.
// J = J_d + Tikhonov; gradient in the convention dJ/dRe e + i dJ/dIm e.
// Reuse of the previous evaluation's Krylov solutions (the paper's conclusion,
// Section 7, proposes recycling Krylov information across the inversion's
// iterations): recycle = 1 starts every column from its own previous field;
// recycle = 2 starts all columns from the best combination of all previous
// fields, X0 = U Y with Y minimising ||B - A U Y||_F column by column (normal
// equations (AU)^H (AU) Y = (AU)^H B, solved by Cholesky on the host), which
// is never worse than recycle = 1 (Y = I is one choice).  The optimiser (mw_lbfgs) is the two-loop recursion
// of limited-memory BFGS (Nocedal and Wright, Numerical Optimization, 2nd
// ed., Algorithms 7.4 and 7.5) with a backtracking Armijo line search; it
// runs on the host over x = [Re e; Im e], the objective on the device.
#include <chrono>
#include <cmath>
#include <deque>
#include <memory>
#include <numeric>

#include "internal.hpp"

using namespace mw;

namespace {

__global__ void k_vertex_mean(int64_t nt, const int32_t* __restrict__ tet, const double2* __restrict__ ev,
                              double2* __restrict__ et) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double2 v = ev[tet[4 * t + k]];
    re += v.x;
    im += v.y;
  }
  et[t] = make_double2(0.25 * re, 0.25 * im);
}

// transpose of the averaging: g_v = sum over the tetrahedra t at v of g_t / 4
// (entries of v in ascending t)
__global__ void k_vertex_gather(int64_t nv, const int64_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt,
                                const double2* __restrict__ gt, double2* __restrict__ gv) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double re = 0.0, im = 0.0;
  for (int64_t k = vt_ptr[v]; k < vt_ptr[v + 1]; ++k) {
    const double2 g = gt[vt[k] >> 2];
    re += 0.25 * g.x;
    im += 0.25 * g.y;
  }
  gv[v] = make_double2(re, im);
}

// P1 stiffness of every tetrahedron: Ke[t][a][b] = vol grad l_a . grad l_b,
// the barycentric gradients from the inverse of [1 x y z] (cofactors)
__global__ void k_p1_stiffness(int64_t nt, const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                               double* __restrict__ Ke) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double p[4][3];
  for (int k = 0; k < 4; ++k)
    for (int a = 0; a < 3; ++a) p[k][a] = xyz[3 * (int64_t)tet[4 * t + k] + a];
  const double e1[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
  const double e2[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
  const double e3[3] = {p[3][0] - p[0][0], p[3][1] - p[0][1], p[3][2] - p[0][2]};
  // rows of the inverse of J = [e1 e2 e3] (as columns) are the gradients of l_1, l_2, l_3
  const double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2], e2[0] * e3[1] - e2[1] * e3[0]};
  const double c31[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2], e3[0] * e1[1] - e3[1] * e1[0]};
  const double c12[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
  double g[4][3];
  for (int a = 0; a < 3; ++a) {
    g[1][a] = c23[a] / det;
    g[2][a] = c31[a] / det;
    g[3][a] = c12[a] / det;
    g[0][a] = -(g[1][a] + g[2][a] + g[3][a]);
  }
  const double vol = fabs(det) / 6.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      Ke[16 * t + 4 * a + b] = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
}

// y = K1 e (complex e, real K1) by vertex: sum over the (t, slot) entries of
// v of Ke[t][slot][:] . e|_t; also the per-vertex term Re(conj(e_v) y_v) of
// e^H K1 e
__global__ void k_p1_apply(int64_t nv, const int64_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt,
                           const int32_t* __restrict__ tet, const double* __restrict__ Ke,
                           const double2* __restrict__ e, double2* __restrict__ y, double* __restrict__ q) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double re = 0.0, im = 0.0;
  for (int64_t k = vt_ptr[v]; k < vt_ptr[v + 1]; ++k) {
    const int64_t t = vt[k] >> 2;
    const int a = vt[k] & 3;
    for (int b = 0; b < 4; ++b) {
      const double kab = Ke[16 * t + 4 * a + b];
      const double2 eb = e[tet[4 * t + b]];
      re += kab * eb.x;
      im += kab * eb.y;
    }
  }
  y[v] = make_double2(re, im);
  q[v] = e[v].x * re + e[v].y * im;
}

// g += alpha y
__global__ void k_axpy_real(int64_t n, double alpha, const double2* __restrict__ y, double2* __restrict__ g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  g[i] = make_double2(g[i].x + alpha * y[i].x, g[i].y + alpha * y[i].y);
}

// fixed-order sum of q[0..n): 256 strided partial sums, then a tree (one workgroup)
__global__ void __launch_bounds__(256) k_sum(int64_t n, const double* __restrict__ q, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += q[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// w = 1 / |S_empty|^2 (inf where S_empty = 0: the caller is told)
__global__ void k_weights(int64_t count, const double2* __restrict__ Se, double* __restrict__ w) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double a = Se[i].x * Se[i].x + Se[i].y * Se[i].y;
  w[i] = 1.0 / a;
}

constexpr int GCHUNK = 2048;   // rows per partial sum of the Gram products

// part[chunk][i][j] = sum over the chunk's rows r of conj(X[r][i]) Y[r][j]
// (i < p, j < q): one workgroup per (row chunk, 16 x 16 output tile), every
// sum over the chunk's rows in row order
__global__ void __launch_bounds__(256) k_xhy_partial(const double2* __restrict__ X, int p,
                                                     const double2* __restrict__ Y, int q, int64_t n,
                                                     int tiles_q, double2* __restrict__ part) {
  const int64_t ch = blockIdx.x;
  const int ti = blockIdx.y / tiles_q, tj = blockIdx.y % tiles_q;
  const int i = 16 * ti + (threadIdx.x >> 4), j = 16 * tj + (threadIdx.x & 15);
  const int64_t r0 = ch * GCHUNK, r1 = min(n, r0 + GCHUNK);
  double re = 0.0, im = 0.0;
  if (i < p && j < q)
    for (int64_t r = r0; r < r1; ++r) {
      const double2 x = X[r * p + i], y = Y[r * q + j];
      re += x.x * y.x + x.y * y.y;
      im += x.x * y.y - x.y * y.x;
    }
  if (i < p && j < q) part[ch * (int64_t)p * q + (int64_t)i * q + j] = make_double2(re, im);
}

// Z[r][c] = sum_k U[r][k] Yc[k][c] (n x p times p x p)
__global__ void k_times_small(const double2* __restrict__ U, const double2* __restrict__ Yc, int p, int64_t n,
                              double2* __restrict__ Z) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t r = id / p;
  const int c = (int)(id % p);
  if (r >= n) return;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < p; ++k) {
    const double2 u = U[r * p + k], y = Yc[(int64_t)k * p + c];
    re += u.x * y.x - u.y * y.y;
    im += u.x * y.y + u.y * y.x;
  }
  Z[r * p + c] = make_double2(re, im);
}

void status_check(mw_status s) {
  if (s != MW_OK) fail(s, mw_last_error());
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

}  // namespace

struct mw_inversion {
  mw_problem* p = nullptr;
  mw_inversion_opts o{};
  int64_t nv = 0, nt = 0, n = 0;
  int32_t ntx = 0, nrx = 0;
  std::vector<int32_t> tx, rx, part;
  bool own_part = false;
  DevBuf tet, Ke, vt_ptr, vt, S_meas, w, S, gS, eps_t, ev, gt, gv, ky, q, red, B, U, F, Lam;
  DevBuf AU, X0, gpart, gram;   // recycle = 2: A U, the projected start, Gram partials and sums
  bool have_prev = false;
  // per evaluation: mean GMRES iterations of the forward and adjoint solves
  std::vector<double> it_fwd, it_adj;
  int64_t solve_columns = 0;
  double seconds = 0.0;
};

namespace {

// recycle = 2: X (the previous solution of A X = B's predecessor) is replaced
// by X Y with Y minimising ||B - A X Y||_F: the Gram matrices (AX)^H (AX) and
// (AX)^H B on the device, the p x p Cholesky solve on the host (a relative
// shift of 1e-13 on the diagonal keeps it defined when two previous fields
// are nearly parallel; any Y is a valid start)
void project_start(mw_inversion* I, double2* X, const double2* B) {
  mw_problem* p = I->p;
  hipStream_t st = problem_stream(p);
  const int pc = I->ntx;
  const int64_t n = I->n;
  problem_spmm(p, X, I->AU.as<double2>(), pc, pc, nullptr);
  const int64_t nch = ceil_div(n, GCHUNK);
  const int tq = (int)ceil_div(pc, 16);
  double2* part = I->gpart.as<double2>();
  double2* G = I->gram.as<double2>();
  const int64_t pp = (int64_t)pc * pc;
  k_xhy_partial<<<dim3((unsigned)nch, (unsigned)(tq * tq)), 256, 0, st>>>(I->AU.as<double2>(), pc,
                                                                         I->AU.as<double2>(), pc, n, tq, part);
  MW_LAUNCH_CHECK();
  launch_sum_chunks_c(part, nch, pp, G, st);
  k_xhy_partial<<<dim3((unsigned)nch, (unsigned)(tq * tq)), 256, 0, st>>>(I->AU.as<double2>(), pc, B, pc, n, tq,
                                                                         part);
  MW_LAUNCH_CHECK();
  launch_sum_chunks_c(part, nch, pp, G + pp, st);
  std::vector<double2> h(2 * pp);
  MW_HIP(hipMemcpyAsync(h.data(), G, 2 * pp * 16, hipMemcpyDeviceToHost, st));
  MW_HIP(hipStreamSynchronize(st));
  // Cholesky G = L L^H (lower, row-major), then L L^H Y = R column by column
  std::vector<double> Lr(pp, 0.0), Li(pp, 0.0);
  double dmax = 0.0;
  for (int k = 0; k < pc; ++k) dmax = std::max(dmax, h[(int64_t)k * pc + k].x);
  const double shift = 1e-13 * dmax;
  for (int j = 0; j < pc; ++j) {
    double d = h[(int64_t)j * pc + j].x + shift;
    for (int k = 0; k < j; ++k) d -= Lr[j * pc + k] * Lr[j * pc + k] + Li[j * pc + k] * Li[j * pc + k];
    if (!(d > 0.0)) return;   // not positive definite in floating point: keep the current start
    const double l = std::sqrt(d);
    Lr[j * pc + j] = l;
    for (int r = j + 1; r < pc; ++r) {
      // L[r][j] = (G[r][j] - sum_k L[r][k] conj(L[j][k])) / L[j][j]
      double sr = h[(int64_t)r * pc + j].x, si = h[(int64_t)r * pc + j].y;
      for (int k = 0; k < j; ++k) {
        sr -= Lr[r * pc + k] * Lr[j * pc + k] + Li[r * pc + k] * Li[j * pc + k];
        si -= Li[r * pc + k] * Lr[j * pc + k] - Lr[r * pc + k] * Li[j * pc + k];
      }
      Lr[r * pc + j] = sr / l;
      Li[r * pc + j] = si / l;
    }
  }
  std::vector<double2> Y(pp);
  for (int c = 0; c < pc; ++c) {
    std::vector<double> zr(pc), zi(pc);
    for (int r = 0; r < pc; ++r) {   // L z = R[:, c]
      double sr = h[pp + (int64_t)r * pc + c].x, si = h[pp + (int64_t)r * pc + c].y;
      for (int k = 0; k < r; ++k) {
        sr -= Lr[r * pc + k] * zr[k] - Li[r * pc + k] * zi[k];
        si -= Lr[r * pc + k] * zi[k] + Li[r * pc + k] * zr[k];
      }
      zr[r] = sr / Lr[r * pc + r];
      zi[r] = si / Lr[r * pc + r];
    }
    for (int r = pc - 1; r >= 0; --r) {   // L^H y = z
      double sr = zr[r], si = zi[r];
      for (int k = r + 1; k < pc; ++k) {   // conj(L[k][r]) y_k
        const double ar = Lr[k * pc + r], ai = -Li[k * pc + r];
        sr -= ar * Y[(int64_t)k * pc + c].x - ai * Y[(int64_t)k * pc + c].y;
        si -= ar * Y[(int64_t)k * pc + c].y + ai * Y[(int64_t)k * pc + c].x;
      }
      Y[(int64_t)r * pc + c] = make_double2(sr / Lr[r * pc + r], si / Lr[r * pc + r]);
    }
  }
  MW_HIP(hipMemcpyAsync(G, Y.data(), pp * 16, hipMemcpyHostToDevice, st));
  k_times_small<<<(unsigned)ceil_div(n * pc, 256), 256, 0, st>>>(X, G, pc, n, I->X0.as<double2>());
  MW_LAUNCH_CHECK();
  MW_HIP(hipMemcpyAsync(X, I->X0.p, n * pc * 16, hipMemcpyDeviceToDevice, st));
  MW_HIP(hipStreamSynchronize(st));
}

// J and gradient (device [nv]) at the vertex field ev (device [nv])
double evaluate(mw_inversion* I, const double2* ev, double2* gv) {
  mw_problem* p = I->p;
  hipStream_t st = problem_stream(p);
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t nt = I->nt, nv = I->nv, n = I->n;
  if (I->o.p1) {
    status_check(mw_update_eps_vertex(p, ev));
  } else {
    k_vertex_mean<<<(unsigned)ceil_div(nt, 256), 256, 0, st>>>(nt, I->tet.as<int32_t>(), ev, I->eps_t.as<double2>());
    MW_LAUNCH_CHECK();
    status_check(mw_update_eps(p, I->eps_t.p));
  }
  status_check(mw_factor_subdomains(p, I->o.n_sub, I->o.overlap, (mw_precision)I->o.precision,
                                    I->own_part ? I->part.data() : nullptr));
  status_check(mw_rhs_ports(p, I->ntx, I->tx.data(), I->B.p));
  mw_solve_opts so = I->o.solve;
  so.use_x0 = (I->o.recycle && I->have_prev) ? 1 : 0;
  if (I->o.recycle == 2 && I->have_prev) project_start(I, I->U.as<double2>(), I->B.as<double2>());
  std::vector<int32_t> its(I->ntx);
  mw_solve_info info{};
  info.iters = its.data();
  status_check(mw_solve(p, I->ntx, I->B.p, I->U.p, &so, &info));
  I->it_fwd.push_back(std::accumulate(its.begin(), its.end(), 0.0) / std::max(1, I->ntx));
  status_check(mw_s_matrix(p, I->nrx, I->rx.data(), I->ntx, I->U.p, I->S.p));
  double Jd = 0.0;
  status_check(mw_misfit_weighted(p, (int64_t)I->nrx * I->ntx, I->S.p, I->S_meas.p, I->w.as<double>(), I->gS.p, &Jd));
  status_check(mw_adjoint_rhs(p, I->nrx, I->rx.data(), I->ntx, I->gS.p, I->Lam.p));
  if (I->o.recycle == 2 && I->have_prev) project_start(I, I->F.as<double2>(), I->Lam.as<double2>());
  status_check(mw_solve(p, I->ntx, I->Lam.p, I->F.p, &so, &info));
  I->it_adj.push_back(std::accumulate(its.begin(), its.end(), 0.0) / std::max(1, I->ntx));
  I->have_prev = true;
  if (I->o.p1) {
    status_check(mw_gradient_vertex(p, I->ntx, I->U.p, I->F.p, gv));
  } else {
    status_check(mw_gradient(p, I->ntx, I->U.p, I->F.p, I->gt.p));
    k_vertex_gather<<<(unsigned)ceil_div(nv, 256), 256, 0, st>>>(nv, I->vt_ptr.as<int64_t>(), I->vt.as<int32_t>(),
                                                                 I->gt.as<double2>(), gv);
    MW_LAUNCH_CHECK();
  }
  double R = 0.0;
  if (I->o.alpha != 0.0) {
    k_p1_apply<<<(unsigned)ceil_div(nv, 256), 256, 0, st>>>(nv, I->vt_ptr.as<int64_t>(), I->vt.as<int32_t>(),
                                                            I->tet.as<int32_t>(), I->Ke.as<double>(), ev,
                                                            I->ky.as<double2>(), I->q.as<double>());
    MW_LAUNCH_CHECK();
    k_axpy_real<<<(unsigned)ceil_div(nv, 256), 256, 0, st>>>(nv, I->o.alpha, I->ky.as<double2>(), gv);
    MW_LAUNCH_CHECK();
    k_sum<<<1, 256, 0, st>>>(nv, I->q.as<double>(), I->red.as<double>());
    MW_LAUNCH_CHECK();
    MW_HIP(hipMemcpyAsync(&R, I->red.p, 8, hipMemcpyDeviceToHost, st));
    MW_HIP(hipStreamSynchronize(st));
    R *= 0.5 * I->o.alpha;
  }
  MW_HIP(hipStreamSynchronize(st));
  I->solve_columns += 2 * (int64_t)I->ntx;
  I->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  (void)n;
  return Jd + R;
}

struct RunCtx {
  mw_inversion* I;
  std::vector<double2> hx, hg;
};

// objective of mw_lbfgs over x = [Re e; Im e]
mw_status run_objective(void* user, const double* x, double* J, double* g) {
  return guarded([&] {
    auto* R = static_cast<RunCtx*>(user);
    mw_inversion* I = R->I;
    const int64_t nv = I->nv;
    hipStream_t st = problem_stream(I->p);
    for (int64_t v = 0; v < nv; ++v) R->hx[v] = make_double2(x[v], x[nv + v]);
    MW_HIP(hipMemcpyAsync(I->ev.p, R->hx.data(), nv * 16, hipMemcpyHostToDevice, st));
    *J = evaluate(I, I->ev.as<double2>(), I->gv.as<double2>());
    MW_HIP(hipMemcpyAsync(R->hg.data(), I->gv.p, nv * 16, hipMemcpyDeviceToHost, st));
    MW_HIP(hipStreamSynchronize(st));
    for (int64_t v = 0; v < nv; ++v) {
      g[v] = R->hg[v].x;
      g[nv + v] = R->hg[v].y;
    }
  });
}

}  // namespace

extern "C" {

mw_status mw_lbfgs(int64_t n, double* x, int32_t iters, const mw_lbfgs_opts* o, mw_objective_fn f, void* user,
                   double* J_hist, double* x_hist, int32_t* accepted, int32_t* evaluations) {
  return guarded([&] {
    MW_CHECK(n >= 1 && x && o && f && iters >= 0, MW_EINVAL, "NULL argument or bad size");
    MW_CHECK(o->mem >= 1 && o->step0 > 0 && o->c1 > 0 && o->c1 < 1 && o->max_backtrack >= 1, MW_EINVAL,
             "L-BFGS options out of range");
    const size_t N = (size_t)n;
    std::vector<double> xc(x, x + N), g(N), d(N), xn(N), gn(N);
    int32_t nev = 0, acc = 0;
    double J = 0.0;
    auto call = [&](const std::vector<double>& xx, double& JJ, std::vector<double>& gg) {
      ++nev;
      mw_status s = f(user, xx.data(), &JJ, gg.data());
      if (s != MW_OK) fail(s, std::string("objective failed: ") + mw_last_error());
    };
    call(xc, J, g);
    if (J_hist) J_hist[0] = J;
    if (x_hist) std::copy(xc.begin(), xc.end(), x_hist);
    struct Pair { std::vector<double> s, y; double rho; };
    std::deque<Pair> pairs;                        // oldest first
    for (int32_t it = 0; it < iters; ++it) {
      // two-loop recursion: d = -H g
      for (size_t i = 0; i < N; ++i) d[i] = -g[i];
      std::vector<double> coef;
      for (auto pr = pairs.rbegin(); pr != pairs.rend(); ++pr) {
        const double a = pr->rho * dot(pr->s, d);
        for (size_t i = 0; i < N; ++i) d[i] -= a * pr->y[i];
        coef.push_back(a);
      }
      double step;
      if (!pairs.empty()) {
        const Pair& l = pairs.back();
        const double sc = dot(l.s, l.y) / dot(l.y, l.y);
        for (size_t i = 0; i < N; ++i) d[i] *= sc;
        step = 1.0;
      } else {
        double m = 0.0;
        for (size_t i = 0; i < N; ++i) m = std::max(m, std::fabs(d[i]));
        MW_CHECK(m > 0.0, MW_EINVAL, "zero gradient at the starting point");
        step = o->step0 / m;
      }
      size_t k = coef.size();
      for (const Pair& pr : pairs) {
        const double a = coef[--k];
        const double b = a - pr.rho * dot(pr.y, d);
        for (size_t i = 0; i < N; ++i) d[i] += b * pr.s[i];
      }
      const double slope = dot(g, d);
      bool ok = false;
      double Jn = 0.0;
      for (int32_t bt = 0; bt < o->max_backtrack; ++bt) {
        for (size_t i = 0; i < N; ++i) xn[i] = xc[i] + step * d[i];
        call(xn, Jn, gn);
        if (Jn <= J + o->c1 * step * slope) { ok = true; break; }
        step *= 0.5;
      }
      if (!ok) break;
      Pair pr{std::vector<double>(N), std::vector<double>(N), 0.0};
      for (size_t i = 0; i < N; ++i) {
        pr.s[i] = xn[i] - xc[i];
        pr.y[i] = gn[i] - g[i];
      }
      const double sy = dot(pr.s, pr.y);
      if (sy > 1e-12 * std::sqrt(dot(pr.s, pr.s) * dot(pr.y, pr.y))) {
        pr.rho = 1.0 / sy;
        pairs.push_back(std::move(pr));
        if ((int)pairs.size() > o->mem) pairs.pop_front();
      }
      xc.swap(xn);
      g.swap(gn);
      J = Jn;
      ++acc;
      if (J_hist) J_hist[acc] = J;
      if (x_hist) std::copy(xc.begin(), xc.end(), x_hist + (size_t)acc * N);
    }
    std::copy(xc.begin(), xc.end(), x);
    if (accepted) *accepted = acc;
    if (evaluations) *evaluations = nev;
  });
}

mw_status mw_inversion_create(mw_problem* p, const mw_mesh* mesh, const int32_t* tet_part, const mw_inversion_opts* o,
                              int32_t ntx, const int32_t* tx, int32_t nrx, const int32_t* rx, const void* S_meas,
                              const void* S_empty, mw_inversion** out) {
  return guarded([&] {
    MW_CHECK(p && mesh && o && tx && rx && S_meas && S_empty && out, MW_EINVAL, "NULL argument");
    MW_CHECK(ntx >= 1 && nrx >= 1, MW_EINVAL, "need at least one transmitting and one receiving port");
    MW_CHECK(o->precision == MW_C64 || o->precision == MW_C128, MW_EINVAL, "precision must be MW_C64 or MW_C128");
    MW_CHECK(o->n_sub >= 1 && o->overlap >= 1, MW_EINVAL, "n_sub and overlap must be >= 1");
    MW_CHECK(o->recycle >= 0 && o->recycle <= 2, MW_EINVAL, "recycle must be 0, 1 or 2");
    mw_problem_info pi{};
    status_check(mw_problem_get_info(p, &pi));
    MW_CHECK(mesh->nt == pi.nt, MW_EINVAL, "mesh does not match the problem (number of tetrahedra)");
    for (int j = 0; j < ntx; ++j) MW_CHECK(tx[j] >= 0 && tx[j] < pi.nports, MW_EINVAL, "tx port out of range");
    for (int j = 0; j < nrx; ++j) MW_CHECK(rx[j] >= 0 && rx[j] < pi.nports, MW_EINVAL, "rx port out of range");
    DeviceGuard dg(problem_device(p));
    hipStream_t st = problem_stream(p);
    auto I = std::make_unique<mw_inversion>();
    I->p = p;
    I->o = *o;
    I->nv = mesh->nv;
    I->nt = mesh->nt;
    I->n = pi.n;
    I->ntx = ntx;
    I->nrx = nrx;
    I->tx.assign(tx, tx + ntx);
    I->rx.assign(rx, rx + nrx);
    if (tet_part) {
      I->part.assign(tet_part, tet_part + mesh->nt);
      I->own_part = true;
    }
    const int64_t nt = I->nt, nv = I->nv, n = I->n;
    std::vector<int32_t> tet(mesh->tet, mesh->tet + 4 * nt);
    for (int32_t v : tet) MW_CHECK(v >= 0 && v < nv, MW_EINVAL, "tetrahedron vertex out of range");
    // (t*4 + slot) entries of every vertex, ascending t
    std::vector<int64_t> ptr(nv + 1, 0);
    for (int64_t e = 0; e < 4 * nt; ++e) ptr[tet[e] + 1]++;
    for (int64_t v = 0; v < nv; ++v) ptr[v + 1] += ptr[v];
    std::vector<int32_t> lst(4 * nt);
    {
      std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
      for (int64_t e = 0; e < 4 * nt; ++e) lst[fill[tet[e]]++] = (int32_t)e;
    }
    std::vector<double> xyz(mesh->xyz, mesh->xyz + 3 * nv);
    const int64_t cnt = (int64_t)nrx * ntx;
    I->tet = problem_upload(p, tet.data(), tet.size() * 4);
    I->vt_ptr = problem_upload(p, ptr.data(), ptr.size() * 8);
    I->vt = problem_upload(p, lst.data(), lst.size() * 4);
    DevBuf dxyz = problem_upload(p, xyz.data(), xyz.size() * 8);
    I->Ke = problem_alloc(p, nt * 16 * 8);
    k_p1_stiffness<<<(unsigned)ceil_div(nt, 256), 256, 0, st>>>(nt, dxyz.as<double>(), I->tet.as<int32_t>(),
                                                                I->Ke.as<double>());
    MW_LAUNCH_CHECK();
    I->S_meas = problem_alloc(p, cnt * 16);
    MW_HIP(hipMemcpyAsync(I->S_meas.p, S_meas, cnt * 16, hipMemcpyDeviceToDevice, st));
    I->w = problem_alloc(p, cnt * 8);
    k_weights<<<(unsigned)ceil_div(cnt, 256), 256, 0, st>>>(cnt, (const double2*)S_empty, I->w.as<double>());
    MW_LAUNCH_CHECK();
    std::vector<double> hw(cnt);
    MW_HIP(hipMemcpyAsync(hw.data(), I->w.p, cnt * 8, hipMemcpyDeviceToHost, st));
    MW_HIP(hipStreamSynchronize(st));
    for (double x : hw) MW_CHECK(std::isfinite(x), MW_EINVAL, "S_empty has a zero entry: the normalised misfit is undefined");
    I->S = problem_alloc(p, cnt * 16);
    I->gS = problem_alloc(p, cnt * 16);
    I->eps_t = problem_alloc(p, nt * 16);
    I->gt = problem_alloc(p, nt * 16);
    I->ev = problem_alloc(p, nv * 16);
    I->gv = problem_alloc(p, nv * 16);
    I->ky = problem_alloc(p, nv * 16);
    I->q = problem_alloc(p, nv * 8);
    I->red = problem_alloc(p, 256);
    I->B = problem_alloc(p, n * ntx * 16);
    I->U = problem_alloc(p, n * ntx * 16);
    I->F = problem_alloc(p, n * ntx * 16);
    I->Lam = problem_alloc(p, n * ntx * 16);
    if (o->recycle == 2) {
      I->AU = problem_alloc(p, n * ntx * 16);
      I->X0 = problem_alloc(p, n * ntx * 16);
      I->gpart = problem_alloc(p, ceil_div(n, GCHUNK) * (int64_t)ntx * ntx * 16);
      I->gram = problem_alloc(p, 2 * (int64_t)ntx * ntx * 16);
    }
    MW_HIP(hipStreamSynchronize(st));
    problem_retain(p);
    *out = I.release();
  });
}

mw_status mw_inversion_objective(mw_inversion* inv, const void* eps_v, double* J, void* grad) {
  return guarded([&] {
    MW_CHECK(inv && eps_v && J && grad, MW_EINVAL, "NULL argument");
    DeviceGuard dg(problem_device(inv->p));
    *J = evaluate(inv, (const double2*)eps_v, (double2*)grad);
  });
}

mw_status mw_inversion_run(mw_inversion* inv, const mw_lbfgs_opts* lo, int32_t iters, void* eps_v, double* J_hist,
                           void* eps_hist, int32_t* accepted, int32_t* evaluations) {
  return guarded([&] {
    MW_CHECK(inv && lo && eps_v && iters >= 0, MW_EINVAL, "NULL argument");
    DeviceGuard dg(problem_device(inv->p));
    hipStream_t st = problem_stream(inv->p);
    const int64_t nv = inv->nv;
    std::vector<double2> h(nv);
    MW_HIP(hipMemcpyAsync(h.data(), eps_v, nv * 16, hipMemcpyDeviceToHost, st));
    MW_HIP(hipStreamSynchronize(st));
    std::vector<double> x(2 * nv);
    for (int64_t v = 0; v < nv; ++v) {
      x[v] = h[v].x;
      x[nv + v] = h[v].y;
    }
    RunCtx rc{inv, std::vector<double2>(nv), std::vector<double2>(nv)};
    std::vector<double> xh;
    if (eps_hist) xh.resize((size_t)(iters + 1) * 2 * nv);
    int32_t acc = 0, nev = 0;
    status_check(mw_lbfgs(2 * nv, x.data(), iters, lo, run_objective, &rc, J_hist, eps_hist ? xh.data() : nullptr,
                          &acc, &nev));
    for (int64_t v = 0; v < nv; ++v) h[v] = make_double2(x[v], x[nv + v]);
    MW_HIP(hipMemcpyAsync(eps_v, h.data(), nv * 16, hipMemcpyHostToDevice, st));
    MW_HIP(hipStreamSynchronize(st));
    if (eps_hist) {
      auto* out = static_cast<double2*>(eps_hist);
      for (int32_t k = 0; k <= acc; ++k)
        for (int64_t v = 0; v < nv; ++v)
          out[(size_t)k * nv + v] = make_double2(xh[(size_t)k * 2 * nv + v], xh[(size_t)k * 2 * nv + nv + v]);
    }
    if (accepted) *accepted = acc;
    if (evaluations) *evaluations = nev;
  });
}

mw_status mw_inversion_get_info(mw_inversion* inv, int32_t cap, double* iters_forward, double* iters_adjoint,
                                mw_inversion_info* info) {
  return guarded([&] {
    MW_CHECK(inv != nullptr, MW_EINVAL, "NULL argument");
    const int32_t ne = (int32_t)inv->it_fwd.size();
    for (int32_t k = 0; k < std::min(cap, ne); ++k) {
      if (iters_forward) iters_forward[k] = inv->it_fwd[k];
      if (iters_adjoint) iters_adjoint[k] = inv->it_adj[k];
    }
    if (info) {
      info->evaluations = ne;
      info->solve_columns = inv->solve_columns;
      info->seconds = inv->seconds;
    }
  });
}

mw_status mw_inversion_destroy(mw_inversion* inv) {
  return guarded([&] {
    if (!inv) return;
    DeviceGuard dg(problem_device(inv->p));
    (void)hipStreamSynchronize(problem_stream(inv->p));
    problem_release(inv->p);
    delete inv;
  });
}

}  // extern "C"
