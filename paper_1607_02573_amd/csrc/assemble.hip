// Device assembly of the edge-element Maxwell operator and its sources
// (paper Section 2, variational form (pbdirectvarf); Section 2.1; Section 4,
// equation (sij); Section 5 adjoint gradient).
//
// Whitney functions N_ab = l_a grad l_b - l_b grad l_a on a tetrahedron with
// ascending vertices; barycentric gradients from the edge vectors
// d_k = x_k - x_0:  grad l_1 = (d2 x d3)/det, grad l_2 = (d3 x d1)/det,
// grad l_3 = (d1 x d2)/det, grad l_0 = -(sum), vol = |det|/6.  Closed forms:
//   K[p][q] = vol * (2 g_a x g_b) . (2 g_c x g_d)
//   M[p][q] = vol/20 [(1+d_ac) g_b.g_d - (1+d_ad) g_b.g_c - (1+d_bc) g_a.g_d + (1+d_bd) g_a.g_c]
// for p = (a,b), q = (c,d).  On a face the same mass form with the surface
// gradients and area/12 gives the tangential mass int (N_p x n).(N_q x n).
#include "kernels.hpp"

namespace mw {

__constant__ int c_tedge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
__constant__ int c_fedge[3][2] = {{0, 1}, {0, 2}, {1, 2}};

__device__ inline int sym21(int p, int q) {
  if (p > q) { int t = p; p = q; q = t; }
  return p * 6 - (p * (p - 1)) / 2 + (q - p);
}

struct V3 { double x, y, z; };
__device__ inline V3 v3(const double* p) { return {p[0], p[1], p[2]}; }
__device__ inline V3 vsub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 vadd(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 vmul(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline double vdot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 vcross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// barycentric gradients and volume of tetrahedron t
__device__ inline double tet_grads(const double* xyz, const int32_t* tet, int64_t t, V3 g[4]) {
  V3 x0 = v3(xyz + 3 * (int64_t)tet[t * 4 + 0]);
  V3 d1 = vsub(v3(xyz + 3 * (int64_t)tet[t * 4 + 1]), x0);
  V3 d2 = vsub(v3(xyz + 3 * (int64_t)tet[t * 4 + 2]), x0);
  V3 d3 = vsub(v3(xyz + 3 * (int64_t)tet[t * 4 + 3]), x0);
  double det = vdot(d1, vcross(d2, d3));
  double id = 1.0 / det;
  g[1] = vmul(vcross(d2, d3), id);
  g[2] = vmul(vcross(d3, d1), id);
  g[3] = vmul(vcross(d1, d2), id);
  g[0] = vmul(vadd(vadd(g[1], g[2]), g[3]), -1.0);
  return fabs(det) / 6.0;
}

__device__ inline double mass_entry(const V3* g, const int (*ed)[2], int p, int q, double scale) {
  int a = ed[p][0], b = ed[p][1], c = ed[q][0], d = ed[q][1];
  double mac = 1.0 + (a == c), mad = 1.0 + (a == d), mbc = 1.0 + (b == c), mbd = 1.0 + (b == d);
  return scale * (mac * vdot(g[b], g[d]) - mad * vdot(g[b], g[c]) - mbc * vdot(g[a], g[d]) +
                  mbd * vdot(g[a], g[c]));
}

// surface gradients (s[3]) and area of the triangle (v0, v1, v2)
__device__ inline double tri_grads(const double* xyz, int32_t a, int32_t b, int32_t c, V3 s[3]) {
  V3 p0 = v3(xyz + 3 * (int64_t)a), p1 = v3(xyz + 3 * (int64_t)b), p2 = v3(xyz + 3 * (int64_t)c);
  V3 e1 = vsub(p1, p0), e2 = vsub(p2, p0);
  V3 nn = vcross(e1, e2);
  double n2 = vdot(nn, nn);
  s[1] = vmul(vcross(e2, nn), 1.0 / n2);
  s[2] = vmul(vcross(nn, e1), 1.0 / n2);
  s[0] = vmul(vadd(s[1], s[2]), -1.0);
  return 0.5 * sqrt(n2);
}

// ---------------------------------------------------------------- K9a
// E_t = K_t - k0^2 eps_t M_t, 21 packed (p <= q) complex entries per tet.
__global__ void k_element_matrices(const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                                   const double2* __restrict__ eps, double k0sq, int64_t nt,
                                   double2* __restrict__ E) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  V3 g[4];
  double vol = tet_grads(xyz, tet, t, g);
  V3 cu[6];
  for (int p = 0; p < 6; ++p) cu[p] = vmul(vcross(g[c_tedge[p][0]], g[c_tedge[p][1]]), 2.0);
  double2 e = eps[t];
  double2* out = E + t * 21;
  for (int p = 0; p < 6; ++p)
    for (int q = p; q < 6; ++q) {
      double k = vol * vdot(cu[p], cu[q]);
      double m = mass_entry(g, c_tedge, p, q, vol / 20.0);
      out[sym21(p, q)] = make_double2(k - k0sq * e.x * m, -k0sq * e.y * m);
    }
}

// int_t l_v l_x l_y / vol (Section 6 discretises kappa with P1 elements):
// 1/120 for three different indices, 1/60 when exactly two agree, 1/20 when
// all three agree.
__device__ inline double w3(int v, int x, int y) {
  const int same = (v == x) + (v == y) + (x == y);
  return same == 0 ? 1.0 / 120.0 : (same == 1 ? 1.0 / 60.0 : 1.0 / 20.0);
}

// mass entry of a coefficient linear on the tetrahedron with vertex values
// ev[4]: sum_v ev[v] int l_v N_p . N_q = vol [W_ac g_b.g_d - W_ad g_b.g_c
// - W_bc g_a.g_d + W_bd g_a.g_c], W_xy = sum_v ev[v] w3(v, x, y)
__device__ inline double2 mass_entry_p1(const V3* g, int p, int q, double vol, const double2 ev[4]) {
  const int a = c_tedge[p][0], b = c_tedge[p][1], c = c_tedge[q][0], d = c_tedge[q][1];
  auto W = [&](int x, int y) {
    double2 s = make_double2(0.0, 0.0);
    for (int v = 0; v < 4; ++v) s = cadd(s, cscale(ev[v], w3(v, x, y)));
    return s;
  };
  const double2 wac = W(a, c), wad = W(a, d), wbc = W(b, c), wbd = W(b, d);
  const double gbd = vdot(g[b], g[d]), gbc = vdot(g[b], g[c]), gad = vdot(g[a], g[d]), gac = vdot(g[a], g[c]);
  return make_double2(vol * (wac.x * gbd - wad.x * gbc - wbc.x * gad + wbd.x * gac),
                      vol * (wac.y * gbd - wad.y * gbc - wbc.y * gad + wbd.y * gac));
}

// E_t with eps_r linear on the tetrahedron (vertex values eps_v), and the
// tetrahedron mean of eps_v (the coefficient the preconditioner's
// transmission wavenumber and the factorisation choice read)
__global__ void k_element_matrices_p1(const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                                      const double2* __restrict__ eps_v, double k0sq, int64_t nt,
                                      double2* __restrict__ E, double2* __restrict__ eps_t) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  V3 g[4];
  double vol = tet_grads(xyz, tet, t, g);
  double2 ev[4];
  for (int v = 0; v < 4; ++v) ev[v] = eps_v[tet[t * 4 + v]];
  V3 cu[6];
  for (int p = 0; p < 6; ++p) cu[p] = vmul(vcross(g[c_tedge[p][0]], g[c_tedge[p][1]]), 2.0);
  double2* out = E + t * 21;
  for (int p = 0; p < 6; ++p)
    for (int q = p; q < 6; ++q) {
      double k = vol * vdot(cu[p], cu[q]);
      double2 m = mass_entry_p1(g, p, q, vol, ev);
      out[sym21(p, q)] = make_double2(k - k0sq * m.x, -k0sq * m.y);
    }
  eps_t[t] = make_double2(0.25 * (ev[0].x + ev[1].x + ev[2].x + ev[3].x),
                          0.25 * (ev[0].y + ev[1].y + ev[2].y + ev[3].y));
}

void launch_element_matrices_p1(const DeviceMesh& m, const double2* eps_v, double k0, double2* E, double2* eps_t,
                                hipStream_t st) {
  k_element_matrices_p1<<<(unsigned)ceil_div(m.nt, 256), 256, 0, st>>>(m.xyz, m.tet, eps_v, k0 * k0, m.nt, E, eps_t);
  MW_LAUNCH_CHECK();
}

// row p of i*beta*M_F for the triangle (a,b,c) (ascending)
__device__ inline void face_row(const double* xyz, int32_t a, int32_t b, int32_t c, double2 beta,
                                int p, double2 out[3]) {
  V3 s[3];
  double area = tri_grads(xyz, a, b, c, s);
  for (int q = 0; q < 3; ++q) {
    double m = mass_entry(s, c_fedge, p, q, area / 12.0);
    out[q] = make_double2(-beta.y * m, beta.x * m);   // i * beta * m
  }
}

__device__ inline int64_t find_col(const int32_t* col, int64_t b, int64_t e, int32_t c) {
  while (b < e) {
    int64_t m = (b + e) >> 1;
    if (col[m] < c) b = m + 1; else e = m;
  }
  return b;
}

// ---------------------------------------------------------------- K9b
// A's values, one thread per row, contributions in a fixed order.
__global__ void k_gather_csr(int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             const int64_t* __restrict__ rt_ptr, const int32_t* __restrict__ rt,
                             const int64_t* __restrict__ rf_ptr, const int32_t* __restrict__ rf,
                             const int32_t* __restrict__ t2e, const int32_t* __restrict__ dof,
                             const double2* __restrict__ E, const int32_t* __restrict__ bface,
                             const int32_t* __restrict__ bf2e, const double2* __restrict__ fbeta,
                             const double* __restrict__ xyz, double2* __restrict__ val) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t b = row_ptr[r], e = row_ptr[r + 1];
  for (int64_t k = b; k < e; ++k) val[k] = make_double2(0.0, 0.0);
  for (int64_t k = rt_ptr[r]; k < rt_ptr[r + 1]; ++k) {
    int32_t tp = rt[k];
    int64_t t = tp / 6;
    int p = tp % 6;
    for (int q = 0; q < 6; ++q) {
      int32_t d = dof[t2e[t * 6 + q]];
      if (d < 0) continue;
      int64_t s = find_col(col, b, e, d);
      if (s < e && col[s] == d) val[s] = cadd(val[s], E[t * 21 + sym21(p, q)]);
    }
  }
  for (int64_t k = rf_ptr[r]; k < rf_ptr[r + 1]; ++k) {
    int32_t fp = rf[k];
    int64_t f = fp / 3;
    int p = fp % 3;
    double2 row[3];
    face_row(xyz, bface[f * 3], bface[f * 3 + 1], bface[f * 3 + 2], fbeta[f], p, row);
    for (int q = 0; q < 3; ++q) {
      int32_t d = dof[bf2e[f * 3 + q]];
      if (d < 0) continue;
      int64_t s = find_col(col, b, e, d);
      if (s < e && col[s] == d) val[s] = cadd(val[s], row[q]);
    }
  }
}

void launch_element_matrices(const DeviceMesh& m, const double2* eps, double k0, double2* E,
                             hipStream_t st) {
  int64_t nt = m.nt;
  k_element_matrices<<<(unsigned)ceil_div(nt, 256), 256, 0, st>>>(m.xyz, m.tet, eps, k0 * k0, nt, E);
  MW_LAUNCH_CHECK();
}

void launch_gather_csr(const DeviceMesh& m, const double2* E, double2* val, hipStream_t st) {
  k_gather_csr<<<(unsigned)ceil_div(m.n, 128), 128, 0, st>>>(
      m.n, m.row_ptr, m.col, m.rt_ptr, m.rt, m.rf_ptr, m.rf, m.t2e, m.dof, E, m.bface, m.bf2e,
      m.fbeta, m.xyz, val);
  MW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- K8
// Local matrices B_i in the factor storage (every stored entry zero, ones on
// the padding diagonal), then the volume, boundary and transmission terms,
// one thread per local row.
template <class C>
__global__ void k_fill_zero(C* __restrict__ F, const int64_t* __restrict__ fac_off) {
  const int i = blockIdx.y;
  const int64_t total = fac_off[i + 1] - fac_off[i];
  C* Fi = F + fac_off[i];
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    C z;
    z.x = 0;
    z.y = 0;
    Fi[k] = z;
  }
}

template <class C>
__global__ void k_fill_pad_diag(C* __restrict__ F, const int64_t* __restrict__ fac_off,
                                const int32_t* __restrict__ n_loc, const int32_t* __restrict__ n_pad,
                                const int64_t* __restrict__ boff, const int32_t* __restrict__ blo,
                                const int32_t* __restrict__ bw, int bstride) {
  const int i = blockIdx.x;
  C* Fi = F + fac_off[i];
  for (int r = n_loc[i] + (int)threadIdx.x; r < n_pad[i]; r += blockDim.x) {
    C one;
    one.x = 1;
    one.y = 0;
    frow(Fi, boff + (int64_t)i * bstride, blo + (int64_t)i * bstride, bw + (int64_t)i * bstride, r)[r] = one;
  }
}

template <class C>
__global__ void k_fill_local(C* __restrict__ F, const int64_t* __restrict__ fac_off,
                             const int64_t* __restrict__ loc_off, const int32_t* __restrict__ n_loc,
                             const int32_t* __restrict__ n_pad, const int64_t* __restrict__ lt_off,
                             const int32_t* __restrict__ lt_tet, const int32_t* __restrict__ lt_loc,
                             const int64_t* __restrict__ lf_off, const int32_t* __restrict__ lf_vert,
                             const int32_t* __restrict__ lf_owner, const int32_t* __restrict__ lf_kind,
                             const int32_t* __restrict__ lf_loc, const int64_t* __restrict__ rtl_ptr,
                             const int32_t* __restrict__ rtl, const int64_t* __restrict__ rfl_ptr,
                             const int32_t* __restrict__ rfl, const double2* __restrict__ E,
                             const double2* __restrict__ fbeta, const double2* __restrict__ eps,
                             const double* __restrict__ xyz, double k0, const int64_t* __restrict__ boff,
                             const int32_t* __restrict__ blo, const int32_t* __restrict__ bw, int bstride) {
  int i = blockIdx.y;
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_loc[i]) return;
  // every entry of row l lies in its structural envelope, stored
  C* row = frow(F + fac_off[i], boff + (int64_t)i * bstride, blo + (int64_t)i * bstride, bw + (int64_t)i * bstride, l);
  int64_t r = loc_off[i] + l;
  const int32_t* tl = lt_loc + lt_off[i] * 6;
  const int32_t* tt = lt_tet + lt_off[i];
  for (int64_t k = rtl_ptr[r]; k < rtl_ptr[r + 1]; ++k) {
    int32_t ep = rtl[k];
    int64_t ent = ep / 6;
    int p = ep % 6;
    int64_t t = tt[ent];
    for (int q = 0; q < 6; ++q) {
      int32_t c = tl[ent * 6 + q];
      if (c < 0) continue;
      double2 v = E[t * 21 + sym21(p, q)];
      C o = row[c];
      o.x += v.x; o.y += v.y;
      row[c] = o;
    }
  }
  const int32_t* fl = lf_loc + lf_off[i] * 3;
  const int32_t* fv = lf_vert + lf_off[i] * 3;
  for (int64_t k = rfl_ptr[r]; k < rfl_ptr[r + 1]; ++k) {
    int32_t ep = rfl[k];
    int64_t ent = ep / 3;
    int p = ep % 3;
    int32_t kind = lf_kind[lf_off[i] + ent];
    double2 beta;
    if (kind >= 0) beta = fbeta[kind];
    else beta = make_double2(k0 * sqrt(eps[lf_owner[lf_off[i] + ent]].x), 0.0);
    double2 vals[3];
    face_row(xyz, fv[ent * 3], fv[ent * 3 + 1], fv[ent * 3 + 2], beta, p, vals);
    for (int q = 0; q < 3; ++q) {
      int32_t c = fl[ent * 3 + q];
      if (c < 0) continue;
      C o = row[c];
      o.x += vals[q].x; o.y += vals[q].y;
      row[c] = o;
    }
  }
}

template <class C>
void launch_fill_local(const DeviceMesh& m, const DeviceDecomp& d, const double2* E, const double2* eps,
                       double k0, C* F, hipStream_t st) {
  k_fill_zero<C><<<dim3(1024, d.nsub), 256, 0, st>>>(F, d.fac_off);
  MW_LAUNCH_CHECK();
  k_fill_pad_diag<C><<<d.nsub, 64, 0, st>>>(F, d.fac_off, d.n_loc, d.n_pad, d.boff, d.blo, d.bw, d.bstride);
  MW_LAUNCH_CHECK();
  dim3 g2((unsigned)ceil_div(d.max_pad, 128), d.nsub);
  k_fill_local<C><<<g2, 128, 0, st>>>(F, d.fac_off, d.loc_off, d.n_loc, d.n_pad, d.lt_off, d.lt_tet,
                                      d.lt_loc, d.lf_off, d.lf_vert, d.lf_owner, d.lf_kind, d.lf_loc,
                                      d.rtl_ptr, d.rtl, d.rfl_ptr, d.rfl, E, m.fbeta, eps, m.xyz, k0, d.boff, d.blo,
                                      d.bw, d.bstride);
  MW_LAUNCH_CHECK();
}
template void launch_fill_local<float2>(const DeviceMesh&, const DeviceDecomp&, const double2*,
                                        const double2*, double, float2*, hipStream_t);
template void launch_fill_local<double2>(const DeviceMesh&, const DeviceDecomp&, const double2*,
                                         const double2*, double, double2*, hipStream_t);

// ---------------------------------------------------------------- ports
// Port projections p_k[e] = int_{Gamma_k} E0_k . N_e with the edge-midpoint
// rule (weights area/3) and nu_k = int |E0_k|^2 (E0 tangential part).
__device__ inline V3 port_mode(const PortDev& pt, V3 x) {
  double phi = atan2(x.y, x.x);
  double d = phi - pt.theta;
  d = atan2(sin(d), cos(d));
  double s = pt.radius * d;
  double a = cos(M_PI * s / pt.width);
  return {pt.pol[0] * a, pt.pol[1] * a, pt.pol[2] * a};
}

// value of face f's contribution to the unknown on its local edge q
__device__ inline double port_face_value(const double* xyz, const int32_t* bface, int64_t f,
                                         const PortDev& pt, int q) {
  int32_t vid[3] = {bface[f * 3], bface[f * 3 + 1], bface[f * 3 + 2]};
  V3 s[3];
  double area = tri_grads(xyz, vid[0], vid[1], vid[2], s);
  V3 P[3] = {v3(xyz + 3 * (int64_t)vid[0]), v3(xyz + 3 * (int64_t)vid[1]), v3(xyz + 3 * (int64_t)vid[2])};
  V3 nn = vcross(vsub(P[1], P[0]), vsub(P[2], P[0]));
  nn = vmul(nn, 1.0 / sqrt(vdot(nn, nn)));
  double acc = 0.0;
  for (int m = 0; m < 3; ++m) {             // midpoint of face edge m
    int u = c_fedge[m][0], w = c_fedge[m][1];
    double lam[3] = {0, 0, 0};
    lam[u] = lam[w] = 0.5;
    V3 xm = vmul(vadd(P[u], P[w]), 0.5);
    V3 e0 = port_mode(pt, xm);
    e0 = vsub(e0, vmul(nn, vdot(e0, nn)));
    int a = c_fedge[q][0], b = c_fedge[q][1];
    V3 Nq = vsub(vmul(s[b], lam[a]), vmul(s[a], lam[b]));
    acc += (area / 3.0) * vdot(e0, Nq);
  }
  return acc;
}

// one thread per (port, distinct unknown): sum of its face contributions
__global__ void k_port_vectors(int64_t nentries, const int32_t* __restrict__ ent_port,
                               const int64_t* __restrict__ ent_ptr, const int32_t* __restrict__ ent_fq,
                               const PortDev* __restrict__ ports, const double* __restrict__ xyz,
                               const int32_t* __restrict__ bface, double* __restrict__ pval) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nentries) return;
  const PortDev pt = ports[ent_port[k]];
  double acc = 0.0;
  for (int64_t j = ent_ptr[k]; j < ent_ptr[k + 1]; ++j) {
    int32_t fq = ent_fq[j];
    acc += port_face_value(xyz, bface, fq / 3, pt, fq % 3);
  }
  pval[k] = acc;
}

// one thread per port: nu_k over its faces in ascending order
__global__ void k_port_norms(int nports, const int64_t* __restrict__ pf_ptr, const int32_t* __restrict__ pf,
                             const PortDev* __restrict__ ports, const double* __restrict__ xyz,
                             const int32_t* __restrict__ bface, double* __restrict__ nu) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nports) return;
  const PortDev pt = ports[k];
  double acc = 0.0;
  for (int64_t j = pf_ptr[k]; j < pf_ptr[k + 1]; ++j) {
    int64_t f = pf[j];
    int32_t vid[3] = {bface[f * 3], bface[f * 3 + 1], bface[f * 3 + 2]};
    V3 s[3];
    double area = tri_grads(xyz, vid[0], vid[1], vid[2], s);
    V3 P[3] = {v3(xyz + 3 * (int64_t)vid[0]), v3(xyz + 3 * (int64_t)vid[1]), v3(xyz + 3 * (int64_t)vid[2])};
    V3 nn = vcross(vsub(P[1], P[0]), vsub(P[2], P[0]));
    nn = vmul(nn, 1.0 / sqrt(vdot(nn, nn)));
    for (int m = 0; m < 3; ++m) {
      V3 xm = vmul(vadd(P[c_fedge[m][0]], P[c_fedge[m][1]]), 0.5);
      V3 e0 = port_mode(pt, xm);
      e0 = vsub(e0, vmul(nn, vdot(e0, nn)));
      acc += (area / 3.0) * vdot(e0, e0);
    }
  }
  nu[k] = acc;
}

void launch_port_setup(const DeviceMesh& m, const DevicePorts& P, hipStream_t st) {
  if (P.nports == 0) return;
  if (P.nent > 0) {
    k_port_vectors<<<(unsigned)ceil_div(P.nent, 128), 128, 0, st>>>(P.nent, P.ent_port, P.ent_ptr, P.ent_fq,
                                                                     P.ports, m.xyz, m.bface, P.pval);
    MW_LAUNCH_CHECK();
  }
  k_port_norms<<<(unsigned)ceil_div(P.nports, 64), 64, 0, st>>>(P.nports, P.pf_ptr, P.pf, P.ports, m.xyz,
                                                                 m.bface, P.nu);
  MW_LAUNCH_CHECK();
}

// B[:, j] = 2 i beta_k p_k for k = tx[j]  (B zeroed by the caller)
__global__ void k_rhs_ports(int ntx, const int32_t* __restrict__ tx, const int64_t* __restrict__ port_ptr,
                            const int32_t* __restrict__ ent_dof, const double* __restrict__ pval,
                            const PortDev* __restrict__ ports, double2* __restrict__ B, int64_t ldb) {
  int j = blockIdx.y;
  int k = tx[j];
  double2 beta = ports[k].beta;
  double2 c = make_double2(-2.0 * beta.y, 2.0 * beta.x);     // 2 i beta
  for (int64_t e = port_ptr[k] + threadIdx.x + (int64_t)blockIdx.x * blockDim.x; e < port_ptr[k + 1];
       e += (int64_t)gridDim.x * blockDim.x)
    B[(int64_t)ent_dof[e] * ldb + j] = cscale(c, pval[e]);
}

void launch_rhs_ports(const DevicePorts& P, int ntx, const int32_t* tx_dev, double2* B, int64_t ldb,
                      hipStream_t st) {
  dim3 g(1, ntx);
  k_rhs_ports<<<g, 128, 0, st>>>(ntx, tx_dev, P.port_ptr, P.ent_dof, P.pval, P.ports, B, ldb);
  MW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- dipoles
// lowest-index tetrahedron containing each point (barycentrics >= -1e-12)
__global__ void k_locate(const double* __restrict__ xyz, const int32_t* __restrict__ tet, int64_t nt,
                         const double* __restrict__ pts, int np, int* __restrict__ found) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  V3 g[4];
  tet_grads(xyz, tet, t, g);
  V3 x0 = v3(xyz + 3 * (int64_t)tet[t * 4]);
  for (int j = 0; j < np; ++j) {
    V3 d = vsub(v3(pts + 3 * j), x0);
    double l1 = vdot(g[1], d), l2 = vdot(g[2], d), l3 = vdot(g[3], d);
    double l0 = 1.0 - l1 - l2 - l3;
    if (l0 >= -1e-12 && l1 >= -1e-12 && l2 >= -1e-12 && l3 >= -1e-12) atomicMin(found + j, (int)t);
  }
}

// B[dof(e), j] = dir_j . N_e(x_j) on the 6 edges of the located tetrahedron
__global__ void k_rhs_dipoles(const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                              const int32_t* __restrict__ t2e, const int32_t* __restrict__ dof,
                              const double* __restrict__ pts, const double* __restrict__ dirs,
                              const int* __restrict__ found, int np, double2* __restrict__ B, int64_t ldb) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np) return;
  int64_t t = found[j];
  V3 g[4];
  tet_grads(xyz, tet, t, g);
  V3 x0 = v3(xyz + 3 * (int64_t)tet[t * 4]);
  V3 d = vsub(v3(pts + 3 * j), x0);
  double lam[4];
  lam[1] = vdot(g[1], d); lam[2] = vdot(g[2], d); lam[3] = vdot(g[3], d);
  lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
  V3 dir = v3(dirs + 3 * j);
  for (int p = 0; p < 6; ++p) {
    int32_t k = dof[t2e[t * 6 + p]];
    if (k < 0) continue;
    int a = c_tedge[p][0], b = c_tedge[p][1];
    V3 N = vsub(vmul(g[b], lam[a]), vmul(g[a], lam[b]));
    B[(int64_t)k * ldb + j] = make_double2(vdot(dir, N), 0.0);
  }
}

void launch_locate(const DeviceMesh& m, const double* pts, int np, int* found, hipStream_t st) {
  k_locate<<<(unsigned)ceil_div(m.nt, 256), 256, 0, st>>>(m.xyz, m.tet, m.nt, pts, np, found);
  MW_LAUNCH_CHECK();
}
void launch_rhs_dipoles(const DeviceMesh& m, const double* pts, const double* dirs, const int* found,
                        int np, double2* B, int64_t ldb, hipStream_t st) {
  k_rhs_dipoles<<<(unsigned)ceil_div(np, 64), 64, 0, st>>>(m.xyz, m.tet, m.t2e, m.dof, pts, dirs, found, np,
                                                            B, ldb);
  MW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- K11
// S[i][j] = conj(p_{rx_i}^T U[:, j]) / nu_{rx_i}
__global__ void k_s_matrix(int nrx, int ntx, const int32_t* __restrict__ rx, const int64_t* __restrict__ port_ptr,
                           const int32_t* __restrict__ ent_dof, const double* __restrict__ pval,
                           const double* __restrict__ nu, const double2* __restrict__ U, int64_t ldu,
                           double2* __restrict__ S) {
  int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= (int64_t)nrx * ntx) return;
  int i = (int)(id / ntx), j = (int)(id % ntx);
  int k = rx[i];
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t e = port_ptr[k]; e < port_ptr[k + 1]; ++e)
    acc = cadd(acc, cscale(U[(int64_t)ent_dof[e] * ldu + j], pval[e]));
  S[id] = make_double2(acc.x / nu[k], -acc.y / nu[k]);
}

void launch_s_matrix(const DevicePorts& P, int nrx, const int32_t* rx_dev, int ntx, const double2* U,
                     int64_t ldu, double2* S, hipStream_t st) {
  int64_t tot = (int64_t)nrx * ntx;
  if (tot == 0) return;
  k_s_matrix<<<(unsigned)ceil_div(tot, 128), 128, 0, st>>>(nrx, ntx, rx_dev, P.port_ptr, P.ent_dof, P.pval,
                                                            P.nu, U, ldu, S);
  MW_LAUNCH_CHECK();
}

// adjoint sources  Lambda[:, j] = sum_i gS[i][j] p_{rx_i} / nu_{rx_i}  (Lambda zeroed)
__global__ void k_adjoint_rhs(int nrx, int ntx, const int32_t* __restrict__ rx, const int64_t* __restrict__ port_ptr,
                              const int32_t* __restrict__ ent_dof, const double* __restrict__ pval,
                              const double* __restrict__ nu, const double2* __restrict__ gS,
                              double2* __restrict__ L, int64_t ldl) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ntx) return;
  for (int i = 0; i < nrx; ++i) {
    int k = rx[i];
    double2 c = cscale(gS[(int64_t)i * ntx + j], 1.0 / nu[k]);
    for (int64_t e = port_ptr[k]; e < port_ptr[k + 1]; ++e) {
      int64_t o = (int64_t)ent_dof[e] * ldl + j;
      L[o] = cadd(L[o], cscale(c, pval[e]));
    }
  }
}

void launch_adjoint_rhs(const DevicePorts& P, int nrx, const int32_t* rx_dev, int ntx, const double2* gS,
                        double2* L, int64_t ldl, hipStream_t st) {
  k_adjoint_rhs<<<(unsigned)ceil_div(ntx, 64), 64, 0, st>>>(nrx, ntx, rx_dev, P.port_ptr, P.ent_dof, P.pval,
                                                             P.nu, gS, L, ldl);
  MW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- K10
// grad_t = conj(k0^2 sum_j f_j|_t^T M_t u_j|_t)
__global__ void k_gradient(const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                           const int32_t* __restrict__ t2e, const int32_t* __restrict__ dof, int64_t nt,
                           const double2* __restrict__ U, const double2* __restrict__ F, int64_t ld, int ncol,
                           double k0sq, double2* __restrict__ grad) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  V3 g[4];
  double vol = tet_grads(xyz, tet, t, g);
  double M[21];
  for (int p = 0; p < 6; ++p)
    for (int q = p; q < 6; ++q) M[sym21(p, q)] = mass_entry(g, c_tedge, p, q, vol / 20.0);
  int32_t d[6];
  for (int p = 0; p < 6; ++p) d[p] = dof[t2e[t * 6 + p]];
  double2 acc = make_double2(0.0, 0.0);
  for (int j = 0; j < ncol; ++j) {
    double2 u[6], f[6];
    for (int p = 0; p < 6; ++p) {
      u[p] = d[p] >= 0 ? U[(int64_t)d[p] * ld + j] : make_double2(0.0, 0.0);
      f[p] = d[p] >= 0 ? F[(int64_t)d[p] * ld + j] : make_double2(0.0, 0.0);
    }
    for (int p = 0; p < 6; ++p) {
      double2 mu = make_double2(0.0, 0.0);
      for (int q = 0; q < 6; ++q) mu = cadd(mu, cscale(u[q], M[sym21(p, q)]));
      acc = cadd(acc, cmul(f[p], mu));
    }
  }
  grad[t] = make_double2(k0sq * acc.x, -k0sq * acc.y);
}

void launch_gradient(const DeviceMesh& m, const double2* U, const double2* F, int64_t ld, int ncol, double k0,
                     double2* grad, hipStream_t st) {
  k_gradient<<<(unsigned)ceil_div(m.nt, 128), 128, 0, st>>>(m.xyz, m.tet, m.t2e, m.dof, m.nt, U, F, ld, ncol,
                                                             k0 * k0, grad);
  MW_LAUNCH_CHECK();
}

// Vertex gradient for eps_r linear on every tetrahedron: G[t][v] =
// conj(k0^2 sum_j f_j|_t^T M1_v u_j|_t), M1_v = int l_v N_p . N_q, then
// grad[v] = sum of G over the (t, slot) pairs of vertex v in a fixed order
// (k_vertex_sum, one thread per vertex).
__global__ void k_gradient_p1(const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                              const int32_t* __restrict__ t2e, const int32_t* __restrict__ dof, int64_t nt,
                              const double2* __restrict__ U, const double2* __restrict__ F, int64_t ld, int ncol,
                              double k0sq, double2* __restrict__ G) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  V3 g[4];
  double vol = tet_grads(xyz, tet, t, g);
  int32_t d[6];
  for (int p = 0; p < 6; ++p) d[p] = dof[t2e[t * 6 + p]];
  for (int v = 0; v < 4; ++v) {
    double2 ev[4];
    for (int u = 0; u < 4; ++u) ev[u] = make_double2(u == v ? 1.0 : 0.0, 0.0);
    double M[21];
    for (int p = 0; p < 6; ++p)
      for (int q = p; q < 6; ++q) M[sym21(p, q)] = mass_entry_p1(g, p, q, vol, ev).x;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < ncol; ++j) {
      double2 uu[6], ff[6];
      for (int p = 0; p < 6; ++p) {
        uu[p] = d[p] >= 0 ? U[(int64_t)d[p] * ld + j] : make_double2(0.0, 0.0);
        ff[p] = d[p] >= 0 ? F[(int64_t)d[p] * ld + j] : make_double2(0.0, 0.0);
      }
      for (int p = 0; p < 6; ++p) {
        double2 mu = make_double2(0.0, 0.0);
        for (int q = 0; q < 6; ++q) mu = cadd(mu, cscale(uu[q], M[sym21(p, q)]));
        acc = cadd(acc, cmul(ff[p], mu));
      }
    }
    G[t * 4 + v] = make_double2(k0sq * acc.x, -k0sq * acc.y);
  }
}

__global__ void k_vertex_sum(int64_t nv, const int64_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt,
                             const double2* __restrict__ G, double2* __restrict__ grad) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double2 s = make_double2(0.0, 0.0);
  for (int64_t k = vt_ptr[v]; k < vt_ptr[v + 1]; ++k) s = cadd(s, G[vt[k]]);
  grad[v] = s;
}

void launch_gradient_p1(const DeviceMesh& m, const double2* U, const double2* F, int64_t ld, int ncol, double k0,
                        const int64_t* vt_ptr, const int32_t* vt, double2* G, double2* grad, hipStream_t st) {
  k_gradient_p1<<<(unsigned)ceil_div(m.nt, 128), 128, 0, st>>>(m.xyz, m.tet, m.t2e, m.dof, m.nt, U, F, ld, ncol,
                                                                k0 * k0, G);
  MW_LAUNCH_CHECK();
  k_vertex_sum<<<(unsigned)ceil_div(m.nv, 256), 256, 0, st>>>(m.nv, vt_ptr, vt, G, grad);
  MW_LAUNCH_CHECK();
}

// out[0] = max_t Im eps_t (one workgroup, fixed order): every B_i has a
// positive definite imaginary part when it is negative (lossy media with the
// e^{+i omega t} convention), which selects the symmetric factorisation.
__global__ void __launch_bounds__(1024) k_max_imag(const double2* __restrict__ eps, int64_t nt,
                                                   double* __restrict__ out) {
  __shared__ double red[1024];
  double m = -INFINITY;
  for (int64_t t = threadIdx.x; t < nt; t += 1024) m = fmax(m, eps[t].y);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}
void launch_max_imag(const double2* eps, int64_t nt, double* out, hipStream_t st) {
  k_max_imag<<<1, 1024, 0, st>>>(eps, nt, out);
  MW_LAUNCH_CHECK();
}

}  // namespace mw
