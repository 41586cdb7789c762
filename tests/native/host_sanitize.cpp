// Host-side checks of the library's mesh and decomposition code, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by the CPU tests (no GPU):
// topology, internal partition, overlapping decompositions, factor storage
// tables and the block least-squares routine run on a mesh read from a file,
// and their outputs are checked for consistency.  Prints "OK" and exits 0
// when every check holds; any sanitizer report makes the process fail.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "mw.h"

static int failures = 0;
#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

template <class T>
static bool read_vec(std::FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  return std::fread(v.data(), sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s mesh.bin\n", argv[0]);
    return 2;
  }
  // file: int32 nv, nt, nbf, n_sub; xyz (f64 nv*3), tet (i32 nt*4),
  // bface (i32 nbf*3), btag (i32 nbf), part (i32 nt)
  std::FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[4];
  if (std::fread(hdr, 4, 4, f) != 4) return 2;
  const int32_t nv = hdr[0], nt = hdr[1], nbf = hdr[2], n_sub = hdr[3];
  std::vector<double> xyz;
  std::vector<int32_t> tet, bface, btag, part;
  if (!read_vec(f, xyz, (size_t)nv * 3) || !read_vec(f, tet, (size_t)nt * 4) || !read_vec(f, bface, (size_t)nbf * 3) ||
      !read_vec(f, btag, (size_t)nbf) || !read_vec(f, part, (size_t)nt))
    return 2;
  std::fclose(f);
  mw_mesh mesh{nv, xyz.data(), nt, tet.data(), nbf, bface.data(), btag.data()};

  // topology: sizes, then the arrays
  int64_t n = 0, nnz = 0, ne = 0;
  CHECK(mw_host_topology(&mesh, &n, &nnz, &ne, nullptr, nullptr, nullptr) == MW_OK);
  CHECK(n > 0 && n <= ne && nnz >= n);
  std::vector<int32_t> edge_of_dof(n), col(nnz);
  std::vector<int64_t> row_ptr(n + 1);
  CHECK(mw_host_topology(&mesh, &n, &nnz, &ne, edge_of_dof.data(), row_ptr.data(), col.data()) == MW_OK);
  CHECK(row_ptr[0] == 0 && row_ptr[n] == nnz);
  for (int64_t r = 0; r < n; ++r) {
    CHECK(row_ptr[r] < row_ptr[r + 1]);
    CHECK(edge_of_dof[r] >= 0 && edge_of_dof[r] < ne);
    bool diag = false;
    for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      CHECK(col[k] >= 0 && col[k] < n);
      if (k > row_ptr[r]) CHECK(col[k] > col[k - 1]);
      diag = diag || col[k] == r;
    }
    CHECK(diag);
  }

  // internal partition: every part used, ids in range
  std::vector<int32_t> rcb(nt, -1);
  CHECK(mw_host_partition(&mesh, n_sub, rcb.data()) == MW_OK);
  std::vector<int32_t> count(n_sub, 0);
  for (int32_t t = 0; t < nt; ++t) {
    CHECK(rcb[t] >= 0 && rcb[t] < n_sub);
    if (rcb[t] >= 0 && rcb[t] < n_sub) ++count[rcb[t]];
  }
  for (int32_t i = 0; i < n_sub; ++i) CHECK(count[i] > 0);
  CHECK(mw_host_partition(&mesh, 0, rcb.data()) == MW_EINVAL);
  CHECK(mw_host_partition(&mesh, nt + 1, rcb.data()) == MW_EINVAL);

  // decompositions for the given partition and the internal one, two overlaps
  for (int which = 0; which < 2; ++which) {
    const int32_t* tp = which == 0 ? part.data() : rcb.data();
    for (int32_t overlap = 1; overlap <= 2; ++overlap) {
      std::vector<int32_t> n_loc(n_sub);
      std::vector<int64_t> n_faces(n_sub);
      CHECK(mw_host_decomposition(&mesh, tp, n_sub, overlap, n_loc.data(), n_faces.data(), nullptr, nullptr) ==
            MW_OK);
      int64_t total = 0;
      for (int32_t i = 0; i < n_sub; ++i) total += n_loc[i];
      CHECK(total >= n);
      std::vector<int32_t> sub_dof(total);
      std::vector<double> D(total);
      CHECK(mw_host_decomposition(&mesh, tp, n_sub, overlap, n_loc.data(), nullptr, sub_dof.data(), D.data()) ==
            MW_OK);
      std::vector<double> sum(n, 0.0);
      std::vector<int32_t> seen(n, -1);
      int64_t o = 0;
      for (int32_t i = 0; i < n_sub; ++i) {
        for (int32_t l = 0; l < n_loc[i]; ++l) {
          const int32_t g = sub_dof[o + l];
          CHECK(g >= 0 && g < n);
          CHECK(D[o + l] >= 0.0 && D[o + l] <= 1.0);
          if (g >= 0 && g < n) {
            sum[g] += D[o + l];
            CHECK(seen[g] != i);   // R_i picks every unknown at most once
            seen[g] = i;
          }
        }
        o += n_loc[i];
      }
      for (int64_t g = 0; g < n; ++g) CHECK(std::fabs(sum[g] - 1.0) < 1e-12);
      // factor storage tables of the first and last subdomains
      for (int32_t sub : {0, n_sub - 1}) {
        const int32_t npad = (n_loc[sub] + 63) / 64 * 64;
        std::vector<int32_t> lo(npad / 64), hi(npad / 64);
        int64_t dense = 0, band = 0;
        CHECK(mw_host_factor_storage(&mesh, tp, n_sub, overlap, sub, lo.data(), hi.data(), &dense, &band) == MW_OK);
        CHECK(band > 0 && band <= dense);
        for (int32_t b = 0; b < npad / 64; ++b) {
          CHECK(lo[b] % 64 == 0 && hi[b] % 64 == 0);
          CHECK(lo[b] <= 64 * b && hi[b] >= 64 * b + 64 && hi[b] <= npad);
        }
      }
      CHECK(mw_host_factor_storage(&mesh, tp, n_sub, overlap, n_sub, nullptr, nullptr, nullptr, nullptr) ==
            MW_EINVAL);
    }
  }
  // a part id out of range is refused, not read past
  {
    std::vector<int32_t> bad(part);
    bad[nt / 2] = n_sub;
    std::vector<int32_t> n_loc(n_sub);
    CHECK(mw_host_decomposition(&mesh, bad.data(), n_sub, 1, n_loc.data(), nullptr, nullptr, nullptr) != MW_OK);
  }

  // block least squares: two block steps on random data, and the Cholesky mode
  {
    std::mt19937_64 rng(7);
    std::normal_distribution<double> g;
    const int steps = 2, W = 32, ld = steps * W;
    std::vector<mw_complex> S0(W * W), H((size_t)(steps + 1) * W * ld), Y((size_t)steps * W * W);
    for (int r = 0; r < W; ++r)
      for (int c = 0; c < W; ++c) S0[r * W + c] = c >= r ? mw_complex{g(rng) + (r == c ? 4.0 : 0.0), g(rng)} : mw_complex{0, 0};
    for (int r = 0; r < (steps + 1) * W; ++r)
      for (int c = 0; c < ld; ++c) {
        const int br = r / W, bc = c / W;
        const bool nz = br <= bc || (br == bc + 1 && (c % W) >= (r % W));
        H[(size_t)r * ld + c] = nz ? mw_complex{g(rng) + (r == c ? 3.0 : 0.0), g(rng)} : mw_complex{0, 0};
      }
    std::vector<double> resid(steps * W);
    CHECK(mw_host_block_lstsq(steps, 20, S0.data(), H.data(), 0.0, resid.data(), Y.data()) == MW_OK);
    for (double v : resid) CHECK(std::isfinite(v) && v >= 0.0);
    std::vector<mw_complex> G(W * W), R(W * W);
    for (int r = 0; r < W; ++r)
      for (int c = 0; c < W; ++c) {
        std::complex<double> s = 0;
        for (int k = 0; k < W; ++k) {
          const mw_complex a = H[(size_t)k * ld + r], b = H[(size_t)k * ld + c];
          s += std::conj(std::complex<double>(a.re, a.im)) * std::complex<double>(b.re, b.im);
        }
        G[r * W + c] = {s.real(), s.imag()};
      }
    double npiv = -1;
    CHECK(mw_host_block_lstsq(0, W, nullptr, G.data(), 1e-12, &npiv, R.data()) == MW_OK);
    CHECK(npiv >= 0);
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
