// Host-side FP64 mathematics of libsgw (projector tiles, KB exponential,
// Chebyshev coefficients, Bessel functions, Jacobi eigensolver, QP solve)
// exercised on small inputs, including rejected ones, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_host_sanitizers.py).
// Prints one line per check and exits non-zero on a failed expectation.
#include <cmath>
#include <cstdio>
#include <vector>

#include "common.h"

using namespace sgw;

static int failures = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) { std::printf("FAILED: %s\n", #c); ++failures; }      \
  } while (0)

static sgw_ctx *grid_ctx(int n, double h) {
  sgw_ctx *c = new sgw_ctx();   // released at exit (its destructor calls the HIP runtime)
  c->nx = c->ny = c->nz = n;
  c->N = (int64_t)n * n * n;
  c->h = h;
  c->dV = h * h * h;
  return c;
}

static void projectors(int n, double h, double rcut_over_rc) {
  sgw_ctx *c = grid_ctx(n, h);
  const double L = n * h;
  // two atoms: s + p_x,y,z on the first, s on the second (the second sits
  // across the periodic boundary)
  std::vector<double> pos = {0.5 * L, 0.5 * L + 0.1, 0.5 * L - 0.2, 0.05, L - 0.1, 0.5 * L};
  std::vector<int32_t> begin = {0, 4, 5}, l = {0, 1, 1, 1, 0}, m = {0, 0, 1, 2, 0};
  std::vector<double> rc = {0.9, 0.9, 0.9, 0.9, 0.7}, ekb = {-2.0, -1.0, -1.0, -1.0, 0.5};
  sgw_projectors P{2, pos.data(), begin.data(), l.data(), m.data(), rc.data(), ekb.data(),
                   rcut_over_rc};
  build_kb(c, &P);
  EXPECT(c->kb.nproj == 5 && c->kb_ntile > 0 && c->kb_support_points > 0);
  for (int p = 0; p < 5; ++p)
    EXPECT(std::fabs(c->kb.gram[p * 5 + p] - 1.0) < 1e-12);   // normalised on the grid
  EXPECT(kb_lambda_bound(c) >= 1.0);
  std::vector<double> K;
  kb_exponential_matrix(c, 0.05, K);
  EXPECT(K.size() == 2 * 25);
  bool finite = true;
  for (double x : K) finite = finite && std::isfinite(x);
  EXPECT(finite);
  std::printf("projectors n=%d: %d tiles, %lld support points\n", n, c->kb_ntile,
              (long long)c->kb_support_points);
  // rejected inputs raise sgw::Error, leaving no partial state behind
  std::vector<int32_t> badl = {0, 2, 1, 1, 0};
  sgw_projectors Q = P;
  Q.l = badl.data();
  bool threw = false;
  try { build_kb(grid_ctx(n, h), &Q); } catch (const Error &e) { threw = e.code == SGW_EUNSUPPORTED; }
  EXPECT(threw);
  std::vector<double> badrc = {0.9, -1.0, 0.9, 0.9, 0.7};
  Q = P;
  Q.rc = badrc.data();
  threw = false;
  try { build_kb(grid_ctx(n, h), &Q); } catch (const Error &e) { threw = e.code == SGW_EINVAL; }
  EXPECT(threw);
}

int main() {
  projectors(16, 0.7, 4.0);    // 16 x 8 x 4 tiles
  projectors(24, 0.6, 4.0);    // 8 x 8 x 8 tiles
  projectors(8, 0.7, 6.0);     // spheres wider than the box
  std::vector<double> a(300);
  fermi_coefficients(-0.3, 20.0, -2.0, 5.0, 300, a.data());
  EXPECT(std::isfinite(a[0]) && std::fabs(a[0]) <= 1.0);
  gapped_coefficients(-0.5, -0.2, 1e-7, -2.0, 5.0, 300, a.data());
  EXPECT(std::isfinite(a[299]));
  std::vector<double> b;
  const int nb = propagator_coefficients(-2.0, 5.0, 0.2, 1e-14, b);
  EXPECT(nb > 1 && (int)b.size() >= 2 * nb);
  std::vector<double> J;
  bessel_j(3.7, 40, J);
  EXPECT((int)J.size() == 41 && std::fabs(J[0] - (-0.3992302033711912)) < 1e-12);   // J_0(3.7)
  std::vector<double> A = {4, 1, 0, 1, 3, 1, 0, 1, 2}, vals, vecs;
  jacobi_eigen(3, A, vals, vecs);
  EXPECT(vals.size() == 3 && vals[0] <= vals[1] && vals[1] <= vals[2]);
  const int nt = 40;
  std::vector<double> sig(2 * (2 * nt + 1));
  for (int j = -nt; j <= nt; ++j) {   // a damped single pole
    const double t = 0.1 * j;
    sig[2 * (j + nt)] = 0.05 * std::exp(-0.3 * std::fabs(t)) * std::cos(0.8 * t);
    sig[2 * (j + nt) + 1] = -0.05 * std::exp(-0.3 * std::fabs(t)) * std::sin(0.8 * std::fabs(t));
  }
  double eg = 0, el = 0, z = 0;
  const int st = qp_solve(sig.data(), nt, 0.1, 0.75, -0.5, -0.2, 0.0, &eg, &el, &z);
  EXPECT(std::isfinite(el) && std::isfinite(z));
  std::printf("qp_solve status %d: eg %.6f el %.6f z %.4f\n", st, eg, el, z);
  std::printf("%s\n", failures ? "FAILURES" : "ALL OK");
  return failures ? 1 : 0;
}
