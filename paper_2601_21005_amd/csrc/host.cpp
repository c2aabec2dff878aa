// Host-side FP64 mathematics of libsgw: projector tiles and Gram matrix,
// the exact KB exponential matrix, Chebyshev coefficients, Bessel functions
// and the quasi-particle equation.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <thread>

#include "common.h"

namespace sgw {

using cd = std::complex<double>;

// ---------------------------------------------------------------- projectors
// beta_p(r) = N_p Y(d) exp(-|d|^2 / (2 rc^2)) on |d| <= rcut (minimum-image
// displacement d), normalised on the grid; laid out per 8x8x8 tile.
void build_kb(sgw_ctx *ctx, const sgw_projectors *P) {
  KBHost &kb = ctx->kb;
  const int na = P->natom;
  SGW_REQUIRE(na > 0 && P->pos && P->proj_begin && P->l && P->m && P->rc && P->ekb,
              SGW_EINVAL, "projectors: null array");
  SGW_REQUIRE(P->proj_begin[0] == 0, SGW_EINVAL, "projectors: proj_begin[0] != 0");
  const int np = P->proj_begin[na];
  SGW_REQUIRE(np > 0, SGW_EINVAL, "projectors: no projector");
  SGW_REQUIRE(P->rcut_over_rc > 0 && std::isfinite(P->rcut_over_rc), SGW_EINVAL,
              "projectors: rcut_over_rc must be > 0");
  // 512-point tiles: 16 x 8 x 4 (rows of 16 complex = 128 B in FP32) when the
  // grid allows it, else 8 x 8 x 8
  int td[3] = {8, 8, 8};
  if (ctx->nx % 16 == 0 && ctx->ny % 8 == 0 && ctx->nz % 4 == 0) { td[0] = 16; td[1] = 8; td[2] = 4; }
  SGW_REQUIRE(ctx->nx % td[0] == 0 && ctx->ny % td[1] == 0 && ctx->nz % td[2] == 0,
              SGW_EUNSUPPORTED, "projectors need grid sizes divisible by 8");
  ctx->kb_lx = td[0] == 16 ? 4 : 3;
  ctx->kb_ly = 3;
  const int n[3] = {ctx->nx, ctx->ny, ctx->nz};
  const double h = ctx->h;
  const double L[3] = {n[0] * h, n[1] * h, n[2] * h};
  const int tn[3] = {n[0] / td[0], n[1] / td[1], n[2] / td[2]};
  const int ntile_all = tn[0] * tn[1] * tn[2];

  struct Pt { int64_t r; double v; };
  std::vector<std::vector<Pt>> pts(np);
  kb.nproj = np;
  kb.ekb.assign(P->ekb, P->ekb + np);
  for (int a = 0; a < na; ++a) {
    SGW_REQUIRE(P->proj_begin[a + 1] >= P->proj_begin[a], SGW_EINVAL, "projectors: bad CSR");
    const double *R = P->pos + 3 * a;
    SGW_REQUIRE(std::isfinite(R[0]) && std::isfinite(R[1]) && std::isfinite(R[2]), SGW_EINVAL,
                "projectors: non-finite position");
    for (int p = P->proj_begin[a]; p < P->proj_begin[a + 1]; ++p) {
      const int l = P->l[p], m = P->m[p];
      const double rc = P->rc[p];
      SGW_REQUIRE(l == 0 || l == 1, SGW_EUNSUPPORTED, "projectors: only l = 0, 1");
      SGW_REQUIRE(m >= 0 && m <= 2 * l, SGW_EINVAL, "projectors: m out of range");
      SGW_REQUIRE(rc > 0 && std::isfinite(rc) && std::isfinite(P->ekb[p]), SGW_EINVAL,
                  "projectors: bad rc or ekb");
      const double rcut = P->rcut_over_rc * rc;
      int lo[3], cnt[3];
      for (int ax = 0; ax < 3; ++ax) {
        lo[ax] = (int)std::floor((R[ax] - rcut) / h);
        cnt[ax] = std::min(n[ax], (int)std::floor(2 * rcut / h) + 2);
      }
      double nrm = 0;
      auto &v = pts[p];
      for (int k = 0; k < cnt[2]; ++k)
        for (int j = 0; j < cnt[1]; ++j)
          for (int i = 0; i < cnt[0]; ++i) {
            const int idx[3] = {((lo[0] + i) % n[0] + n[0]) % n[0],
                                ((lo[1] + j) % n[1] + n[1]) % n[1],
                                ((lo[2] + k) % n[2] + n[2]) % n[2]};
            double d[3], d2 = 0;
            for (int ax = 0; ax < 3; ++ax) {
              double x = idx[ax] * h - R[ax];
              x = std::fmod(x + 0.5 * L[ax], L[ax]);
              if (x < 0) x += L[ax];
              d[ax] = x - 0.5 * L[ax];
              d2 += d[ax] * d[ax];
            }
            if (d2 > rcut * rcut) continue;
            double g = std::exp(-d2 / (2 * rc * rc));
            if (l == 1) g *= d[m];
            const int64_t r = idx[0] + (int64_t)n[0] * (idx[1] + (int64_t)n[1] * idx[2]);
            v.push_back({r, g});
            nrm += g * g;
          }
      nrm = std::sqrt(nrm * ctx->dV);
      SGW_REQUIRE(nrm > 0, SGW_EINVAL, "projector has no support on the grid");
      for (auto &q : v) q.v /= nrm;
      std::sort(v.begin(), v.end(), [](const Pt &x, const Pt &y) { return x.r < y.r; });
    }
  }
  auto tile_of = [&](int64_t r, int &local) {
    const int ix = (int)(r % n[0]);
    const int iy = (int)((r / n[0]) % n[1]);
    const int iz = (int)(r / ((int64_t)n[0] * n[1]));
    local = (ix % td[0]) + td[0] * ((iy % td[1]) + td[1] * (iz % td[2]));
    return (ix / td[0]) + tn[0] * ((iy / td[1]) + tn[1] * (iz / td[2]));
  };
  // projector lists per tile (ascending projector ids)
  std::vector<std::vector<int>> tproj(ntile_all);
  for (int p = 0; p < np; ++p) {
    int last = -1;
    std::vector<int> ts;
    for (auto &q : pts[p]) {
      int loc;
      ts.push_back(tile_of(q.r, loc));
    }
    std::sort(ts.begin(), ts.end());
    for (int t : ts)
      if (t != last) { tproj[t].push_back(p); last = t; }
  }
  std::vector<int> tile_index(ntile_all, -1);
  kb.tile_base.clear();
  kb.tile_off.assign(1, 0);
  kb.entry_proj.clear();
  for (int t = 0; t < ntile_all; ++t) {
    if (tproj[t].empty()) continue;
    tile_index[t] = (int)kb.tile_base.size();
    const int tx = t % tn[0], ty = (t / tn[0]) % tn[1], tz = t / (tn[0] * tn[1]);
    kb.tile_base.push_back(tx * td[0] + n[0] * (ty * td[1] + n[1] * tz * td[2]));
    for (int p : tproj[t]) kb.entry_proj.push_back(p);
    kb.tile_off.push_back((int)kb.entry_proj.size());
  }
  const int ntile = (int)kb.tile_base.size();
  const int nentry = (int)kb.entry_proj.size();
  kb.beta.assign((size_t)nentry * KB_TP, 0.0);
  for (int p = 0; p < np; ++p)
    for (auto &q : pts[p]) {
      int loc;
      const int t = tile_index[tile_of(q.r, loc)];
      const int off = kb.tile_off[t];
      const int cnt = kb.tile_off[t + 1] - off;
      const int *lst = kb.entry_proj.data() + off;
      const int pos = (int)(std::lower_bound(lst, lst + cnt, p) - lst);
      kb.beta[(size_t)(off + pos) * KB_TP + loc] = q.v;
    }
  int maxe = 0;
  for (int t = 0; t < ntile; ++t) maxe = std::max(maxe, kb.tile_off[t + 1] - kb.tile_off[t]);
  SGW_REQUIRE(maxe <= 256, SGW_EUNSUPPORTED, "more than 256 projectors meet one 512-point tile");
  // entries grouped per projector, ascending entry id
  kb.proj_off.assign(np + 1, 0);
  for (int e = 0; e < nentry; ++e) kb.proj_off[kb.entry_proj[e] + 1]++;
  for (int p = 0; p < np; ++p) kb.proj_off[p + 1] += kb.proj_off[p];
  kb.proj_entries.assign(nentry, 0);
  std::vector<int> fill(kb.proj_off.begin(), kb.proj_off.end() - 1);
  for (int e = 0; e < nentry; ++e) kb.proj_entries[fill[kb.entry_proj[e]]++] = e;
  // Gram matrix S_pq = dV sum_r beta_p beta_q
  kb.gram.assign((size_t)np * np, 0.0);
  for (int t = 0; t < ntile; ++t)
    for (int a = kb.tile_off[t]; a < kb.tile_off[t + 1]; ++a)
      for (int b = a; b < kb.tile_off[t + 1]; ++b) {
        const double *x = &kb.beta[(size_t)a * KB_TP];
        const double *y = &kb.beta[(size_t)b * KB_TP];
        double s = 0;
        for (int i = 0; i < KB_TP; ++i) s += x[i] * y[i];
        s *= ctx->dV;
        const int p = kb.entry_proj[a], q = kb.entry_proj[b];
        kb.gram[(size_t)p * np + q] += s;
        if (p != q) kb.gram[(size_t)q * np + p] += s;
      }
  ctx->kb_ntile = ntile;
  ctx->kb_nentry = nentry;
  // grid points inside some projector's support, and nonzero beta values
  ctx->kb_support_points = 0;
  ctx->kb_nnz = 0;
  kb.mask.assign((size_t)ntile * (KB_TP / 32), 0u);
  for (int t = 0; t < ntile; ++t)
    for (int i = 0; i < KB_TP; ++i) {
      int hit = 0;
      for (int e = kb.tile_off[t]; e < kb.tile_off[t + 1]; ++e)
        hit += kb.beta[(size_t)e * KB_TP + i] != 0.0;
      ctx->kb_support_points += hit > 0;
      ctx->kb_nnz += hit;
      if (hit) kb.mask[(size_t)t * (KB_TP / 32) + i / 32] |= 1u << (i % 32);
    }
}

// lambda_max(S) <= max_p sum_q |S_pq|  (Gershgorin)
double kb_lambda_bound(const sgw_ctx *ctx) {
  const int np = ctx->kb.nproj;
  double smax = 0;
  for (int p = 0; p < np; ++p) {
    double s = 0;
    for (int q = 0; q < np; ++q) s += std::fabs(ctx->kb.gram[(size_t)p * np + q]);
    smax = std::max(smax, s);
  }
  return smax;
}

// ---------------------------------------------------------------- KB exponential
// C = A B (n x n, row-major); rows of C split over host threads (each row is
// summed in the same order whatever the thread count)
static void cmatmul(const std::vector<cd> &A, const std::vector<cd> &B, std::vector<cd> &C,
                    int n) {
  C.assign((size_t)n * n, cd(0, 0));
  auto rows = [&](int i0, int i1) {
    for (int i = i0; i < i1; ++i)
      for (int k = 0; k < n; ++k) {
        const cd a = A[(size_t)i * n + k];
        if (a == cd(0, 0)) continue;
        const double ar = a.real(), ai = a.imag();
        const double *b = reinterpret_cast<const double *>(&B[(size_t)k * n]);
        double *c = reinterpret_cast<double *>(&C[(size_t)i * n]);
        for (int j = 0; j < n; ++j) {
          const double br = b[2 * j], bi = b[2 * j + 1];
          c[2 * j] += ar * br - ai * bi;
          c[2 * j + 1] += ar * bi + ai * br;
        }
      }
  };
  const int nt = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), n / 64));
  if (nt <= 1) {
    rows(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int per = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int i0 = t * per, i1 = std::min(n, i0 + per);
    if (i0 < i1) th.emplace_back(rows, i0, i1);
  }
  for (auto &x : th) x.join();
}

// exp(-i tau V_NL) = I + dV B K B^T with K = (-i tau) E phi1(X), X = -i tau S E,
// phi1(X) = sum_k X^k/(k+1)!; phi1 by scaling and squaring:
// phi1(2Y) = phi1(Y) (e^Y + I) / 2, e^{2Y} = (e^Y)^2.
void kb_exponential_matrix(const sgw_ctx *ctx, double tau, std::vector<double> &Kout) {
  const int n = ctx->kb.nproj;
  const auto &S = ctx->kb.gram;
  const auto &E = ctx->kb.ekb;
  std::vector<cd> X((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) X[(size_t)i * n + j] = cd(0, -tau) * S[(size_t)i * n + j] * E[j];
  double norm1 = 0;
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += std::abs(X[(size_t)i * n + j]);
    norm1 = std::max(norm1, s);
  }
  int sq = 0;
  while (norm1 > 0.5) { norm1 *= 0.5; ++sq; }
  const double scale = std::ldexp(1.0, -sq);
  for (auto &x : X) x *= scale;
  // Taylor: eY = sum Y^k/k!, P = sum Y^k/(k+1)!
  std::vector<cd> eY((size_t)n * n, cd(0, 0)), Pm((size_t)n * n, cd(0, 0)), term, tmp;
  for (int i = 0; i < n; ++i) { eY[(size_t)i * n + i] = 1; Pm[(size_t)i * n + i] = 1; }
  term = X;  // Y^1
  double fact = 1;
  for (int k = 1; k <= 30; ++k) {
    fact *= k;  // k!
    double tn = 0;
    for (size_t q = 0; q < term.size(); ++q) {
      eY[q] += term[q] / fact;
      Pm[q] += term[q] / (fact * (k + 1));
      tn = std::max(tn, std::abs(term[q]));
    }
    if (tn / fact < 1e-20) break;
    cmatmul(term, X, tmp, n);
    term.swap(tmp);
  }
  for (int s = 0; s < sq; ++s) {
    std::vector<cd> ep = eY;
    for (int i = 0; i < n; ++i) ep[(size_t)i * n + i] += 1.0;
    cmatmul(Pm, ep, tmp, n);
    for (auto &x : tmp) x *= 0.5;
    Pm.swap(tmp);
    cmatmul(eY, eY, tmp, n);
    eY.swap(tmp);
  }
  Kout.assign((size_t)2 * n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const cd k = cd(0, -tau) * E[i] * Pm[(size_t)i * n + j];
      Kout[2 * ((size_t)i * n + j)] = k.real();
      Kout[2 * ((size_t)i * n + j) + 1] = k.imag();
    }
}

// ---------------------------------------------------------------- Chebyshev
static double fermi(double E, double mu, double beta) {
  const double z = beta * (E - mu);
  if (z > 0) {
    const double e = std::exp(-z);
    return e / (1 + e);
  }
  return 1 / (1 + std::exp(z));
}

// a_n = (2 - delta_n0)/M sum_j F(c + R cos t_j) cos(n t_j), t_j = pi (j+1/2)/M,
// M = 4 n; cos(n t_j) by rotation, re-seeded every 64 orders from an exactly
// reduced argument.
// a_n = (2 - delta_n0)/M sum_j f(c + R cos t_j) cos(n t_j), t_j = pi (j + 1/2)/M,
// M = 4 ncoef; cos(n t_j) by rotation, re-seeded every 64 orders
template <typename F>
static void step_coefficients(F f, double emin, double emax, int ncoef, double *a) {
  const double c = 0.5 * (emax + emin), R = 0.5 * (emax - emin);
  const int64_t M = 4 * (int64_t)ncoef;
  std::vector<double> acc(ncoef, 0.0);
  for (int64_t j = 0; j < M; ++j) {
    const double th = M_PI * (j + 0.5) / (double)M;
    const double fv = f(c + R * std::cos(th));
    if (fv == 0.0) continue;
    const double wr = std::cos(th), wi = std::sin(th);
    double cr = 1, ci = 0;
    for (int k = 0; k < ncoef; ++k) {
      if ((k & 63) == 0) {
        // cos/sin(k t_j) = cos/sin(pi k (2j+1) / (2M)), argument reduced mod 4M
        const int64_t m = ((int64_t)k * (2 * j + 1)) % (4 * M);
        const double ang = M_PI * (double)m / (2.0 * (double)M);
        cr = std::cos(ang);
        ci = std::sin(ang);
      }
      acc[k] += fv * cr;
      const double nr = cr * wr - ci * wi;
      ci = cr * wi + ci * wr;
      cr = nr;
    }
  }
  for (int k = 0; k < ncoef; ++k) a[k] = acc[k] * 2.0 / (double)M;
  a[0] *= 0.5;
}

void fermi_coefficients(double mu, double beta, double emin, double emax, int ncoef,
                        double *a) {
  step_coefficients([&](double E) { return fermi(E, mu, beta); }, emin, emax, ncoef, a);
}

// y with erfc(y) = t, 0 < t < 1, by bisection (erfc decreases; 200 halvings
// of [0, 27] reach the last bit)
static double erfc_inverse(double t) {
  double lo = 0.0, hi = 27.0;
  for (int i = 0; i < 200; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (std::erfc(mid) > t) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Gapped filter: erfc((E - mu)/sigma)/2 with mu mid-gap and sigma such that
// the step is 1 - eps at E_HOMO and eps at E_LUMO (the cutoff spread over
// the band gap, Sec. 2.1)
void gapped_coefficients(double e_homo, double e_lumo, double eps, double emin, double emax,
                         int ncoef, double *a) {
  const double mu = 0.5 * (e_homo + e_lumo);
  const double sigma = (e_lumo - e_homo) / (2.0 * erfc_inverse(2.0 * eps));
  step_coefficients([&](double E) { return 0.5 * std::erfc((E - mu) / sigma); }, emin, emax,
                    ncoef, a);
}

// J_0..J_nmax(x), x >= 0, by Miller's backward recurrence
// J_{k-1} = (2k/x) J_k - J_{k+1}, normalised with J_0 + 2 sum_k J_2k = 1.
void bessel_j(double x, int nmax, std::vector<double> &J) {
  J.assign(nmax + 1, 0.0);
  if (x == 0.0) { J[0] = 1.0; return; }
  const int base = std::max(nmax, (int)x);
  int m = base + 20 + (int)std::sqrt(40.0 * (base + 1));
  if (m % 2) ++m;
  std::vector<double> j(m + 2, 0.0);
  j[m + 1] = 0.0;
  j[m] = 1e-30;
  for (int k = m; k >= 1; --k) {
    j[k - 1] = (2.0 * k / x) * j[k] - j[k + 1];
    if (std::fabs(j[k - 1]) > 1e250)
      for (int q = k - 1; q <= m + 1; ++q) j[q] *= 1e-250;
  }
  double norm = j[0];
  for (int k = 2; k <= m; k += 2) norm += 2.0 * j[k];
  for (int k = 0; k <= nmax; ++k) J[k] = j[k] / norm;
}

// b_n = e^{-i c tau} (2 - delta_n0) (-i)^n J_n(R tau), n < nterms, nterms the
// first n > R|tau| (n >= 1) with |J_n(R|tau|)| < tol.
int propagator_coefficients(double emin, double emax, double tau, double tol,
                            std::vector<double> &out) {
  const double c = 0.5 * (emax + emin), R = 0.5 * (emax - emin);
  const double x = std::fabs(R * tau);
  int nmax = (int)x + 64;
  std::vector<double> J;
  int nt = -1;
  for (int attempt = 0; attempt < 8 && nt < 0; ++attempt) {
    bessel_j(x, nmax, J);
    for (int n = std::max(1, (int)std::floor(x) + 1); n <= nmax; ++n)
      if (std::fabs(J[n]) < tol) { nt = n; break; }
    nmax *= 2;
  }
  SGW_REQUIRE(nt > 0, SGW_EINVAL, "propagator: no truncation order found");
  out.assign(2 * nt, 0.0);
  const cd ph = std::exp(cd(0, -c * tau));
  for (int n = 0; n < nt; ++n) {
    double jn = J[n];
    if (tau < 0 && (n & 1)) jn = -jn;            // J_n(-x) = (-1)^n J_n(x)
    const cd mi[4] = {cd(1, 0), cd(0, -1), cd(-1, 0), cd(0, 1)};
    const cd b = ph * (n == 0 ? 1.0 : 2.0) * mi[n & 3] * jn;
    out[2 * n] = b.real();
    out[2 * n + 1] = b.imag();
  }
  return nt;
}

// ---------------------------------------------------------------- QP
namespace {
struct SigW {
  const double *sig;
  int n_tau;
  double dt, gamma;
  // Re Sigma(w) and d Re Sigma/dw (trapezoid, Gaussian damping)
  void eval(double w, double *re, double *dre) const {
    double s = 0, d = 0;
    for (int j = -n_tau; j <= n_tau; ++j) {
      const double t = dt * j;
      const double wt = dt * ((j == -n_tau || j == n_tau) ? 0.5 : 1.0) *
                        std::exp(-0.5 * gamma * gamma * t * t);
      const double sr = sig[2 * (j + n_tau)], si = sig[2 * (j + n_tau) + 1];
      const double cs = std::cos(w * t), sn = std::sin(w * t);
      s += wt * (cs * sr - sn * si);
      d += wt * (-t * sn * sr - t * cs * si);
    }
    *re = s;
    if (dre) *dre = d;
  }
};
}  // namespace

int qp_solve(const double *sig, int n_tau, double dt, double gamma, double eks, double x,
             double vxc, double *eg, double *el, double *z) {
  SigW S{sig, n_tau, dt, gamma};
  double s0, d0;
  S.eval(eks, &s0, &d0);
  const double Z = 1.0 / (1.0 - d0);
  const double lin = eks + Z * (x + s0 - vxc);
  auto f = [&](double w) {
    double s;
    S.eval(w, &s, nullptr);
    return eks + x + s - vxc - w;
  };
  *el = lin;
  *z = Z;
  const double step = 1e-3, tol = 1e-10, search = 2.0;
  if (f(lin) == 0.0) { *eg = lin; return 0; }
  const int nsteps = (int)std::ceil(search / step);
  for (int k = 0; k < nsteps; ++k) {
    const double cand[2][2] = {{lin + k * step, lin + (k + 1) * step},
                               {lin - (k + 1) * step, lin - k * step}};
    for (int c = 0; c < 2; ++c) {
      double a = cand[c][0], b = cand[c][1];
      double fa = f(a);
      const double fb = f(b);
      if (fa == 0.0) { *eg = a; return 0; }
      if (fa * fb < 0.0) {
        while (b - a > tol) {
          const double m = 0.5 * (a + b);
          const double fm = f(m);
          if (fa * fm <= 0.0) b = m;
          else { a = m; fa = fm; }
        }
        *eg = 0.5 * (a + b);
        return 0;
      }
    }
  }
  return -1;
}


// ---------------------------------------------------------------- tuner cache
// The file holds one flat JSON object {"key": choice, ...} with keys made of
// [A-Za-z0-9_/x.:+-] only, written whole after every new entry.
namespace {
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

const char *tune_path() {
  const char *p = std::getenv("SGW_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = tune_path();
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  while (true) {
    const size_t q0 = t.find('"', i);
    if (q0 == std::string::npos) break;
    const size_t q1 = t.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const size_t colon = t.find(':', q1);
    if (colon == std::string::npos) break;
    char *end = nullptr;
    const long v = std::strtol(t.c_str() + colon + 1, &end, 10);
    if (end == t.c_str() + colon + 1) break;
    g_tune[t.substr(q0 + 1, q1 - q0 - 1)] = (int)v;
    i = (size_t)(end - t.c_str());
  }
}
}  // namespace

bool tune_cache_lookup(const std::string &key, int &choice) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  const auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  choice = it->second;
  return true;
}

void tune_cache_store(const std::string &key, int choice) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[key] = choice;
  const char *path = tune_path();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return;                      // the cache is an optimisation: never an error
    f << "{\n";
    size_t n = 0;
    for (const auto &kv : g_tune)
      f << "  \"" << kv.first << "\": " << kv.second << (++n < g_tune.size() ? ",\n" : "\n");
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}


// ---------------------------------------------------------------- small eigenproblems
// Eigenvalues (ascending) and eigenvectors of a symmetric n x n matrix by
// cyclic Jacobi rotations (Rutishauser's form); a: row-major, destroyed;
// vecs: row-major, column i is the eigenvector of vals[i].
void jacobi_eigen(int n, std::vector<double> &a, std::vector<double> &vals,
                  std::vector<double> &vecs) {
  vecs.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) vecs[(size_t)i * n + i] = 1.0;
  double scale = 0;
  for (double x : a) scale = std::max(scale, std::fabs(x));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[(size_t)p * n + q] * a[(size_t)p * n + q];
    if (off <= 1e-60 * scale * scale + 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < n; ++r) {          // columns p, q
          const double arp = a[(size_t)r * n + p], arq = a[(size_t)r * n + q];
          a[(size_t)r * n + p] = c * arp - sn * arq;
          a[(size_t)r * n + q] = sn * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {          // rows p, q
          const double apr = a[(size_t)p * n + r], aqr = a[(size_t)q * n + r];
          a[(size_t)p * n + r] = c * apr - sn * aqr;
          a[(size_t)q * n + r] = sn * apr + c * aqr;
        }
        for (int r = 0; r < n; ++r) {
          const double vrp = vecs[(size_t)r * n + p], vrq = vecs[(size_t)r * n + q];
          vecs[(size_t)r * n + p] = c * vrp - sn * vrq;
          vecs[(size_t)r * n + q] = sn * vrp + c * vrq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(),
            [&](int x, int y) { return a[(size_t)x * n + x] < a[(size_t)y * n + y]; });
  std::vector<double> v2((size_t)n * n);
  vals.resize(n);
  for (int i = 0; i < n; ++i) {
    vals[i] = a[(size_t)idx[i] * n + idx[i]];
    for (int r = 0; r < n; ++r) v2[(size_t)r * n + i] = vecs[(size_t)r * n + idx[i]];
  }
  vecs.swap(v2);
}

}  // namespace sgw
