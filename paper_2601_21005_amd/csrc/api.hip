// C ABI of libsgw (include/sgw.h): context set-up, H|psi>, the Chebyshev
// filter and propagator, the TDH response and the full Sigma_c(t) estimate.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <mutex>
#include <numeric>
#include <thread>

#include "common.h"
#include "kernels.h"
#include "rng.h"

using namespace sgw;

// Scratch of sgw_apply_H_noalloc (see below): 64 MiB per GPU, reserved when
// the library is loaded.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

thread_local std::string g_create_error;
// set on the worker threads of sgw_batch_sigma_estimate: they replay graphs
// that a context already holds but capture none (a capture on one thread
// does not mix with allocations and copies that other workers issue)
thread_local bool g_no_capture = false;

template <typename F> sgw_status guarded(sgw_ctx *ctx, F &&f) {
  try {
    f();
    return SGW_OK;
  } catch (const Error &e) {
    if (ctx) ctx->err = e.msg;
    else g_create_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    if (ctx) ctx->err = "host allocation failed";
    else g_create_error = "host allocation failed";
    return SGW_ENOMEM;
  } catch (const std::exception &e) {
    if (ctx) ctx->err = e.what();
    else g_create_error = e.what();
    return SGW_EINVAL;
  }
}

// upload host doubles as the working real type
void upload_real(sgw_ctx *ctx, DevBuf &b, const double *src, size_t n) {
  b.ensure(n * ctx->rsize());
  if (ctx->dbl) {
    SGW_HIP(hipMemcpyAsync(b.p, src, n * 8, hipMemcpyHostToDevice, ctx->stream));
  } else {
    std::vector<float> f(src, src + n);
    SGW_HIP(hipMemcpyAsync(b.p, f.data(), n * 4, hipMemcpyHostToDevice, ctx->stream));
    SGW_HIP(hipStreamSynchronize(ctx->stream));   // f goes out of scope
    return;
  }
  SGW_HIP(hipStreamSynchronize(ctx->stream));
}

void upload_cplx(sgw_ctx *ctx, DevBuf &b, const double *re_im, size_t n) {
  upload_real(ctx, b, re_im, 2 * n);
}

template <typename T> void upload(DevBuf &b, const T *src, size_t n) {
  b.ensure(n * sizeof(T));
  SGW_HIP(hipMemcpy(b.p, src, n * sizeof(T), hipMemcpyHostToDevice));
}

std::vector<double> fftfreq_k2(int n, double h) {
  std::vector<double> k2(n);
  const double L = n * h;
  for (int i = 0; i < n; ++i) {
    const int m = (i <= (n - 1) / 2) ? i : i - n;
    const double k = 2.0 * M_PI * m / L;
    k2[i] = k * k;
  }
  return k2;
}

void check_ptr(const void *p, const char *what) {
  SGW_REQUIRE(p != nullptr, SGW_EINVAL, std::string(what) + " is NULL");
  SGW_REQUIRE(((uintptr_t)p & 15) == 0, SGW_EINVAL, std::string(what) + " is not 16-byte aligned");
}

// Issue work on another stream of the context, with its own scratch buffers.
struct OnStream {
  sgw_ctx *c;
  hipStream_t s0;
  std::string n0;
  OnStream(sgw_ctx *ctx, hipStream_t s, const char *ns) : c(ctx), s0(ctx->stream), n0(ctx->ns) {
    c->stream = s;
    c->ns = ns;
  }
  ~OnStream() {
    c->stream = s0;
    c->ns = n0;
  }
};

// ---------------------------------------------------------------- graphs
// Capture the launches of `body` on the context's stream into a graph kept
// under `key` (nothing runs during the capture); a later call with the same
// key gets the cached executable.  The body must not allocate, synchronise
// or autotune: callers run the same sequence eagerly first.
template <typename F> hipGraphExec_t captured(sgw_ctx *ctx, const std::string &key, F &&body) {
  auto it = ctx->gexec.find(key);
  if (it != ctx->gexec.end()) return it->second;
  if (g_no_capture) return nullptr;                // caller runs eagerly
  SGW_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  try {
    body();
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(ctx->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hipGraph_t g = nullptr;
  SGW_HIP(hipStreamEndCapture(ctx->stream, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  SGW_HIP(e);
  ctx->gexec[key] = ex;
  return ex;
}

std::string ptr_key(std::initializer_list<const void *> ps) {
  std::string k;
  char b[24];
  for (const void *p : ps) {
    std::snprintf(b, sizeof b, "%p|", p);
    k += b;
  }
  return k;
}

std::string num_key(std::initializer_list<double> xs) {
  std::string k;
  char b[32];
  for (double x : xs) {
    std::snprintf(b, sizeof b, "%a|", x);
    k += b;
  }
  return k;
}

// ------------------------------------------------------ projections beside
// C = E B^T x (kb_gather_e) on the context's second stream, ordered after the
// work issued so far on the context's stream; join_gather makes the context's
// stream wait for it.  The gather is latency-bound and the FFT passes that
// run meanwhile on the context's stream bandwidth-bound, so the two share the
// device well; kbC must not be read on the context's stream in between.
void fork_gather(sgw_ctx *ctx, const void *x, int64_t nvec, int64_t ld, void *kbC) {
  SGW_HIP(hipEventRecord(ctx->kb_fork[0], ctx->stream));
  SGW_HIP(hipStreamWaitEvent(ctx->aux, ctx->kb_fork[0], 0));
  {
    OnStream on(ctx, ctx->aux, "|k");
    kb_gather_e(ctx, x, nvec, ld, kbC);
  }
  SGW_HIP(hipEventRecord(ctx->kb_fork[1], ctx->aux));
}

void join_gather(sgw_ctx *ctx) {
  SGW_HIP(hipStreamWaitEvent(ctx->stream, ctx->kb_fork[1], 0));
}

// whether the projector gathers of a batch of nvec vectors go beside the FFT
// passes (on the context's stream, with projectors, for batches that fill
// more than a sliver of the device); creates the second stream on first use
bool gather_beside(sgw_ctx *ctx, int64_t nvec) {
  const bool ovl = ctx->has_kb && ctx->kb_overlap && ctx->ns.empty() && nvec >= 16;
  if (ovl) ctx->make_aux();
  return ovl;
}

// ---------------------------------------------------------------- Chebyshev
// Term k of the fused recurrence on (cur = v_k, old = v_{k-1}):
// old <- v_{k+1} (out <- v_{k+1} when out is given); acc_mode 1 / 2: acc = /
// += b_{k-1} v_{k-1} + b_k v_k.  With coef_dev the coefficients are read on
// the device at coef_dev[d_counter[0]] and the entry before.  With tmp2 the z
// pencils write it rather than tmp (out of place: the Chebyshev batches stream
// faster so; the TDH's larger batches do not, and keep them in place).  rev
// (odd terms) starts the FFT passes from the last vector: each pass then
// begins on the vectors the pass before it wrote last, which are still in the
// last-level cache.
void cheb_term(sgw_ctx *ctx, void *cur, void *old, void *acc, void *tmp, void *kbC,
               int64_t nvec, bool first, int acc_mode, const double *bprev, const double *b,
               double c, double invR, const double *coef_dev, void *out = nullptr,
               void *tmp2 = nullptr, bool rev = false, bool ovl = false) {
  const int64_t N = ctx->N;
  const double s2 = first ? 1.0 : 2.0;
  // with ovl the projections of v_n go on the second stream, beside the FFT
  // passes (both only read v_n), and the scatter waits for them
  if (ctx->has_kb && ovl) fork_gather(ctx, cur, nvec, N, kbC);
  else if (ctx->has_kb) kb_gather_e(ctx, cur, nvec, N, kbC);
  EpiArgs e;
  e.x = cur;
  e.vold = old;
  e.vout = out;
  e.acc = acc;
  e.vloc = ctx->d_vloc.p;
  e.c = c;
  e.invR = invR;
  e.acc_mode = acc_mode;
  if (bprev) { e.cprev_re = bprev[0]; e.cprev_im = bprev[1]; }
  if (b) { e.coef_re = b[0]; e.coef_im = b[1]; }
  e.first = first ? 1 : 0;
  e.scale2 = s2;
  e.coef_dev = coef_dev;
  e.term_dev = coef_dev ? ctx->d_counter.as<int>() : nullptr;
  fft3d_apply(ctx, cur, tmp, nullptr, nvec, N, MUL_KIN, 0.0, PLANE_INV_CHEB, e, 0, tmp2, rev);
  if (ctx->has_kb && ovl) join_gather(ctx);
  if (ctx->has_kb) kb_scatter(ctx, kbC, nvec, out ? out : old, N, s2 * invR, 0.0, nullptr, 0.0, 0.0);
}

constexpr int SHORT_SERIES = 64;   // up to this many terms a series is one graph

// out = sum_n coef_n T_n(H~) v0 over nvec vectors (ld = N) with the fused
// recurrence; v0 and w1 are overwritten.  coef interleaved (re, im).
// Returns the vector holding v_last (for the norm check).  Term k works on
// cur = v0 (k even) or w1 (k odd); the accumulator takes the terms in pairs
// on odd k (b_{k-1} v_{k-1} + b_k v_k, both complete there), and the last
// one or two terms at the end.  With graphs on, a short series is replayed
// whole (one graph per set of buffers and coefficients), a long one as a
// graph of two terms that reads its coefficients from the device.
void *cheb_series(sgw_ctx *ctx, void *v0, void *w1, void *acc, void *tmp, int64_t nvec,
                  const std::vector<double> &coef, double emin, double emax) {
  const int nc = (int)coef.size() / 2;
  const int64_t N = ctx->N;
  const double c = 0.5 * (emax + emin), R = 0.5 * (emax - emin), invR = 1.0 / R;
  if (nc == 1) {
    launch_scale_copy(ctx, v0, N, acc, N, nvec, coef[0], coef[1]);
    return v0;
  }
  void *kbC = nullptr;
  if (ctx->has_kb) kbC = ctx->buf("kbC", ctx->csize() * ctx->kb.nproj * nvec).p;
  void *tmp2 = ctx->buf("cheb_tmp2", ctx->csize() * N * nvec).p;
  const bool ovl = gather_beside(ctx, nvec);
  auto cur_of = [&](int k) { return (k % 2 == 0) ? v0 : w1; };
  auto old_of = [&](int k) { return (k % 2 == 0) ? w1 : v0; };
  auto mode_of = [&](int k) { return k % 2 == 0 ? 0 : (k == 1 ? 1 : 2); };
  auto eager = [&](int k0, int k1) {       // terms k0 .. k1 - 1, host coefficients
    for (int k = k0; k < k1; ++k)
      cheb_term(ctx, cur_of(k), old_of(k), acc, tmp, kbC, nvec, k == 0, mode_of(k),
                k > 0 ? &coef[2 * (k - 1)] : nullptr, &coef[2 * k], c, invR, nullptr, nullptr,
                tmp2, k % 2 == 1, ovl);
  };
  auto last = [&]() {
    const int k = nc - 1;                  // the loop ran terms 0 .. nc - 2
    if ((nc - 2) % 2 == 1)                 // its last term was odd: acc holds 0 .. nc - 2
      launch_axpy(ctx, cur_of(k), N, acc, N, nvec, coef[2 * k], coef[2 * k + 1]);
    else                                   // b_{nc-2} v_{nc-2} is still pending
      launch_axpy2(ctx, old_of(k), cur_of(k), N, acc, nvec, coef[2 * k - 2], coef[2 * k - 1],
                   coef[2 * k], coef[2 * k + 1], nc == 2);
    return cur_of(k);
  };
  const bool graph = ctx->graphs && !ctx->ktimer;
  if (!graph) {
    eager(0, nc - 1);
    return last();
  }
  const std::string base = ptr_key({v0, w1, acc, tmp, tmp2, kbC}) + num_key({(double)nvec, c, invR});
  if (nc <= SHORT_SERIES) {
    std::string key = "series|" + base;
    for (double x : coef) key += num_key({x});
    auto it = ctx->gexec.find(key);
    if (it == ctx->gexec.end()) {
      eager(0, nc - 1);                   // this call runs eagerly, later ones replay
      last();
      if (!g_no_capture) captured(ctx, key, [&] { eager(0, nc - 1); last(); });
    } else {
      SGW_HIP(hipGraphLaunch(it->second, ctx->stream));
    }
    return cur_of(nc - 1);
  }
  // long series: terms 0, 1 eagerly, then pairs (even, odd) from the graph
  DevBuf &dc = ctx->buf("cheb_coef_dev", sizeof(double) * coef.size());
  SGW_HIP(hipMemcpyAsync(dc.p, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice,
                         ctx->stream));
  eager(0, 2);
  const int npair = (nc - 3) / 2;
  if (npair > 0) {
    const std::string key = "pair|" + base + ptr_key({dc.p, ctx->d_counter.p});
    hipGraphExec_t ex = captured(ctx, key, [&] {
      for (int k = 2; k < 4; ++k) {
        cheb_term(ctx, cur_of(k), old_of(k), acc, tmp, kbC, nvec, false, mode_of(k), nullptr,
                  nullptr, c, invR, dc.as<double>(), nullptr, tmp2, k % 2 == 1, ovl);
        launch_counter(ctx, 0, 1, true);
      }
    });
    if (ex) {
      launch_counter(ctx, 0, 2, false);
      for (int p = 0; p < npair; ++p) SGW_HIP(hipGraphLaunch(ex, ctx->stream));
    } else {
      eager(2, 2 + 2 * npair);
    }
  }
  eager(2 + 2 * npair, nc - 1);
  return last();
}

// G sums of one recurrence on v0: acc_g = sum_n coef_g,n T_n(H~) v0 for
// g < G (accumulators G-major, acc + g nvec N; ld = N), each series padded
// with zeros to the longest.  The zeta propagation takes the states of G
// consecutive output steps from one sweep (the Jacobi-Anger coefficients of
// the times dt, 2 dt, ..., G dt, Eq. 4), instead of G series of one step
// each.  Term k >= 1 is written to slot (k - 1) mod kSweepGroup of a ring
// (term 0 is v0 itself), and the G sums take the terms in groups of
// kSweepGroup: each group's terms are read once for all G accumulators, as
// soon as the group is complete and before term k + 1 takes the slot of
// term k + 1 - kSweepGroup (at most kSweepGroup - 1 terms are pending then).
// v0 is left as it was.  With graphs on, the sweep is replayed whole (one
// graph per buffers and coefficients).
void cheb_sweep(sgw_ctx *ctx, void *v0, void *acc, void *tmp, int64_t nvec,
                const std::vector<std::vector<double>> &coefs, double emin, double emax) {
  const int G = (int)coefs.size();
  SGW_REQUIRE(G >= 1 && G <= kMaxSweep, SGW_EINVAL, "sweep: bad number of outputs");
  int nc = 0;
  for (const auto &cg : coefs) nc = std::max(nc, (int)cg.size() / 2);
  const double c = 0.5 * (emax + emin), R = 0.5 * (emax - emin), invR = 1.0 / R;
  void *kbC = nullptr;
  if (ctx->has_kb) kbC = ctx->buf("kbC", ctx->csize() * ctx->kb.nproj * nvec).p;
  const size_t slot = ctx->csize() * (size_t)ctx->N * nvec;
  char *ring = static_cast<char *>(ctx->buf("sweep_ring", slot * kSweepGroup).p);
  void *tmp2 = ctx->buf("sweep_tmp2", slot).p;
  auto term = [&](int k) -> void * {
    return k == 0 ? v0 : static_cast<void *>(ring + slot * ((k - 1) % kSweepGroup));
  };
  auto b_of = [&](int g, int n, int part) {
    return 2 * n + 1 < (int)coefs[g].size() ? coefs[g][2 * n + part] : 0.0;
  };
  // acc_g (= for the first group, else +=) sum_{k0 <= k < k1} b_g,k v_k
  auto group = [&](int k0, int k1) {
    ChebAccTerms t{};
    for (int j = 0; j < k1 - k0; ++j) {
      t.x[j] = term(k0 + j);
      for (int g = 0; g < G; ++g) {
        t.c[g][2 * j] = b_of(g, k0 + j, 0);
        t.c[g][2 * j + 1] = b_of(g, k0 + j, 1);
      }
    }
    launch_cheb_accs(ctx, t, k1 - k0, acc, nvec, G, k0 == 0);
  };
  auto run = [&]() {
    int f = 0;                          // first term not yet in the sums
    for (int k = 0; k + 1 < nc; ++k) {
      cheb_term(ctx, term(k), k == 0 ? v0 : term(k - 1), nullptr, tmp, kbC, nvec, k == 0, 0,
                nullptr, nullptr, c, invR, nullptr, term(k + 1), tmp2, k % 2 == 1);
      if (k + 2 - f == kSweepGroup) {
        group(f, k + 2);
        f = k + 2;
      }
    }
    if (f < nc || nc == 0) group(f, nc);
  };
  if (!(ctx->graphs && !ctx->ktimer) || nc > 2 * SHORT_SERIES) {
    run();
    return;
  }
  std::string key = "sweep|" + ptr_key({v0, acc, tmp, tmp2, kbC, ring}) +
                    num_key({(double)nvec, c, invR, (double)G});
  for (const auto &cg : coefs) {
    key += "/";
    for (double x : cg) key += num_key({x});
  }
  auto it = ctx->gexec.find(key);
  if (it == ctx->gexec.end()) {
    run();                              // this call runs eagerly, later ones replay
    if (!g_no_capture) captured(ctx, key, run);
  } else {
    SGW_HIP(hipGraphLaunch(it->second, ctx->stream));
  }
}

// ||v_last|| <= ||v_0|| when spec(H~) lies in [-1, 1]; growth means the
// interval did not enclose the spectrum.
void check_growth(sgw_ctx *ctx, const std::vector<double> &n0, const void *vlast, int64_t nvec) {
  DevBuf &d = ctx->buf("norm_out", sizeof(double) * nvec);
  launch_norm2(ctx, vlast, ctx->N, nvec, d.as<double>());
  std::vector<double> n1(nvec);
  SGW_HIP(hipMemcpyAsync(n1.data(), d.p, sizeof(double) * nvec, hipMemcpyDeviceToHost,
                         ctx->stream));
  SGW_HIP(hipStreamSynchronize(ctx->stream));
  for (int64_t v = 0; v < nvec; ++v)
    if (!std::isfinite(n1[v]) || n1[v] > 1.02 * n0[v] + 1e-300)
      throw Error{SGW_EDIVERGED, "Chebyshev recurrence grew: [emin, emax] does not enclose spec(H)"};
}

std::vector<double> norms_of(sgw_ctx *ctx, const void *x, int64_t nvec) {
  DevBuf &d = ctx->buf("norm_in", sizeof(double) * nvec);
  launch_norm2(ctx, x, ctx->N, nvec, d.as<double>());
  std::vector<double> n(nvec);
  SGW_HIP(hipMemcpyAsync(n.data(), d.p, sizeof(double) * nvec, hipMemcpyDeviceToHost,
                         ctx->stream));
  SGW_HIP(hipStreamSynchronize(ctx->stream));
  return n;
}

void check_interval(double emin, double emax) {
  SGW_REQUIRE(std::isfinite(emin) && std::isfinite(emax) && emax > emin, SGW_EINVAL,
              "spectral interval must satisfy emin < emax");
}

// ---------------------------------------------------------------- TDH
const void *kb_exp_matrix(sgw_ctx *ctx, double tau) {
  // cache the device matrix per tau
  char key[64];
  std::snprintf(key, sizeof key, "kbexp_%.17g", tau);
  auto it = ctx->scratch.find(key + ctx->ns);
  if (it != ctx->scratch.end()) return it->second->p;
  std::vector<double> K;
  kb_exponential_matrix(ctx, tau, K);
  DevBuf &b = ctx->buf(key, ctx->csize() * K.size() / 2);
  upload_cplx(ctx, b, K.data(), K.size() / 2);
  return b.p;
}

void kb_exp_apply(sgw_ctx *ctx, void *psi, int64_t ld, int64_t nvec, double tau) {
  const void *K = kb_exp_matrix(ctx, tau);
  void *C = ctx->buf("kbC", ctx->csize() * ctx->kb.nproj * nvec).p;
  void *C2 = ctx->buf("kbC2", ctx->csize() * ctx->kb.nproj * nvec).p;
  kb_gather(ctx, psi, nvec, ld, C);
  kb_mix_dense(ctx, K, C, C2, nvec);
  kb_scatter(ctx, C2, nvec, psi, ld, 1.0, 0.0, nullptr, 0.0, 0.0);
}

// Poisson of S complex fields rho (ld = N): POISSON -> v, u; SPLIT -> r0, r1
void poisson(sgw_ctx *ctx, const void *rho, int64_t S, PlaneMode mode, void *r0, void *r1,
             const void *vh0) {
  void *tmp = ctx->buf("poisson_tmp", ctx->csize() * ctx->N * S).p;
  EpiArgs e;
  e.vloc = ctx->d_vloc.p;
  e.r0 = r0;
  e.r1 = r1;
  e.vh0 = vh0;
  fft3d_apply(ctx, rho, tmp, nullptr, S, ctx->N, MUL_COUL, 0.0, mode, e);
}

// Potentials of the TDH densities: rho[0] = n + i dn_0 gives r0 (v, or vh0
// at the start) and u_0; rho[b] = dn_{2b-1} + i dn_{2b} gives u_{2b-1}, u_{2b}.
void tdh_potentials(sgw_ctx *ctx, const void *rho, int64_t S, int nk, PlaneMode m0, void *r0,
                    void *u, const void *vh0) {
  const size_t cs = ctx->csize(), rs = ctx->rsize();
  const int64_t N = ctx->N;
  poisson(ctx, rho, S, m0, r0, u, vh0);
  for (int b = 1; 2 * b - 1 < nk; ++b) {
    char *ub = static_cast<char *>(u);
    poisson(ctx, static_cast<const char *>(rho) + cs * N * S * b, S, PLANE_INV_SPLIT,
            ub + rs * N * S * (2 * b - 1), 2 * b < nk ? ub + rs * N * S * (2 * b) : nullptr,
            nullptr);
  }
}

// One or more Strang substeps for nk response states (psi vectors ldp
// apart);  the local half steps of consecutive substeps are merged (a = tau).
// `open`: the state is synchronised at entry (first half step a = tau/2);
// `close`: apply the closing half step.
void tdh_substeps(sgw_ctx *ctx, sgw_tdh_state *st, int64_t ldp, int nk, int nsub, double tau,
                  bool open, bool close) {
  const int64_t S = st->nsample, nv = (1 + nk) * (int64_t)st->nsample * st->neta;
  void *tmp = ctx->buf("tdh_tmp", ctx->csize() * ctx->N * nv).p;
  void *rho = ctx->buf("tdh_rho", ctx->csize() * ctx->N * S * (1 + nk / 2)).p;
  for (int k = 0; k < nsub; ++k) {
    launch_tdh_local(ctx, st->psi, ldp, st->v, st->u, st->nsample, st->neta, nk,
                     (k == 0 && open) ? 0.5 * tau : tau);
    if (ctx->has_kb) kb_exp_apply(ctx, st->psi, ldp, nv, 0.5 * tau);
    // the first pass from the last vector (where the local step ended), the
    // last one ending on the first (where the density starts)
    fft3d_apply(ctx, st->psi, tmp, st->psi, nv, ldp, MUL_PROP, tau, PLANE_INV_STORE,
                EpiArgs(), 0, nullptr, true);
    if (ctx->has_kb) kb_exp_apply(ctx, st->psi, ldp, nv, 0.5 * tau);
    launch_tdh_density(ctx, st->psi, ldp, rho, st->nsample, st->neta, nk, st->weight);
    tdh_potentials(ctx, rho, S, nk, PLANE_INV_POISSON, st->v, st->u, st->vh0);
  }
  if (close)
    launch_tdh_local(ctx, st->psi, ldp, st->v, st->u, st->nsample, st->neta, nk, 0.5 * tau);
}

void tdh_start(sgw_ctx *ctx, sgw_tdh_state *st, int64_t ldp, int nk, const void *dv) {
  const int64_t S = st->nsample;
  void *rho = ctx->buf("tdh_rho", ctx->csize() * ctx->N * S * (1 + nk / 2)).p;
  launch_tdh_tangent(ctx, st->psi, ldp, dv, st->nsample, st->neta, nk);
  launch_bcast_real(ctx, ctx->d_vloc.p, st->v, st->nsample);
  launch_tdh_density(ctx, st->psi, ldp, rho, st->nsample, st->neta, nk, st->weight);
  tdh_potentials(ctx, rho, S, nk, PLANE_INV_SPLIT, st->vh0, st->u, nullptr);
}

void check_state(sgw_ctx *ctx, const sgw_tdh_state *st) {
  SGW_REQUIRE(st != nullptr, SGW_EINVAL, "state is NULL");
  SGW_REQUIRE(st->nsample > 0 && st->neta > 0, SGW_EINVAL, "state: nsample, neta must be > 0");
  SGW_REQUIRE(std::isfinite(st->weight), SGW_EINVAL, "state: weight not finite");
  check_ptr(st->psi, "state.psi");
  check_ptr(st->v, "state.v");
  check_ptr(st->u, "state.u");
  check_ptr(st->vh0, "state.vh0");
  (void)ctx;
}

// Rigorous interval [min V + min(0, min E) s, T_max + max V + max(0, max E) s]
// (s: Gershgorin bound of the projector Gram matrix), widened by pad times
// its width on each side.
void weyl_bounds(sgw_ctx *ctx, double pad, double &emin, double &emax) {
  double lo = 0, hi = 0;
  if (ctx->has_kb) {
    const double s = kb_lambda_bound(ctx);
    const double emn = *std::min_element(ctx->kb.ekb.begin(), ctx->kb.ekb.end());
    const double emx = *std::max_element(ctx->kb.ekb.begin(), ctx->kb.ekb.end());
    lo = std::min(0.0, emn) * s;
    hi = std::max(0.0, emx) * s;
  }
  const double a = ctx->vmin + lo, b = ctx->tmax + ctx->vmax + hi;
  const double w = b - a;
  emin = a - pad * w;
  emax = b + pad * w;
}

// y = H x for nvec vectors (ld), in chunks of max_nvec
void apply_h(sgw_ctx *ctx, const void *psi, void *hpsi, int64_t nvec, int64_t ld) {
  const int64_t chunk = ctx->max_nvec;
  void *tmp = ctx->buf("tmp", ctx->csize() * ctx->N * chunk).p;
  for (int64_t v0 = 0; v0 < nvec; v0 += chunk) {
    const int64_t nv = std::min(chunk, nvec - v0);
    const char *x = static_cast<const char *>(psi) + v0 * ld * ctx->csize();
    char *y = static_cast<char *>(hpsi) + v0 * ld * ctx->csize();
    void *kbC = nullptr;
    if (ctx->has_kb) {
      kbC = ctx->buf("kbC", ctx->csize() * ctx->kb.nproj * nv).p;
      kb_gather_e(ctx, x, nv, ld, kbC);
    }
    EpiArgs e;
    e.x = x;
    e.vloc = ctx->d_vloc.p;
    fft3d_apply(ctx, x, tmp, y, nv, ld, MUL_KIN, 0.0, PLANE_INV_HPSI, e);
    if (ctx->has_kb) kb_scatter(ctx, kbC, nv, y, ld, 1.0, 0.0, nullptr, 0.0, 0.0);
  }
}

// ---------------------------------------------------------------- no-alloc H
// Scratch of sgw_apply_H_noalloc: one statically sized device array per GPU
// (module-scope, so loading the library reserves it; nothing is allocated
// per call).  Host code uses only the address that hipGetSymbolAddress gives
// for the current device, kept per device from the first sgw_create there.
constexpr int kNoAllocMaxDev = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocMaxDev] = {};

// with `dev` current: look up this device's copy of the array once
void noalloc_setup(int dev) {
  SGW_REQUIRE(dev >= 0 && dev < kNoAllocMaxDev, SGW_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[dev]) return;
  void *p = nullptr;
  SGW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  SGW_REQUIRE(p != nullptr, SGW_EHIP, "no device address for the no-alloc scratch");
  g_noalloc_ptr[dev] = p;
}

void *noalloc_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  return (dev >= 0 && dev < kNoAllocMaxDev) ? g_noalloc_ptr[dev] : nullptr;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// apply_h with the projector partials and coefficients in `scr` (kNoAllocBytes)
// and the FFT intermediate in hpsi itself; chunks of as many vectors as the
// scratch holds.  Kernel variants are not timed here (all give identical
// results): the remembered, cached or forced choice, else the first.
void apply_h_noalloc(sgw_ctx *ctx, const void *psi, void *hpsi, int64_t nvec, int64_t ld,
                     void *scr) {
  int64_t chunk = nvec;
  size_t part_per = 0, coef_per = 0;
  if (ctx->has_kb) {
    part_per = kb_partial_bytes_per_vec(ctx);
    coef_per = ctx->csize() * (size_t)ctx->kb.nproj;
    // both blocks 256-byte aligned: at most 512 bytes of padding per chunk
    chunk = std::min<int64_t>(nvec, (int64_t)((kNoAllocBytes - 512) / (part_per + coef_per)));
    SGW_REQUIRE(chunk >= 1, SGW_EUNSUPPORTED,
                "sgw_apply_H_noalloc: one vector's projector scratch exceeds the 64 MiB "
                "static buffer");
  }
  struct Restore {
    sgw_ctx *c;
    int kt;
    ~Restore() { c->no_tune = false; c->ktimer = kt; }
  } restore{ctx, ctx->ktimer};
  ctx->no_tune = true;
  ctx->ktimer = 0;                       // the launch timers create events
  for (int64_t v0 = 0; v0 < nvec; v0 += chunk) {
    const int64_t nv = std::min(chunk, nvec - v0);
    const char *x = static_cast<const char *>(psi) + v0 * ld * ctx->csize();
    char *y = static_cast<char *>(hpsi) + v0 * ld * ctx->csize();
    void *kbC = nullptr;
    if (ctx->has_kb) {
      void *partial = scr;
      kbC = static_cast<char *>(scr) + align256(part_per * nv);
      kb_gather_e(ctx, x, nv, ld, kbC, partial);
    }
    EpiArgs e;
    e.x = x;
    e.vloc = ctx->d_vloc.p;
    fft3d_apply(ctx, x, y, y, nv, ld, MUL_KIN, 0.0, PLANE_INV_HPSI, e, ld);
    if (ctx->has_kb) kb_scatter(ctx, kbC, nv, y, ld, 1.0, 0.0, nullptr, 0.0, 0.0);
  }
}

int next_pow2(int n) {
  int p = 1;
  while (p < n) p *= 2;
  return p;
}

}  // namespace

// =================================================================== ABI
extern "C" {

const char *sgw_last_error(const sgw_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

sgw_status sgw_create(const sgw_grid *grid, const double *v_loc, const sgw_projectors *proj,
                      sgw_precision prec, void *hip_stream, int64_t max_nvec, sgw_ctx **out) {
  if (out) *out = nullptr;
  sgw_ctx *ctx = nullptr;
  sgw_status st = guarded(nullptr, [&] {
    SGW_REQUIRE(out != nullptr, SGW_EINVAL, "out is NULL");
    SGW_REQUIRE(grid != nullptr && v_loc != nullptr, SGW_EINVAL, "grid or v_loc is NULL");
    SGW_REQUIRE(prec == SGW_C128 || prec == SGW_C64 || prec == SGW_C64_BF16KB ||
                    prec == SGW_C64_BF16X2KB,
                SGW_EINVAL, "unknown precision");
    SGW_REQUIRE(grid->nx > 0 && grid->ny > 0 && grid->nz > 0, SGW_EINVAL, "grid sizes must be > 0");
    SGW_REQUIRE(grid->h > 0 && std::isfinite(grid->h), SGW_EINVAL, "grid spacing must be > 0");
    SGW_REQUIRE(std::isfinite(grid->ecut), SGW_EINVAL, "ecut not finite");
    SGW_REQUIRE(max_nvec > 0, SGW_EINVAL, "max_nvec must be > 0");
    const bool dbl = prec == SGW_C128;
    SGW_REQUIRE(fft_size_supported(grid->nx, dbl) && fft_size_supported(grid->ny, dbl) &&
                    fft_size_supported(grid->nz, dbl),
                SGW_EUNSUPPORTED, "grid size not built into this library");
    SGW_REQUIRE(grid->nx == grid->ny, SGW_EUNSUPPORTED, "nx must equal ny");
    SGW_REQUIRE(fft_pencils_cover(grid->nx, grid->ny, grid->nz, dbl), SGW_EUNSUPPORTED,
                "nx must be a multiple of the z pencils' width (16 when nz % 16 == 0, "
                "else 8 when nz % 8 == 0, else 4)");
    std::unique_ptr<sgw_ctx> c(new sgw_ctx());
    c->nx = grid->nx; c->ny = grid->ny; c->nz = grid->nz;
    c->N = (int64_t)c->nx * c->ny * c->nz;
    c->h = grid->h;
    c->dV = grid->h * grid->h * grid->h;
    c->ecut = grid->ecut > 0 ? grid->ecut : 0.0;
    c->prec = prec;
    c->dbl = dbl;
    {
      int dev = 0;
      hipDeviceProp_t prop;
      SGW_HIP(hipGetDevice(&dev));
      SGW_HIP(hipGetDeviceProperties(&prop, dev));
      c->arch = prop.gcnArchName;
      const size_t colon = c->arch.find(':');           // drop feature suffixes
      if (colon != std::string::npos) c->arch.resize(colon);
      c->dev = dev;
      noalloc_setup(dev);
    }
    if (const char *fc = std::getenv("SGW_FILTER_CHUNK")) c->filter_chunk = std::atoi(fc);
    if (const char *ov = std::getenv("SGW_ZETA_OVERLAP")) c->overlap = std::atoi(ov) != 0;
    if (const char *ov = std::getenv("SGW_KB_OVERLAP")) c->kb_overlap = std::atoi(ov) != 0;
    if (const char *zw = std::getenv("SGW_ZETA_SWEEP")) c->zeta_sweep = std::atoi(zw);
    if (const char *fv = std::getenv("SGW_FORCE_VARIANT")) {
      // "name=i,name=i": pin autotuned kernel variants (testing)
      std::string spec(fv);
      size_t pos = 0;
      while (pos < spec.size()) {
        const size_t comma = spec.find(',', pos);
        const std::string item = spec.substr(pos, comma == std::string::npos ? std::string::npos : comma - pos);
        const size_t eq = item.find('=');
        if (eq != std::string::npos) c->forced[item.substr(0, eq)] = std::atoi(item.c_str() + eq + 1);
        if (comma == std::string::npos) break;
        pos = comma + 1;
      }
    }
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->max_nvec = max_nvec;
    c->d_counter.ensure(64);
    SGW_HIP(hipMemset(c->d_counter.p, 0, 64));
    c->vloc.assign(v_loc, v_loc + c->N);
    for (double v : c->vloc) SGW_REQUIRE(std::isfinite(v), SGW_EINVAL, "v_loc has a non-finite value");
    c->vmin = *std::min_element(c->vloc.begin(), c->vloc.end());
    c->vmax = *std::max_element(c->vloc.begin(), c->vloc.end());
    // k tables and twiddles (FP64 on the host, stored in the working type)
    std::vector<double> k2, tw;
    double kmax2 = 0;
    const int ns[3] = {c->nx, c->ny, c->nz};
    for (int ax = 0; ax < 3; ++ax) {
      auto a = fftfreq_k2(ns[ax], c->h);
      kmax2 += *std::max_element(a.begin(), a.end());
      k2.insert(k2.end(), a.begin(), a.end());
      for (int j = 0; j < ns[ax]; ++j) {
        tw.push_back(std::cos(2.0 * M_PI * j / ns[ax]));
        tw.push_back(-std::sin(2.0 * M_PI * j / ns[ax]));
      }
    }
    c->tmax = 0.5 * kmax2;
    if (c->ecut > 0) c->tmax = std::min(c->tmax, c->ecut);
    upload_real(c.get(), c->d_k2, k2.data(), k2.size());
    upload_real(c.get(), c->d_tw, tw.data(), tw.size());
    upload_real(c.get(), c->d_vloc, c->vloc.data(), c->N);
    if (proj) {
      build_kb(c.get(), proj);
      c->has_kb = true;
      upload(c->d_kb_tile_base, c->kb.tile_base.data(), c->kb.tile_base.size());
      upload(c->d_kb_tile_off, c->kb.tile_off.data(), c->kb.tile_off.size());
      upload(c->d_kb_entry_proj, c->kb.entry_proj.data(), c->kb.entry_proj.size());
      upload(c->d_kb_proj_off, c->kb.proj_off.data(), c->kb.proj_off.size());
      upload(c->d_kb_proj_entries, c->kb.proj_entries.data(), c->kb.proj_entries.size());
      upload(c->d_kb_ekb, c->kb.ekb.data(), c->kb.ekb.size());
      if (const char *km = std::getenv("SGW_KB_MASK"); km && std::atoi(km) == 0)
        std::fill(c->kb.mask.begin(), c->kb.mask.end(), ~0u);   // every point live (timing)
      upload(c->d_kb_mask, c->kb.mask.data(), c->kb.mask.size());
      upload_real(c.get(), c->d_kb_beta, c->kb.beta.data(), c->kb.beta.size());
      if (!c->dbl) kb_upload_operands(c.get());
    }
    ctx = c.release();
  });
  if (st == SGW_OK) *out = ctx;
  return st;
}

void sgw_destroy(sgw_ctx *ctx) { delete ctx; }

sgw_status sgw_bounds(sgw_ctx *ctx, double pad, double *emin, double *emax) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(emin && emax, SGW_EINVAL, "emin/emax NULL");
    SGW_REQUIRE(pad >= 0 && std::isfinite(pad), SGW_EINVAL, "pad must be >= 0");
    weyl_bounds(ctx, pad, *emin, *emax);
  });
}

sgw_status sgw_apply_H(sgw_ctx *ctx, const void *psi, void *hpsi, int64_t nvec, int64_t ld) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(nvec >= 0 && ld >= ctx->N, SGW_EINVAL, "nvec < 0 or ld < N");
    if (nvec == 0) return;
    check_ptr(psi, "psi");
    check_ptr(hpsi, "hpsi");
    SGW_REQUIRE(psi != hpsi, SGW_EINVAL, "psi and hpsi must not overlap");
    apply_h(ctx, psi, hpsi, nvec, ld);
  });
}

sgw_status sgw_apply_H_noalloc(sgw_ctx *ctx, const void *psi, void *hpsi, int64_t nvec,
                               int64_t ld) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(nvec >= 0 && ld >= ctx->N, SGW_EINVAL, "nvec < 0 or ld < N");
    if (nvec == 0) return;
    check_ptr(psi, "psi");
    check_ptr(hpsi, "hpsi");
    const size_t bytes = ctx->csize() * (size_t)((nvec - 1) * ld + ctx->N);
    const char *a = static_cast<const char *>(psi), *b = static_cast<const char *>(hpsi);
    SGW_REQUIRE(a + bytes <= b || b + bytes <= a, SGW_EINVAL, "psi and hpsi must not overlap");
    int cur = -1;
    SGW_HIP(hipGetDevice(&cur));
    SGW_REQUIRE(cur == ctx->dev, SGW_EINVAL,
                "sgw_apply_H_noalloc: the context's device must be current");
    void *scr = noalloc_ptr(cur);
    SGW_REQUIRE(scr != nullptr, SGW_EHIP, "no-alloc scratch not set up on this device");
    apply_h_noalloc(ctx, psi, hpsi, nvec, ld, scr);
  });
}

sgw_status sgw_lanczos_bounds(sgw_ctx *ctx, int32_t k, uint64_t seed, double pad, double *emin,
                              double *emax) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(emin && emax, SGW_EINVAL, "emin/emax NULL");
    SGW_REQUIRE(k >= 2 && k <= 1000, SGW_EINVAL, "k must be in 2..1000");
    SGW_REQUIRE(pad >= 0 && std::isfinite(pad), SGW_EINVAL, "pad must be >= 0");
    const int64_t N = ctx->N;
    const size_t cs = ctx->csize();
    void *v = ctx->buf("lz_v", cs * N).p, *vp = ctx->buf("lz_vp", cs * N).p;
    void *w = ctx->buf("lz_w", cs * N).p;
    double *d = ctx->buf("lz_dot", sizeof(double)).as<double>();
    auto fetch = [&]() {
      double x = 0;
      SGW_HIP(hipMemcpyAsync(&x, d, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      SGW_HIP(hipStreamSynchronize(ctx->stream));
      return x;
    };
    // start: +-1 white noise of stream (BOUNDS, 0, 0), unit Euclidean norm
    const uint64_t key = rng_key(seed, rng_stream(RNG_BOUNDS, 0, 0));
    DevBuf &dk = ctx->buf("lz_key", sizeof(uint64_t));
    SGW_HIP(hipMemcpyAsync(dk.p, &key, sizeof key, hipMemcpyHostToDevice, ctx->stream));
    launch_fill_noise(ctx, dk.as<uint64_t>(), 1, v);
    launch_norm2(ctx, v, N, 1, d);
    launch_scale_copy(ctx, v, N, v, N, 1, 1.0 / std::sqrt(fetch()), 0.0);
    launch_scale_copy(ctx, v, N, vp, N, 1, 0.0, 0.0);
    std::vector<double> alpha, beta;
    double b = 0;
    for (int j = 0; j < k; ++j) {
      apply_h(ctx, v, w, 1, N);
      launch_redot(ctx, v, w, N, 1, d);
      const double a = fetch();
      launch_axpy(ctx, v, N, w, N, 1, -a, 0.0);
      launch_axpy(ctx, vp, N, w, N, 1, -b, 0.0);
      launch_norm2(ctx, w, N, 1, d);
      b = std::sqrt(fetch());
      SGW_REQUIRE(std::isfinite(a) && std::isfinite(b), SGW_EDIVERGED, "Lanczos produced a non-finite value");
      alpha.push_back(a);
      beta.push_back(b);
      if (b == 0) break;
      launch_copy(ctx, v, N, vp, N, 1);
      launch_scale_copy(ctx, w, N, v, N, 1, 1.0 / b, 0.0);
    }
    const int n = (int)alpha.size();
    std::vector<double> T((size_t)n * n, 0.0), vals, vecs;
    for (int i = 0; i < n; ++i) {
      T[(size_t)i * n + i] = alpha[i];
      if (i + 1 < n) T[(size_t)i * n + i + 1] = T[(size_t)(i + 1) * n + i] = beta[i];
    }
    jacobi_eigen(n, T, vals, vecs);
    const double r0 = beta[n - 1] * std::fabs(vecs[(size_t)(n - 1) * n + 0]);
    const double r1 = beta[n - 1] * std::fabs(vecs[(size_t)(n - 1) * n + n - 1]);
    const double width = vals[n - 1] - vals[0];
    double lo_w = 0, hi_w = 0;
    weyl_bounds(ctx, 0.0, lo_w, hi_w);
    *emin = std::max(lo_w, vals[0] - r0 - pad * width);
    *emax = std::min(hi_w, vals[n - 1] + r1 + pad * width);
  });
}

sgw_status sgw_gapped_coefficients(double e_homo, double e_lumo, double eps, double emin,
                                   double emax, int32_t ncoef, double *coef) {
  try {
    if (!coef || ncoef <= 0 || !std::isfinite(e_homo) || !std::isfinite(e_lumo) ||
        !(e_lumo > e_homo) || !(eps > 0 && eps < 0.5) || !(emax > emin) ||
        !std::isfinite(emin) || !std::isfinite(emax))
      return SGW_EINVAL;
    gapped_coefficients(e_homo, e_lumo, eps, emin, emax, ncoef, coef);
    return SGW_OK;
  } catch (...) {
    return SGW_ENOMEM;
  }
}

sgw_status sgw_fermi_coefficients(double mu, double beta, double emin, double emax,
                                  int32_t ncoef, double *coef) {
  try {
    if (!coef || ncoef <= 0 || !std::isfinite(mu) || !std::isfinite(beta) ||
        !(emax > emin) || !std::isfinite(emin) || !std::isfinite(emax))
      return SGW_EINVAL;
    fermi_coefficients(mu, beta, emin, emax, ncoef, coef);
    return SGW_OK;
  } catch (...) {
    return SGW_ENOMEM;
  }
}

sgw_status sgw_propagator_coefficients(double emin, double emax, double tau, double tol,
                                       int32_t max_terms, double *coef, int32_t *nterms) {
  try {
    if (!coef || !nterms || !(emax > emin) || !std::isfinite(tau) || !(tol > 0))
      return SGW_EINVAL;
    std::vector<double> b;
    const int nt = propagator_coefficients(emin, emax, tau, tol, b);
    *nterms = nt;
    if (nt > max_terms) return SGW_EINVAL;
    std::memcpy(coef, b.data(), sizeof(double) * b.size());
    return SGW_OK;
  } catch (const Error &e) {
    return e.code;
  } catch (...) {
    return SGW_ENOMEM;
  }
}

sgw_status sgw_fermi_filter(sgw_ctx *ctx, void *v, int64_t nvec, int64_t ld, const double *coef,
                            int32_t ncoef, double emin, double emax) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(nvec >= 0 && ld >= ctx->N, SGW_EINVAL, "nvec < 0 or ld < N");
    SGW_REQUIRE(coef != nullptr && ncoef > 0, SGW_EINVAL, "no coefficients");
    check_interval(emin, emax);
    if (nvec == 0) return;
    check_ptr(v, "v");
    std::vector<double> c(2 * ncoef, 0.0);
    for (int i = 0; i < ncoef; ++i) {
      SGW_REQUIRE(std::isfinite(coef[i]), SGW_EINVAL, "coefficient not finite");
      c[2 * i] = coef[i];
    }
    const int64_t chunk = ctx->max_nvec;
    const size_t bytes = ctx->csize() * ctx->N * chunk;
    void *A = ctx->buf("cheb_a", bytes).p, *B = ctx->buf("cheb_b", bytes).p;
    void *acc = ctx->buf("cheb_acc", bytes).p, *tmp = ctx->buf("tmp", bytes).p;
    for (int64_t v0 = 0; v0 < nvec; v0 += chunk) {
      const int64_t nv = std::min(chunk, nvec - v0);
      char *x = static_cast<char *>(v) + v0 * ld * ctx->csize();
      launch_copy(ctx, x, ld, A, ctx->N, nv);
      const auto n0 = norms_of(ctx, A, nv);
      void *last = cheb_series(ctx, A, B, acc, tmp, nv, c, emin, emax);
      check_growth(ctx, n0, last, nv);
      launch_copy(ctx, acc, ctx->N, x, ld, nv);
    }
  });
}

sgw_status sgw_cheb_propagate(sgw_ctx *ctx, void *psi, int64_t nvec, int64_t ld, double dt,
                              int32_t nsteps, double emin, double emax, double tol) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(nvec >= 0 && ld >= ctx->N && nsteps >= 0, SGW_EINVAL, "bad sizes");
    SGW_REQUIRE(std::isfinite(dt) && tol > 0, SGW_EINVAL, "bad dt or tol");
    check_interval(emin, emax);
    if (nvec == 0 || nsteps == 0) return;
    check_ptr(psi, "psi");
    std::vector<double> b;
    propagator_coefficients(emin, emax, dt, tol, b);
    const int64_t chunk = ctx->max_nvec;
    const size_t bytes = ctx->csize() * ctx->N * chunk;
    void *bufs[3] = {ctx->buf("cheb_a", bytes).p, ctx->buf("cheb_b", bytes).p,
                     ctx->buf("cheb_acc", bytes).p};
    void *tmp = ctx->buf("tmp", bytes).p;
    for (int64_t v0 = 0; v0 < nvec; v0 += chunk) {
      const int64_t nv = std::min(chunk, nvec - v0);
      char *x = static_cast<char *>(psi) + v0 * ld * ctx->csize();
      void *cur = bufs[0], *w = bufs[1], *acc = bufs[2];
      launch_copy(ctx, x, ld, cur, ctx->N, nv);
      const auto n0 = norms_of(ctx, cur, nv);
      for (int s = 0; s < nsteps; ++s) {
        cheb_series(ctx, cur, w, acc, tmp, nv, b, emin, emax);
        std::swap(cur, acc);
      }
      // unitary: the norm is conserved
      check_growth(ctx, n0, cur, nv);
      launch_copy(ctx, cur, ctx->N, x, ld, nv);
    }
  });
}

sgw_status sgw_tdh_init(sgw_ctx *ctx, sgw_tdh_state *st, const void *dv) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    check_state(ctx, st);
    check_ptr(dv, "dv");
    tdh_start(ctx, st, ctx->N, 1, dv);
  });
}

sgw_status sgw_tdh_step(sgw_ctx *ctx, sgw_tdh_state *st, int32_t nsub, double dt_sub) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    check_state(ctx, st);
    SGW_REQUIRE(nsub >= 0 && std::isfinite(dt_sub), SGW_EINVAL, "bad nsub or dt_sub");
    if (nsub == 0) return;
    tdh_substeps(ctx, st, ctx->N, 1, nsub, dt_sub, true, true);
  });
}

sgw_status sgw_qp_solve(const double *sigma_t, int32_t n_tau, double dt, double gamma,
                        double eps_ks, double x, double vxc, double *eqp_graphical,
                        double *eqp_linear, double *z) {
  if (!sigma_t || n_tau < 1 || !(dt > 0) || !(gamma >= 0) || !eqp_graphical || !eqp_linear || !z)
    return SGW_EINVAL;
  for (int i = 0; i < 2 * (2 * n_tau + 1); ++i)
    if (!std::isfinite(sigma_t[i])) return SGW_EINVAL;
  const int r = qp_solve(sigma_t, n_tau, dt, gamma, eps_ks, x, vxc, eqp_graphical, eqp_linear, z);
  return r == 0 ? SGW_OK : SGW_ENOROOT;
}

sgw_status sgw_sigma_omega(const double *sigma_t, int32_t n_tau, double dt, double gamma,
                           const double *omega, int32_t n_omega, double *out) {
  if (!sigma_t || !omega || !out || n_tau < 1 || n_omega < 0 || !(dt > 0) || !(gamma >= 0))
    return SGW_EINVAL;
  for (int k = 0; k < n_omega; ++k) {
    double re = 0, im = 0;
    for (int j = -n_tau; j <= n_tau; ++j) {
      const double t = dt * j;
      const double wt = dt * ((j == -n_tau || j == n_tau) ? 0.5 : 1.0) *
                        std::exp(-0.5 * gamma * gamma * t * t);
      const double sr = sigma_t[2 * (j + n_tau)], si = sigma_t[2 * (j + n_tau) + 1];
      const double cs = std::cos(omega[k] * t), sn = std::sin(omega[k] * t);
      re += wt * (cs * sr - sn * si);
      im += wt * (cs * si + sn * sr);
    }
    out[2 * k] = re;
    out[2 * k + 1] = im;
  }
  return SGW_OK;
}

sgw_status sgw_kernel_timer(sgw_ctx *ctx, int32_t which) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE((which & ~(SGW_TIMER_CHEB_PLANE | SGW_TIMER_KB_SCATTER | SGW_TIMER_KB_GATHER)) ==
                    0,
                SGW_EINVAL, "unknown timer bits");
    ctx->ktimer = which;
  });
}

sgw_status sgw_kb_stats(const sgw_ctx *ctx, int64_t *out) {
  if (!ctx || !out) return SGW_EINVAL;
  out[0] = ctx->kb_ntile;
  out[1] = (int64_t)ctx->kb_ntile * KB_TP;
  out[2] = ctx->kb_support_points;
  out[3] = ctx->kb_nentry;
  out[4] = ctx->kb_nnz;
  return SGW_OK;
}

sgw_status sgw_use_graphs(sgw_ctx *ctx, int32_t enable) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(!enable || ctx->stream != nullptr, SGW_EINVAL,
                "graphs need a context created on a non-default stream");
    SGW_HIP(hipStreamSynchronize(ctx->stream));
    ctx->graphs = enable != 0;
    if (!ctx->graphs) ctx->clear_graphs();
  });
}

sgw_status sgw_kernel_timer_read(sgw_ctx *ctx, int32_t which, double *total_ms,
                                 int64_t *launches, int64_t *points) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(total_ms && launches && points, SGW_EINVAL, "NULL output");
    SGW_REQUIRE(which == SGW_TIMER_CHEB_PLANE || which == SGW_TIMER_KB_SCATTER ||
                    which == SGW_TIMER_KB_GATHER,
                SGW_EINVAL, "which must name one timer");
    sgw_ctx::KTimer &t =
        ctx->kt[which == SGW_TIMER_CHEB_PLANE ? 0 : which == SGW_TIMER_KB_SCATTER ? 1 : 2];
    SGW_HIP(hipStreamSynchronize(ctx->stream));
    double ms = 0;
    for (int64_t i = 0; i < t.used; ++i) {
      float e = 0;
      SGW_HIP(hipEventElapsedTime(&e, t.events[2 * i], t.events[2 * i + 1]));
      ms += e;
    }
    *total_ms = ms;
    *launches = t.used;
    *points = t.points;
    t.used = 0;
    t.points = 0;
  });
}

// ------------------------------------------------------------------ Sigma
sgw_status sgw_sigma_estimate(sgw_ctx *ctx, const sgw_sigma_params *P, const double *phi,
                              double *sigma_t, double *x_out, double *phase_ms) {
  return sgw_sigma_estimate_states(ctx, P, 1, phi, sigma_t, x_out, phase_ms);
}

sgw_status sgw_sigma_estimate_states(sgw_ctx *ctx, const sgw_sigma_params *P, int32_t nstate,
                                     const double *phi, double *sigma_t, double *x_out,
                                     double *phase_ms) {
  if (!ctx) return SGW_EINVAL;
  return guarded(ctx, [&] {
    SGW_REQUIRE(P && phi && sigma_t && x_out, SGW_EINVAL, "NULL argument");
    SGW_REQUIRE(nstate >= 1 && nstate <= SGW_MAX_STATES, SGW_EINVAL,
                "nstate must be in 1..SGW_MAX_STATES");
    const int K = nstate;
    const int64_t N = ctx->N;
    SGW_REQUIRE(P->n_zeta > 0 && P->first_sample >= 0, SGW_EINVAL, "n_zeta must be > 0");
    SGW_REQUIRE(P->n_eta > 0 && P->n_eta % 2 == 0, SGW_EINVAL, "n_eta must be even and > 0");
    SGW_REQUIRE(P->first_sample + P->n_zeta < (1 << 20) && P->n_eta < (1 << 20), SGW_EINVAL,
                "sample or eta index beyond the RNG stream range");
    SGW_REQUIRE(P->n_tau >= 1 && P->m_sub >= 1 && P->dt > 0 && std::isfinite(P->dt), SGW_EINVAL,
                "bad time grid");
    SGW_REQUIRE(P->ncoef >= 1 && std::isfinite(P->mu) && std::isfinite(P->beta), SGW_EINVAL,
                "bad filter");
    SGW_REQUIRE(P->mode == 0 || P->mode == 1, SGW_EINVAL, "mode must be 0 or 1");
    SGW_REQUIRE(P->filter == 0 || P->filter == 1, SGW_EINVAL, "filter must be 0 or 1");
    if (P->filter == 1)
      SGW_REQUIRE(std::isfinite(P->e_homo) && std::isfinite(P->e_lumo) &&
                      P->e_lumo > P->e_homo && P->filter_eps > 0 && P->filter_eps < 0.5,
                  SGW_EINVAL, "gapped filter needs e_homo < e_lumo and 0 < filter_eps < 0.5");
    SGW_REQUIRE(P->prop_tol > 0, SGW_EINVAL, "prop_tol must be > 0");
    check_interval(P->emin, P->emax);
    const bool xi = P->mode == 0;
    if (xi) {
      SGW_REQUIRE(N % 32 == 0, SGW_EINVAL, "xi mode needs N_g divisible by 32");
      SGW_REQUIRE(P->n_xi >= 1 && P->f_g > 0 && P->f_g <= 1, SGW_EINVAL, "bad n_xi or f_g");
    }
    for (int64_t r = 0; r < K * N; ++r)
      SGW_REQUIRE(std::isfinite(phi[r]), SGW_EINVAL, "phi not finite");
    const int nt1 = P->n_tau + 1;
    const int nft = P->n_ft > 0 ? P->n_ft : next_pow2(4 * nt1);
    SGW_REQUIRE(nft >= 2 * nt1, SGW_EINVAL, "n_ft < 2 (n_tau + 1)");
    const int Sb = P->batch > 0 ? std::min(P->batch, P->n_zeta) : P->n_zeta;
    const int neta = P->n_eta;
    const size_t cs = ctx->csize(), rs = ctx->rsize();

    // coefficients
    std::vector<double> a(P->ncoef), fc(2 * P->ncoef, 0.0);
    if (P->filter == 1)
      gapped_coefficients(P->e_homo, P->e_lumo, P->filter_eps, P->emin, P->emax, P->ncoef,
                          a.data());
    else
      fermi_coefficients(P->mu, P->beta, P->emin, P->emax, P->ncoef, a.data());
    for (int i = 0; i < P->ncoef; ++i) fc[2 * i] = a[i];
    // zeta propagator: the output steps come G at a time from one sweep
    // (coefficients of the times dt .. G dt)
    const int G = std::max(1, std::min(ctx->zeta_sweep, std::min(kMaxSweep, P->n_tau)));
    std::vector<std::vector<double>> pbs(G);
    for (int g = 0; g < G; ++g)
      propagator_coefficients(P->emin, P->emax, (g + 1) * P->dt, P->prop_tol, pbs[g]);
    // time-ordering twiddles
    std::vector<double> tw(2 * nft);
    for (int j = 0; j < nft; ++j) {
      tw[2 * j] = std::cos(2.0 * M_PI * j / nft);
      tw[2 * j + 1] = -std::sin(2.0 * M_PI * j / nft);
    }
    DevBuf &d_tw = ctx->buf("to_tw", cs * nft);
    upload_cplx(ctx, d_tw, tw.data(), nft);
    DevBuf &d_phi = ctx->buf("phi", rs * N * K);
    upload_real(ctx, d_phi, phi, (size_t)K * N);
    auto phi_of = [&](int k) { return static_cast<const char *>(d_phi.p) + rs * N * k; };
    const int nseg = xi ? std::max(1, (int)std::floor(P->f_g * N / 32.0 + 0.5)) : 0;
    SGW_REQUIRE(!xi || nseg <= N / 32, SGW_EINVAL, "f_g too large");
    const double amp = xi ? 1.0 / std::sqrt(P->n_xi * (32.0 * nseg / N) * ctx->dV) : 0.0;
    const int64_t n_inner = xi ? P->n_xi : N;

    hipEvent_t ev[9];                    // phases; [7], [8]: zeta stream fork and join
    for (auto &e : ev) SGW_HIP(hipEventCreate(&e));
    double ph[6] = {0, 0, 0, 0, 0, 0};
    struct EvGuard { hipEvent_t *e; ~EvGuard() { for (int i = 0; i < 9; ++i) (void)hipEventDestroy(e[i]); } } eg{ev};

    for (int b0 = 0; b0 < P->n_zeta; b0 += Sb) {
      const int S = std::min(Sb, P->n_zeta - b0);
      const int64_t nr = (int64_t)S * (1 + neta), nc = (nr + 1) / 2;
      SGW_HIP(hipEventRecord(ev[0], ctx->stream));
      // 1. white noise keys (zeta-bar, then eta-bar_l, per sample)
      std::vector<uint64_t> keys(nr), ksup(S), ksign(S);
      for (int s = 0; s < S; ++s) {
        const uint64_t g = (uint64_t)(P->first_sample + b0 + s);
        keys[(int64_t)s * (1 + neta)] = rng_key(P->seed, rng_stream(RNG_ZETA, g, 0));
        for (int l = 0; l < neta; ++l)
          keys[(int64_t)s * (1 + neta) + 1 + l] = rng_key(P->seed, rng_stream(RNG_ETA, g, l));
        ksup[s] = rng_key(P->seed, rng_stream(RNG_XI_SUPPORT, g, 0));
        ksign[s] = rng_key(P->seed, rng_stream(RNG_XI_SIGN, g, 0));
      }
      DevBuf &d_keys = ctx->buf("keys", sizeof(uint64_t) * nr);
      SGW_HIP(hipMemcpyAsync(d_keys.p, keys.data(), sizeof(uint64_t) * nr, hipMemcpyHostToDevice, ctx->stream));
      DevBuf &d_ksup = ctx->buf("ksup", sizeof(uint64_t) * S);
      DevBuf &d_ksign = ctx->buf("ksign", sizeof(uint64_t) * S);
      SGW_HIP(hipMemcpyAsync(d_ksup.p, ksup.data(), sizeof(uint64_t) * S, hipMemcpyHostToDevice, ctx->stream));
      SGW_HIP(hipMemcpyAsync(d_ksign.p, ksign.data(), sizeof(uint64_t) * S, hipMemcpyHostToDevice, ctx->stream));
      const size_t fbytes = cs * N * nc;
      void *F0 = ctx->buf("f_a", fbytes).p, *F1 = ctx->buf("f_b", fbytes).p;
      void *FA = ctx->buf("f_acc", fbytes).p, *FT = ctx->buf("f_tmp", fbytes).p;
      launch_fill_noise(ctx, d_keys.as<uint64_t>(), nr, F0);
      SGW_HIP(hipEventRecord(ev[1], ctx->stream));
      // 2. filter, Eq. (3), in chunks of vectors whose working set (four
      // vectors each) can stay in the last-level cache between passes
      const int64_t fchunk = ctx->filter_chunk > 0 ? std::min<int64_t>(ctx->filter_chunk, nc) : nc;
      DevBuf &d_n1 = ctx->buf("norm_out", sizeof(double) * nc);
      for (int64_t c0 = 0; c0 < nc; c0 += fchunk) {
        const int64_t ncc = std::min(fchunk, nc - c0);
        const size_t o = cs * N * c0;
        void *last = cheb_series(ctx, static_cast<char *>(F0) + o, static_cast<char *>(F1) + o,
                                 static_cast<char *>(FA) + o, static_cast<char *>(FT) + o, ncc, fc,
                                 P->emin, P->emax);
        launch_norm2(ctx, last, N, ncc, d_n1.as<double>() + c0);
      }
      SGW_HIP(hipEventRecord(ev[2], ctx->stream));
      {
        // ||T_n(H~) x|| <= ||x|| = sqrt(2 N) per complex vector of +-1/sqrt(dV)
        DevBuf &d = d_n1;
        std::vector<double> n1(nc);
        SGW_HIP(hipMemcpyAsync(n1.data(), d.p, sizeof(double) * nc, hipMemcpyDeviceToHost, ctx->stream));
        SGW_HIP(hipStreamSynchronize(ctx->stream));
        const double bound = 1.02 * 2.0 * (double)N / ctx->dV;
        for (double v : n1)
          SGW_REQUIRE(std::isfinite(v) && v <= bound, SGW_EDIVERGED,
                      "filter recurrence grew: [emin, emax] does not enclose spec(H)");
      }
      // 3. unpack, kick potentials, exchange (per state), TDH start.  psi
      // holds per sample the eta set and one tangent copy per state.
      // a leading dimension off a multiple of 1024 points spreads the same
      // tile of successive vectors over cache sets (the KB kernels)
      const int64_t ldp = N % 1024 == 0 ? N + 64 : N;
      void *psi = ctx->buf("tdh_psi", cs * ldp * (1 + K) * neta * S).p;
      void *zeta = ctx->buf("zeta", cs * N * 2 * S).p;
      char *kick = static_cast<char *>(ctx->buf("kick", cs * N * S * K).p);
      const int64_t nxf = (int64_t)S * neta / 2;
      DevBuf &d_xd = ctx->buf("xdots", sizeof(double) * nxf * K);
      for (int k = 0; k < K; ++k) {
        UnpackArgs ua;
        ua.filt = FA; ua.keys = d_keys.as<uint64_t>(); ua.phi = phi_of(k);
        ua.psi = k == 0 ? psi : nullptr; ua.zeta = k == 0 ? zeta : nullptr;
        ua.kick = kick + cs * N * S * k; ua.xsrc = F0; ua.S = S; ua.neta = neta;
        ua.ncopy = 1 + K;
        ua.ldp = ldp;
        launch_unpack(ctx, ua);
        fft3d_apply(ctx, F0, FT, F1, nxf, N, MUL_COUL, 0.0, PLANE_INV_STORE, EpiArgs());
        launch_redot(ctx, F0, F1, N, nxf, d_xd.as<double>() + nxf * k);
      }
      void *dv = ctx->buf("dv", rs * N * S * K).p;
      poisson(ctx, kick, (int64_t)S * K, PLANE_INV_SPLIT, dv, nullptr, nullptr);
      std::vector<double> xd(nxf * K);
      SGW_HIP(hipMemcpyAsync(xd.data(), d_xd.p, sizeof(double) * nxf * K, hipMemcpyDeviceToHost,
                             ctx->stream));
      sgw_tdh_state st;
      st.nsample = S; st.neta = neta; st.weight = 2.0 / neta; st.psi = psi;
      st.v = ctx->buf("tdh_v", rs * N * S).p;
      st.u = ctx->buf("tdh_u", rs * N * S * K).p;
      st.vh0 = ctx->buf("tdh_vh0", rs * N * S).p;
      tdh_start(ctx, &st, ldp, K, dv);
      // u and the stored rows of state k
      const size_t cr_state = rs * (size_t)S * nt1 * n_inner;
      auto u_of = [&](int k) { return static_cast<const char *>(st.u) + rs * N * S * k; };
      int *blocks = nullptr;
      void *cR = nullptr;
      if (xi) {
        blocks = ctx->buf("xi_blocks", sizeof(int) * (size_t)S * P->n_xi * nseg).as<int>();
        launch_xi_supports(ctx, d_ksup.as<uint64_t>(), S, P->n_xi, nseg, blocks);
        cR = ctx->buf("xi_cR", cr_state * K).p;
        for (int k = 0; k < K; ++k)
          launch_xi_real(ctx, u_of(k), blocks, d_ksign.as<uint64_t>(), S, P->n_xi, nseg,
                         amp * ctx->dV, static_cast<char *>(cR) + cr_state * k,
                         (int64_t)nt1 * P->n_xi, 0);
      } else {
        cR = ctx->buf("U", cr_state * K).p;
        SGW_HIP(hipMemcpy2DAsync(cR, rs * N * nt1, st.u, rs * N, rs * N, (size_t)S * K,
                                 hipMemcpyDeviceToDevice, ctx->stream));
      }
      SGW_HIP(hipEventRecord(ev[3], ctx->stream));
      // zeta propagation, Eq. (4).  In xi mode it runs on the context's second
      // stream beside the TDH steps (the two meet only in the contraction),
      // and its overlaps d_m(t_j) are kept for every output step.
      const bool ovl = xi && ctx->overlap;
      if (ovl) ctx->make_aux();
      hipStream_t zs = ovl ? ctx->aux : ctx->stream;
      const char *zns = ovl ? "|z" : "";
      void *zacc, *zt;
      {
        OnStream on(ctx, zs, zns);
        zacc = ctx->buf("z_acc", cs * N * 2 * S * G).p;
        zt = ctx->buf("z_tmp", cs * N * 2 * S).p;
      }
      const size_t dstep = cs * (size_t)S * (ovl ? P->n_xi : 0);   // one (step, state) of d
      char *dpa = ovl ? static_cast<char *>(ctx->buf("xi_dp_all", dstep * nt1 * K).p) : nullptr;
      char *dta = ovl ? static_cast<char *>(ctx->buf("xi_dt_all", dstep * nt1 * K).p) : nullptr;
      // zeta(t_j) for j = 0, 1, 2, ... in turn: a sweep from zeta(t_{j-1})
      // gives the steps j .. j + G - 1 (fewer at the end); the last of them
      // is copied back to be the next sweep's start
      auto zeta_at = [&](int j) -> void * {
        if (j == 0) return zeta;
        const int g = (j - 1) % G;
        if (g == 0) {
          const int64_t nz = 2 * S;
          if (j > 1)
            launch_copy(ctx, static_cast<char *>(zacc) + cs * N * nz * (G - 1), N, zeta, N, nz);
          const int gn = std::min(G, nt1 - j);
          const std::vector<std::vector<double>> sub(pbs.begin(), pbs.begin() + gn);
          cheb_sweep(ctx, zeta, zacc, zt, nz, sub, P->emin, P->emax);
        }
        return static_cast<char *>(zacc) + cs * N * 2 * S * g;
      };
      auto zeta_step = [&](int j) {
        OnStream on(ctx, zs, zns);
        void *zc = zeta_at(j);
        for (int k = 0; k < K; ++k)
          launch_xi_zeta(ctx, zc, phi_of(k), blocks, d_ksign.as<uint64_t>(), S, P->n_xi, nseg,
                         amp * ctx->dV, dpa + dstep * ((size_t)j * K + k),
                         dta + dstep * ((size_t)j * K + k));
      };
      if (ovl) {
        SGW_HIP(hipEventRecord(ev[7], ctx->stream));
        SGW_HIP(hipStreamWaitEvent(zs, ev[7], 0));
        zeta_step(0);
      }
      // 4. TDH response, stored at the output steps
      const double tau = P->dt / P->m_sub;
      const bool tdh_graph = ctx->graphs && !ctx->ktimer && xi && nt1 > 2;
      for (int j = 1; j < nt1; ++j) {
        if (tdh_graph && j == 2) {
          // output steps 2 .. n_tau replay one captured step; j on the device
          const std::string key =
              "tdh|" + ptr_key({st.psi, st.v, st.u, st.vh0, cR, blocks, d_ksign.p}) +
              num_key({(double)S, (double)neta, (double)P->m_sub, tau, (double)P->n_xi,
                       (double)nseg, amp * ctx->dV, (double)nt1, (double)K});
          hipGraphExec_t ex = captured(ctx, key, [&] {
            tdh_substeps(ctx, &st, ldp, K, P->m_sub, tau, false, false);
            for (int k = 0; k < K; ++k)
              launch_xi_real(ctx, u_of(k), blocks, d_ksign.as<uint64_t>(), S, P->n_xi, nseg,
                             amp * ctx->dV, static_cast<char *>(cR) + cr_state * k,
                             (int64_t)nt1 * P->n_xi, 0, ctx->d_counter.as<int>() + 1, P->n_xi);
            launch_counter(ctx, 1, 1, true);
          });
          if (ex) {
            launch_counter(ctx, 1, 2, false);
            for (; j < nt1; ++j) {
              SGW_HIP(hipGraphLaunch(ex, ctx->stream));
              if (ovl) zeta_step(j);
            }
            break;
          }
        }
        tdh_substeps(ctx, &st, ldp, K, P->m_sub, tau, j == 1, false);
        if (xi)
          for (int k = 0; k < K; ++k)
            launch_xi_real(ctx, u_of(k), blocks, d_ksign.as<uint64_t>(), S, P->n_xi, nseg,
                           amp * ctx->dV, static_cast<char *>(cR) + cr_state * k,
                           (int64_t)nt1 * P->n_xi, (int64_t)j * P->n_xi);
        else
          SGW_HIP(hipMemcpy2DAsync(static_cast<char *>(cR) + rs * N * j, rs * N * nt1, st.u, rs * N,
                                   rs * N, (size_t)S * K, hipMemcpyDeviceToDevice, ctx->stream));
        if (ovl) zeta_step(j);
      }
      SGW_HIP(hipEventRecord(ev[4], ctx->stream));
      // 5. time ordering
      const size_t cto_state = cs * (size_t)S * nt1 * n_inner;
      char *cto = static_cast<char *>(ctx->buf("cTO", cto_state * K).p);
      SGW_REQUIRE(launch_time_order(ctx, cR, cto, (int64_t)K * S * n_inner, n_inner, nt1, nft,
                                    d_tw.p),
                  SGW_EUNSUPPORTED, "time-ordering length not built");
      SGW_HIP(hipEventRecord(ev[5], ctx->stream));
      // 6. contraction, Eq. (5) (with the zeta propagation here when it did
      // not run beside the TDH)
      double *d_sig = ctx->buf("sig", sizeof(double) * 4 * S * nt1 * K).as<double>();
      if (ovl) {
        SGW_HIP(hipEventRecord(ev[8], zs));
        SGW_HIP(hipStreamWaitEvent(ctx->stream, ev[8], 0));
        // all steps of a state in one launch (overlaps of step j at (j K + k) dstep)
        for (int k = 0; k < K; ++k)
          for (int j0 = 0; j0 < nt1; j0 += 65535)
            launch_contract_xi(ctx, cto + cto_state * k, dpa + dstep * ((size_t)j0 * K + k),
                               dta + dstep * ((size_t)j0 * K + k), S, P->n_xi, nt1, j0,
                               d_sig + (size_t)4 * S * nt1 * k, std::min(65535, nt1 - j0),
                               (int64_t)(dstep / cs) * K);
      }
      void *dp = nullptr, *dtl = nullptr;
      double *partial = nullptr;
      if (xi) {
        dp = ctx->buf("xi_dp", cs * (size_t)S * P->n_xi).p;
        dtl = ctx->buf("xi_dt", cs * (size_t)S * P->n_xi).p;
      } else {
        partial = ctx->buf("c_partial", sizeof(double) * 4 * S * ((N + 4095) / 4096)).as<double>();
      }
      for (int j = 0; j < (ovl ? 0 : nt1); ++j) {
        void *zc = zeta_at(j);
        for (int k = 0; k < K; ++k) {
          double *sig_k = d_sig + (size_t)4 * S * nt1 * k;
          if (xi) {
            launch_xi_zeta(ctx, zc, phi_of(k), blocks, d_ksign.as<uint64_t>(), S, P->n_xi, nseg,
                           amp * ctx->dV, dp, dtl);
            launch_contract_xi(ctx, cto + cto_state * k, dp, dtl, S, P->n_xi, nt1, j, sig_k);
          } else {
            launch_contract_exact(ctx, cto + cto_state * k, zc, phi_of(k), S, nt1, j, partial,
                                  sig_k);
          }
        }
      }
      SGW_HIP(hipEventRecord(ev[6], ctx->stream));
      std::vector<double> sig(4 * (size_t)S * nt1 * K);
      SGW_HIP(hipMemcpyAsync(sig.data(), d_sig, sizeof(double) * sig.size(), hipMemcpyDeviceToHost, ctx->stream));
      SGW_HIP(hipStreamSynchronize(ctx->stream));
      // assemble
      for (int k = 0; k < K; ++k)
      for (int s = 0; s < S; ++s) {
        double *o = sigma_t + ((size_t)k * P->n_zeta + b0 + s) * 2 * (2 * P->n_tau + 1);
        const double *g = sig.data() + ((size_t)k * S + s) * nt1 * 4;
        for (int j = 1; j < nt1; ++j) {
          o[2 * (P->n_tau + j)] = g[4 * j];
          o[2 * (P->n_tau + j) + 1] = g[4 * j + 1];
          o[2 * (P->n_tau - j)] = g[4 * j + 2];
          o[2 * (P->n_tau - j) + 1] = g[4 * j + 3];
        }
        o[2 * P->n_tau] = 0.5 * (g[0] + g[2]);
        o[2 * P->n_tau + 1] = 0.5 * (g[1] + g[3]);
        double xs = 0;
        for (int q = 0; q < neta / 2; ++q) xs += xd[(size_t)nxf * k + (size_t)s * (neta / 2) + q];
        x_out[(size_t)k * P->n_zeta + b0 + s] = -ctx->dV * xs / neta;
      }
      float t;
      SGW_HIP(hipEventElapsedTime(&t, ev[1], ev[2])); ph[0] += t;
      SGW_HIP(hipEventElapsedTime(&t, ev[3], ev[4])); ph[1] += t;
      SGW_HIP(hipEventElapsedTime(&t, ev[4], ev[5])); ph[2] += t;
      SGW_HIP(hipEventElapsedTime(&t, ev[5], ev[6])); ph[3] += t;
      float t1, t2;
      SGW_HIP(hipEventElapsedTime(&t1, ev[0], ev[1]));
      SGW_HIP(hipEventElapsedTime(&t2, ev[2], ev[3]));
      ph[4] += t1 + t2;
      SGW_HIP(hipEventElapsedTime(&t, ev[0], ev[6])); ph[5] += t;
    }
    if (phase_ms)
      for (int i = 0; i < 6; ++i) phase_ms[i] = ph[i];
  });
}

// ------------------------------------------------------------------ batch
sgw_status sgw_batch_sigma_estimate(sgw_batch_item *items, int32_t n, int32_t nworkers) {
  if (!items || n < 0 || nworkers < 1) return SGW_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!items[i].ctx || !items[i].params) return SGW_EINVAL;
    for (int j = 0; j < i; ++j)
      if (items[j].ctx == items[i].ctx) return SGW_EINVAL;   // one context per item
  }
  // longest processing time first: cost ~ N log N x (filter terms x filter
  // vectors + TDH substeps x TDH vectors + propagation steps x 2 x terms)
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) {
    const sgw_sigma_params *P = items[i].params;
    const double N = (double)items[i].ctx->N;
    const double fv = 0.5 * P->n_zeta * (1.0 + P->n_eta);
    const double work = P->ncoef * fv + 2.0 * P->n_zeta * P->n_eta * P->n_tau * P->m_sub * 3.0 +
                        2.0 * P->n_zeta * P->n_tau * 16.0;
    cost[i] = N * std::log2(std::max(2.0, N)) * work;
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  const int nw = std::max(1, std::min<int>(nworkers, n));
  std::vector<std::vector<int>> plan(nw);
  std::vector<double> load(nw, 0.0);
  for (int i : order) {
    const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    plan[w].push_back(i);
    load[w] += cost[i];
  }
  auto run = [&](int w) {
    const bool prev = g_no_capture;
    g_no_capture = true;
    struct Restore { bool v; ~Restore() { g_no_capture = v; } } restore{prev};
    for (int i : plan[w]) {
      sgw_batch_item &it = items[i];
      const auto t0 = std::chrono::steady_clock::now();
      it.status = sgw_sigma_estimate(it.ctx, it.params, it.phi, it.sigma_t, it.x, nullptr);
      it.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < nw; ++w) th.emplace_back(run, w);
  if (nw > 0 && n > 0) run(0);
  for (auto &t : th) t.join();
  for (int i = 0; i < n; ++i)
    if (items[i].status != SGW_OK) return items[i].status;
  return SGW_OK;
}

}  // extern "C"
