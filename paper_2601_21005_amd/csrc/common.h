// Internal declarations of libsgw: device types, the context, launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sgw.h"

namespace sgw {

// ---------------------------------------------------------------- types
template <typename R> struct CT;
template <> struct CT<float> { using C = float2; };
template <> struct CT<double> { using C = double2; };
template <typename R> using cplx = typename CT<R>::C;

template <typename C> __host__ __device__ inline C cmake(double re, double im) {
  C c; c.x = re; c.y = im; return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C c; c.x = a.x - b.x; c.y = a.y - b.y; return c; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c;
}
template <typename C> __device__ __forceinline__ C cconj(C a) { a.y = -a.y; return a; }
template <typename C, typename R> __device__ __forceinline__ C cscale(C a, R s) { a.x *= s; a.y *= s; return a; }

// ---------------------------------------------------------------- errors
struct Error {
  sgw_status code;
  std::string msg;
};

#define SGW_HIP(call)                                                            \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw ::sgw::Error{SGW_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define SGW_REQUIRE(cond, code, text)                                            \
  do {                                                                           \
    if (!(cond)) throw ::sgw::Error{code, text};                                 \
  } while (0)

// ---------------------------------------------------------------- device memory
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { if (p) (void)hipFree(p); }
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) { SGW_HIP(hipFree(p)); p = nullptr; bytes = 0; }
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) throw Error{SGW_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed"};
    bytes = b;
  }
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------- KB tiles
// Projector data laid out per 512-point grid tile (16 x 8 x 4, or 8 x 8 x 8):
// for each touched tile the list of projectors whose support meets it and
// their values on the tile's points (zero outside the support).
constexpr int KB_TP = 512;  // points per tile

struct KBHost {
  int nproj = 0;
  std::vector<double> ekb;
  std::vector<int> tile_base;       // [ntile] flat index of the tile's first point
  std::vector<int> tile_off;        // [ntile + 1] CSR into entries
  std::vector<int> entry_proj;      // [nentry] projector of each (tile, projector) entry
  std::vector<double> beta;         // [nentry][512]
  std::vector<int> proj_off;        // [nproj + 1] CSR of entries per projector
  std::vector<int> proj_entries;    // [nentry] entry ids grouped by projector
  std::vector<double> gram;         // [nproj][nproj] S = <beta_p|beta_q>
  std::vector<uint32_t> mask;       // [ntile][16] support bits of the tile's points
};

// ---------------------------------------------------------------- autotuner cache
// Process-wide map of tuned kernel choices, loaded from and saved to the JSON
// file named by SGW_TUNE_CACHE (no file: memory only).  Thread-safe.
bool tune_cache_lookup(const std::string &key, int &choice);
void tune_cache_store(const std::string &key, int choice);

// ---------------------------------------------------------------- context
struct Plan;  // FFT dispatch (sizes, kernels)

}  // namespace sgw

struct sgw_ctx {
  int nx = 0, ny = 0, nz = 0;
  int64_t N = 0;
  double h = 0, dV = 0, ecut = 0;
  sgw_precision prec = SGW_C64;
  bool dbl = false;                  // complex double arithmetic
  hipStream_t stream = nullptr;
  int64_t max_nvec = 0;
  std::vector<double> vloc;          // host copy, FP64
  double vmin = 0, vmax = 0, tmax = 0;
  sgw::KBHost kb;
  bool has_kb = false;
  std::string err;

  // device data
  sgw::DevBuf d_vloc;                // [N] real (R)
  sgw::DevBuf d_k2;                  // kx2 [nx], ky2 [ny], kz2 [nz] (R)
  sgw::DevBuf d_tw;                  // twiddles nx, ny, nz (C), forward sign
  sgw::DevBuf d_kb_tile_base, d_kb_tile_off, d_kb_entry_proj, d_kb_beta,
      d_kb_proj_off, d_kb_proj_entries, d_kb_ekb;
  sgw::DevBuf d_kb_tile_offT;        // [ntile + 1] per-tile offsets of betaT in entry rows
  sgw::DevBuf d_kb_betaT;            // per tile [512][entries padded to the K group], FP32 or BF16
  sgw::DevBuf d_kb_beta16;           // [entry][512] BF16 (the BF16 precisions)
  sgw::DevBuf d_kb_mask;             // [ntile][16] uint32: bit p set where some beta_e(p) != 0
  int kb_ntile = 0, kb_nentry = 0;
  int64_t kb_support_points = 0;     // grid points where some beta_p is nonzero
  int64_t kb_nnz = 0;                // nonzero beta values (point, projector)
  int kb_nek_max = 0;                // largest padded entry count of a tile (scatter LDS)
  int kb_lx = 3, kb_ly = 3;          // tile extent log2 along x and y (512 points)

  // HIP graphs: repeated launch sequences (Chebyshev terms, TDH output
  // steps) captured once and replayed; step-dependent scalars live in
  // d_counter ([0] Chebyshev term, [1] TDH output step)
  bool graphs = false;
  std::map<std::string, hipGraphExec_t> gexec;
  sgw::DevBuf d_counter;

  // launch timers: ktimer bit 0 the inverse plane pass with the Chebyshev
  // epilogue, bit 1 the KB scatter, bit 2 the KB gather (launches on the
  // context's stream)
  struct KTimer {
    std::vector<hipEvent_t> events;   // pairs (start, stop)
    int64_t used = 0, points = 0;
    hipEvent_t event(int which) {
      const size_t i = 2 * (size_t)used + which;
      while (events.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) throw sgw::Error{SGW_EHIP, "hipEventCreate failed"};
        events.push_back(e);
      }
      return events[i];
    }
  };
  int ktimer = 0;
  KTimer kt[3];
  int dev = 0;                 // HIP device the context was created on
  // set while a call must not time kernel variants (sgw_apply_H_noalloc):
  // tune() then returns the forced, remembered or cached choice, else 0
  bool no_tune = false;
  // second stream of the context (non-blocking, default priority): the zeta
  // propagation of sgw_sigma_estimate runs on it beside the TDH steps.  While
  // work is issued there, `ns` suffixes every scratch buffer name so the two
  // streams never share scratch memory.
  hipStream_t aux = nullptr;
  bool overlap = true;
  // the Chebyshev terms' projector gathers run on `aux` beside the FFT passes
  bool kb_overlap = true;
  hipEvent_t kb_fork[2] = {nullptr, nullptr};
  void make_aux() {
    if (!aux) SGW_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
    for (auto &e : kb_fork)
      if (!e) SGW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  int zeta_sweep = 8;   // zeta output steps per Chebyshev sweep (1 .. 8)
  std::string ns;
  ~sgw_ctx() {
    (void)hipDeviceSynchronize();   // no graph or buffer is released while in use
    if (aux) {
      (void)hipStreamSynchronize(aux);
      (void)hipStreamDestroy(aux);
    }
    for (auto e : kb_fork)
      if (e) (void)hipEventDestroy(e);
    for (auto &t : kt)
      for (auto e : t.events) (void)hipEventDestroy(e);
    for (auto &g : gexec) (void)hipGraphExecDestroy(g.second);
  }

  // autotuned kernel variants: key "name/nvec" -> variant index.  Every
  // variant of one name gives bit-identical results (only speed differs).
  std::map<std::string, int> tuned;
  std::map<std::string, int> forced;   // from SGW_FORCE_VARIANT="name=i,name=i"
  int64_t filter_chunk = 0;            // vectors per filter chunk (0: the whole batch)
  // Persistent choices: with SGW_TUNE_CACHE=<file> the choice of every
  // (arch, kernel, grid, precision, batch width) is read from and appended
  // to a JSON object in that file, so later runs select without timing.
  std::string arch;                    // gcnArchName of the device
  std::string tune_key(const char *name, int64_t nvec) const {
    return arch + "/" + name + "/" + std::to_string(nx) + "x" + std::to_string(ny) + "x" +
           std::to_string(nz) + "/p" + std::to_string((int)prec) + "/" + std::to_string(nvec);
  }
  // Time every variant four times after a warm-up (the fastest run counts)
  // and keep the lowest index whose time is within 3% of the fastest.
  template <typename F> int tune(const char *name, int64_t nvec, int nvar, F &&trial) {
    const auto fit = forced.find(name);
    if (fit != forced.end() && fit->second >= 0 && fit->second < nvar) return fit->second;
    const std::string key = tune_key(name, nvec);
    const auto it = tuned.find(key);
    if (it != tuned.end()) return it->second;
    int cached = -1;
    if (sgw::tune_cache_lookup(key, cached) && cached >= 0 && cached < nvar) {
      if (!no_tune) tuned[key] = cached;
      return cached;
    }
    if (no_tune) return 0;
    // trials run alone on the device: work of other streams (the context's
    // second stream, other contexts) would otherwise skew their times
    (void)hipDeviceSynchronize();
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      throw sgw::Error{SGW_EHIP, "hipEventCreate failed"};
    std::vector<float> ms(nvar, 1e30f);
    for (int i = 0; i < nvar; ++i) {
      trial(i);                               // warm-up
      for (int rep = 0; rep < 4; ++rep) {
        (void)hipEventRecord(e0, stream);
        trial(i);
        (void)hipEventRecord(e1, stream);
        (void)hipEventSynchronize(e1);
        float t = 0;
        (void)hipEventElapsedTime(&t, e0, e1);
        if (hipGetLastError() == hipSuccess) ms[i] = std::min(ms[i], t);
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const float best_ms = *std::min_element(ms.begin(), ms.end());
    int best = 0;
    while (best + 1 < nvar && ms[best] > 1.03f * best_ms) ++best;
    tuned[key] = best;
    sgw::tune_cache_store(key, best);
    return best;
  }

  // scratch (grown on demand)
  std::map<std::string, std::unique_ptr<sgw::DevBuf>> scratch;
  sgw::DevBuf &buf(const std::string &name, size_t bytes) {
    auto &p = scratch[name + ns];
    if (!p) p.reset(new sgw::DevBuf());
    if (bytes > p->bytes && p->p) clear_graphs();   // captured graphs hold the old address
    p->ensure(bytes);
    return *p;
  }
  void clear_graphs() {
    // a replay of one of them may still run on either stream
    if (!gexec.empty()) (void)hipDeviceSynchronize();
    for (auto &g : gexec) (void)hipGraphExecDestroy(g.second);
    gexec.clear();
  }
  size_t csize() const { return dbl ? 16 : 8; }
  size_t rsize() const { return dbl ? 8 : 4; }
};

namespace sgw {

// ---------------------------------------------------------------- launchers
// FFT pass kinds
enum PlaneMode : int {
  PLANE_FWD = 0,          // dst = FFT_xy(src)
  PLANE_INV_STORE = 1,    // dst = IFFT_xy(src) (no 1/N: folded into the z pass)
  PLANE_INV_HPSI = 2,     // dst = IFFT_xy(tmp) + V x
  PLANE_INV_CHEB = 3,     // Chebyshev update (see EpiArgs)
  PLANE_INV_POISSON = 4,  // v = Vloc + Re - vh0, u = Im  (per sample fields)
  PLANE_INV_SPLIT = 5,    // r0 = Re, r1 = Im  (real fields)
};

enum MulMode : int { MUL_NONE = 0, MUL_KIN = 1, MUL_PROP = 2, MUL_COUL = 3 };

struct EpiArgs {
  const void *x = nullptr;    // complex: current vector (HPSI, CHEB)
  void *vold = nullptr;       // complex: v_{n-1} in, v_{n+1} out (CHEB)
  void *vout = nullptr;       // complex: v_{n+1} out instead of vold when set (CHEB)
  void *acc = nullptr;        // complex: accumulated series (CHEB)
  const void *vloc = nullptr; // real [N]
  const void *vh0 = nullptr;  // real per field (POISSON)
  void *r0 = nullptr;         // real outputs per field
  void *r1 = nullptr;
  double c = 0, invR = 0;     // spectral map
  // CHEB on term n (x = v_n, vold = v_{n-1}): the series takes its terms in
  // pairs, acc (+)= b_{n-1} v_{n-1} + b_n v_n on odd n only
  double cprev_re = 0, cprev_im = 0;  // b_{n-1}
  double coef_re = 0, coef_im = 0;    // b_n
  int acc_mode = 0;           // CHEB: 0 acc untouched, 1 acc = pair, 2 acc += pair
  int first = 0;              // CHEB: v_1 = H~ v_0 (no v_{n-1} term)
  double scale2 = 2.0;        // CHEB: factor of H~ v_n (2, or 1 when first)
  // CHEB inside a replayed graph: b_n = coef_dev[term_dev[0]] and b_{n-1} the
  // entry before (interleaved re, im; FP64), read when the pass runs
  const double *coef_dev = nullptr;
  const int *term_dev = nullptr;
};

// Full forward+multiply+inverse 3D transform of nvec vectors of `src` (ld),
// result written through the inverse pass mode into dst / epilogue outputs.
// tmp holds nvec vectors ld_tmp apart (0: N); it may be dst itself when
// ld_tmp equals ld (every pass after the first works in place per plane,
// pencil or line).  With tmp2 (the layout of tmp) the z pencils read tmp and
// write tmp2, and the inverse passes take tmp2; without it they work in tmp.
// Successive passes take the vectors in alternate directions, the first in
// descending order when rev is set.
void fft3d_apply(sgw_ctx *ctx, const void *src, void *tmp, void *dst, int64_t nvec,
                 int64_t ld, MulMode mul, double tau, PlaneMode inv_mode,
                 const EpiArgs &epi, int64_t ld_tmp = 0, void *tmp2 = nullptr,
                 bool rev = false);

// KB (kb.hip)
// C[p][v] = <beta_p|psi_v>  (kb_gather_e: times E_p)
void kb_gather(sgw_ctx *ctx, const void *psi, int64_t nvec, int64_t ld, void *coef_out);
void kb_gather_e(sgw_ctx *ctx, const void *psi, int64_t nvec, int64_t ld, void *coef_out,
                 void *partial = nullptr);
// bytes of per-(tile, projector) partial sums the gather needs per vector
size_t kb_partial_bytes_per_vec(const sgw_ctx *ctx);
// C' = K C  (K complex [nproj][nproj] in the working precision)
void kb_mix_dense(sgw_ctx *ctx, const void *K, const void *coef_in, void *coef_out,
                  int64_t nvec);
// dst[v] += s1 * B C[v];  if dst2: dst2[v] += s2 * B C[v]  (s1, s2 complex)
// (the MFMA kernels of the complex FP32 precisions take s1 real and no dst2)
void kb_scatter(sgw_ctx *ctx, const void *coef, int64_t nvec, void *dst, int64_t ld,
                double s1re, double s1im, void *dst2, double s2re, double s2im);

// operand arrays of the MFMA kernels (after build_kb and the upload of beta)
void kb_upload_operands(sgw_ctx *ctx);

// host utilities (host.cpp)
// eigenvalues (ascending) and eigenvectors (columns, row-major) of a small
// symmetric matrix (row-major, destroyed)
void jacobi_eigen(int n, std::vector<double> &a, std::vector<double> &vals,
                  std::vector<double> &vecs);
void build_kb(sgw_ctx *ctx, const sgw_projectors *p);
// K (complex, [nproj][nproj] interleaved) with exp(-i tau V_NL) = I + dV B K B^T
void kb_exponential_matrix(const sgw_ctx *ctx, double tau, std::vector<double> &K);
void fermi_coefficients(double mu, double beta, double emin, double emax, int n,
                        double *a);
// gapped filter: erfc step, 1 - eps at e_homo and eps at e_lumo
void gapped_coefficients(double e_homo, double e_lumo, double eps, double emin, double emax,
                         int n, double *a);
// b_n (interleaved re, im) of exp(-i H tau); returns the number of terms
int propagator_coefficients(double emin, double emax, double tau, double tol,
                            std::vector<double> &re_im);
// Bessel J_0..J_nmax(x) by Miller's backward recurrence
void bessel_j(double x, int nmax, std::vector<double> &J);
double kb_lambda_bound(const sgw_ctx *ctx);
int qp_solve(const double *sig, int n_tau, double dt, double gamma, double eks, double x,
             double vxc, double *eg, double *el, double *z);

}  // namespace sgw
