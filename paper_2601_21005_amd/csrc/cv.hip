// Learned control variate for the per-sample self-energy: features of the
// white-noise vectors, a 64 -> 256 -> 256 -> 1 tanh network trained with
// Adam, and the cheap-sample mean of the network's output.  An addition to
// the paper's Monte Carlo average (Sec. 3 averages samples until the QP
// error bar is below 0.03 eV): the control variate lowers the spread of the
// per-sample values without bias when the mean of g is known well.
//
// Every product runs on MFMA with BF16 operands (nearest-even rounding) and
// FP32 accumulation; elementwise work is FP32, sums over samples FP64.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "rng.h"

using namespace sgw;

struct sgw_mlp {
  int din = 0, h1 = 0, h2 = 0;
  int64_t nparam = 0;
  hipStream_t stream = nullptr;
  std::string err;
  DevBuf theta, m, v, grad;            // FP32 master parameters, Adam moments, gradient
  DevBuf mean, inv_std;                // standardization of the features (FP32)
  int64_t t = 0;                       // Adam step count
  std::map<std::string, std::unique_ptr<DevBuf>> scratch;
  DevBuf &buf(const std::string &name, size_t bytes) {
    auto &p = scratch[name];
    if (!p) p.reset(new DevBuf());
    p->ensure(bytes);
    return *p;
  }
  // offsets of the parameter blocks in the packed vector
  int64_t oW1() const { return 0; }
  int64_t ob1() const { return (int64_t)h1 * din; }
  int64_t oW2() const { return ob1() + h1; }
  int64_t ob2() const { return oW2() + (int64_t)h2 * h1; }
  int64_t ow3() const { return ob2() + h2; }
  int64_t ob3() const { return ow3() + h2; }
};

namespace {

thread_local std::string g_mlp_error;

template <typename F> sgw_status guard_mlp(sgw_mlp *m, F &&f) {
  try {
    f();
    return SGW_OK;
  } catch (const Error &e) {
    (m ? m->err : g_mlp_error) = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    (m ? m->err : g_mlp_error) = "host allocation failed";
    return SGW_ENOMEM;
  } catch (const std::exception &e) {
    (m ? m->err : g_mlp_error) = e.what();
    return SGW_EINVAL;
  }
}

template <typename F> sgw_status guard_ctx(sgw_ctx *c, F &&f) {
  try {
    f();
    return SGW_OK;
  } catch (const Error &e) {
    c->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    c->err = "host allocation failed";
    return SGW_ENOMEM;
  } catch (const std::exception &e) {
    c->err = e.what();
    return SGW_EINVAL;
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16r(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// D += A B on v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + s]
// and B[8 (l / 16) + s][l % 16], s = 0..7, and holds D[4 (l / 16) + r][l % 16]
__device__ __forceinline__ void mma(f32x4 &acc, const u32x4 &a, const u32x4 &b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
}

constexpr int NT = 256;

// ---------------------------------------------------------------- features
// phi (FP32 [K][ld]) -> BF16 [64][N], rows K..63 zero
__global__ void k_phi_bf16(const float *phi, int64_t ld, int K, int64_t N, uint16_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 64 * N) return;
  const int k = (int)(i / N);
  const int64_t r = i % N;
  out[i] = k < K ? (uint16_t)bf16r(phi[k * ld + r]) : (uint16_t)0;
}

// x[s][k] = dV (sum_r phi_k(r) sign_s(r))^2 = |<phi_k|zeta_s>|^2 for zeta_s =
// sign / sqrt(dV).  Workgroup: 4 waves x NS tiles of 16 samples; every wave
// runs the whole grid (K = N points, groups of 32) for its samples with the
// 4 x 16 state rows as A and the signs of its samples as B, made in
// registers from the counter-based generator: the 8 signs a lane feeds for
// points r0..r0+7 are 8 bits of word(r0 / 64), bit 0 -> +1.  The A rows of
// each 64-point chunk are staged once per workgroup in LDS (two buffers: the
// next chunk is loaded while the current one is multiplied), so the four
// waves share one read of phi from the cache.
// With neta > 0 the columns are the occupied-orbital noise vectors instead:
// column s is eta-bar_{s / neta, s % neta} (stream kind ETA), and x holds one
// row per column (averaged over l by k_eta_mean).  Rows of x are ldx apart.
template <int NS>
__global__ __launch_bounds__(NT) void k_features(const uint16_t *phi16, int64_t N, int K,
                                                 uint64_t seed, int64_t s0, int64_t nsamp,
                                                 float dV, float *x, int neta, int64_t ldx) {
  constexpr int PA = 72;                           // LDS row pitch (BF16): 64 points + 8
  __shared__ __align__(16) uint16_t sa[2][64 * PA];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, q = lane >> 4, col = lane & 15;
  const int64_t sbase = s0 + ((int64_t)blockIdx.x * 4 + w) * (16 * NS);
  uint64_t key[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const uint64_t c = (uint64_t)(sbase + 16 * t + col);
    key[t] = neta > 0 ? rng_key(seed, rng_stream(RNG_ETA, c / (uint64_t)neta, c % (uint64_t)neta))
                      : rng_key(seed, rng_stream(RNG_ZETA, c, 0));
  }
  f32x4 acc[4][NS];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < NS; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // chunk staging: 64 rows x 64 points = 512 pieces of 16 B, two per thread
  const int row0 = tid >> 3, seg = tid & 7;
  auto fetch = [&](int64_t r64, u32x4 *g) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      g[i] = *reinterpret_cast<const u32x4 *>(phi16 + (int64_t)(row0 + 32 * i) * N + r64 + 8 * seg);
  };
  auto stage = [&](int buf, const u32x4 *g) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      *reinterpret_cast<u32x4 *>(&sa[buf][(row0 + 32 * i) * PA + 8 * seg]) = g[i];
  };
  u32x4 gnext[2];
  fetch(0, gnext);
  stage(0, gnext);
  __syncthreads();
  int buf = 0;
  for (int64_t r64 = 0; r64 < N; r64 += 64) {
    const bool more = r64 + 64 < N;
    if (more) fetch(r64 + 64, gnext);
    uint64_t word[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) word[t] = sm64(key[t] + (uint64_t)(r64 >> 6));
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      u32x4 a[4];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        a[m] = *reinterpret_cast<const u32x4 *>(&sa[buf][(16 * m + col) * PA + 32 * half + 8 * q]);
      const int sh = 32 * half + 8 * q;
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const uint32_t bits = (uint32_t)(word[t] >> sh);
        u32x4 b;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[j] = 0x3F803F80u | ((bits >> (2 * j)) & 1u) << 15 | ((bits >> (2 * j + 1)) & 1u) << 31;
#pragma unroll
        for (int m = 0; m < 4; ++m) mma(acc[m][t], a[m], b);
      }
    }
    if (more) stage(buf ^ 1, gnext);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int64_t s = sbase + 16 * t + col;
    if (s - s0 >= nsamp) continue;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 16 * m + 4 * q + r;
        if (k < K) x[(s - s0) * ldx + k] = dV * acc[m][t][r] * acc[m][t][r];
      }
  }
}

constexpr int FEAT_NS = 4;                     // 256 samples per workgroup

// x[i][k] = (1/neta) sum_l y[i neta + l][k], summed in order of l
__global__ void k_eta_mean(const float *y, int64_t nsamp, int neta, int K, float *x,
                           int64_t ldx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsamp * K) return;
  const int64_t s = i / K;
  const int k = (int)(i % K);
  float acc = 0.f;
  for (int l = 0; l < neta; ++l) acc += y[(s * neta + l) * K + k];
  x[s * ldx + k] = acc / (float)neta;
}

// features of nsamp samples from s0 into x (rows ldx apart): zeta-bar
// (neta = 0) or the mean over the sample's neta eta-bar vectors
void features(sgw_ctx *ctx, const float *phi, int K, int64_t ld, uint64_t seed, int64_t s0,
              int64_t nsamp, float *x, int neta = 0, int64_t ldx = 0) {
  const int64_t N = ctx->N;
  if (ldx <= 0) ldx = K;
  DevBuf &p16 = ctx->buf("cv_phi16", sizeof(uint16_t) * 64 * (size_t)N);
  hipLaunchKernelGGL(k_phi_bf16, dim3((unsigned)((64 * N + NT - 1) / NT)), dim3(NT), 0,
                     ctx->stream, phi, ld, K, N, p16.as<uint16_t>());
  SGW_HIP(hipGetLastError());
  const int64_t per = 4 * 16 * FEAT_NS;
  if (neta <= 0) {
    const int64_t nblk = (nsamp + per - 1) / per;
    hipLaunchKernelGGL(k_features<FEAT_NS>, dim3((unsigned)nblk), dim3(NT), 0, ctx->stream,
                       p16.as<uint16_t>(), N, K, seed, s0, nsamp, (float)ctx->dV, x, 0, ldx);
    SGW_HIP(hipGetLastError());
    return;
  }
  const int64_t ncol = nsamp * neta;
  float *y = ctx->buf("cv_eta_cols", sizeof(float) * (size_t)ncol * K).as<float>();
  const int64_t nblk = (ncol + per - 1) / per;
  hipLaunchKernelGGL(k_features<FEAT_NS>, dim3((unsigned)nblk), dim3(NT), 0, ctx->stream,
                     p16.as<uint16_t>(), N, K, seed, s0 * neta, ncol, (float)ctx->dV, y, neta,
                     (int64_t)K);
  SGW_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_eta_mean, dim3((unsigned)((nsamp * K + NT - 1) / NT)), dim3(NT), 0,
                     ctx->stream, y, nsamp, neta, K, x, ldx);
  SGW_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- MLP GEMM
// C(m, n) = sum_k A(m, k) B(k, n) for strided FP32 operands, rounded to BF16
// in LDS; 64 x 64 output tile per workgroup, wave w owns rows 16 w .. 16 w + 15.
enum Epi { EPI_STORE = 0, EPI_TANH_BIAS = 1, EPI_DTANH = 2 };

struct GemmArgs {
  const float *a; int64_t sam, sak;
  const float *b; int64_t sbk, sbn;
  float *c; int64_t scm, scn;
  const float *bias;        // EPI_TANH_BIAS: [M]
  const float *aux;         // EPI_DTANH: activation at the strides of C
  int M, N, K;
};

template <int EPI>
__global__ __launch_bounds__(NT) void k_gemm(GemmArgs g) {
  constexpr int P = 40;                       // LDS pitch (bf16): 80 B, conflict-free 16 B reads
  __shared__ __align__(16) uint16_t As[64 * P], Bs[64 * P];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, col = lane & 15;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool ak = g.sak == 1, bk = g.sbk == 1;
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    float av[8], bv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = tid + NT * i;
      const int am = ak ? idx / 32 : idx % 64, akk = ak ? idx % 32 : idx / 64;
      const int bn = bk ? idx / 32 : idx % 64, bkk = bk ? idx % 32 : idx / 64;
      av[i] = (m0 + am < g.M && k0 + akk < g.K) ? g.a[(m0 + am) * g.sam + (k0 + akk) * g.sak] : 0.f;
      bv[i] = (n0 + bn < g.N && k0 + bkk < g.K) ? g.b[(k0 + bkk) * g.sbk + (n0 + bn) * g.sbn] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = tid + NT * i;
      const int am = ak ? idx / 32 : idx % 64, akk = ak ? idx % 32 : idx / 64;
      const int bn = bk ? idx / 32 : idx % 64, bkk = bk ? idx % 32 : idx / 64;
      As[am * P + akk] = (uint16_t)bf16r(av[i]);
      Bs[bn * P + bkk] = (uint16_t)bf16r(bv[i]);
    }
    __syncthreads();
    const u32x4 a = *reinterpret_cast<const u32x4 *>(As + (16 * w + col) * P + 8 * q);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const u32x4 b = *reinterpret_cast<const u32x4 *>(Bs + (16 * t + col) * P + 8 * q);
      mma(acc[t], a, b);
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + 16 * w + 4 * q + r, n = n0 + 16 * t + col;
      if (m >= g.M || n >= g.N) continue;
      const int64_t o = m * g.scm + n * g.scn;
      float v = acc[t][r];
      if (EPI == EPI_TANH_BIAS) v = tanhf(v + g.bias[m]);
      if (EPI == EPI_DTANH) {
        const float h = g.aux[o];
        v *= 1.f - h * h;
      }
      g.c[o] = v;
    }
}

template <int EPI> void gemm(hipStream_t st, const GemmArgs &g) {
  if (g.M <= 0 || g.N <= 0) return;
  const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  SGW_REQUIRE(grid.y <= 65535, SGW_EUNSUPPORTED, "GEMM: M too large");
  hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(NT), 0, st, g);
  SGW_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- small kernels
// xh[s][k] = (x[s][k] - mean[k]) * inv_std[k]
__global__ void k_standardize(const float *x, const float *mean, const float *inv_std, int din,
                              int64_t n, float *xh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * din) return;
  const int k = (int)(i % din);
  xh[i] = (x[i] - mean[k]) * inv_std[k];
}

// g[s] = w3 . a2[s] + b3  (FP32, fixed order)
__global__ void k_output(const float *a2, const float *w3, const float *b3, int h2, int64_t n,
                         float *g) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float acc = 0.f;
  for (int j = 0; j < h2; ++j) acc += w3[j] * a2[s * h2 + j];
  g[s] = acc + b3[0];
}

// dg[s] = 2 (g[s] - y[s]) / n;  e2[s] = (g[s] - y[s])^2 (FP64)
__global__ void k_residual(const float *g, const float *y, int64_t n, float *dg, double *e2) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double r = (double)g[s] - (double)y[s];
  dg[s] = (float)(2.0 * r / (double)n);
  e2[s] = r * r;
}

// d2[s][j] = dg[s] w3[j] (1 - a2[s][j]^2)
__global__ void k_back_out(const float *dg, const float *w3, const float *a2, int h2, int64_t n,
                           float *d2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * h2) return;
  const int j = (int)(i % h2);
  const float h = a2[i];
  d2[i] = dg[i / h2] * w3[j] * (1.f - h * h);
}

// out[j] = sum_s a[s][j] * (wt ? wt[s] : 1) for j < cols (FP64 accumulation, fixed order)
__global__ void k_colsum(const float *a, const float *wt, int cols, int64_t n, float *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double acc = 0.0;
  for (int64_t s = 0; s < n; ++s) acc += (double)a[s * cols + j] * (wt ? (double)wt[s] : 1.0);
  out[j] = (float)acc;
}

// deterministic FP64 sums: stage 1 per block, stage 2 in block order
template <int POW>
__global__ void k_sum1(const float *x, const double *xd, int64_t n, double *partial) {
  __shared__ double sh[NT];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const double v = x ? (double)x[i] : xd[i];
    acc += POW == 2 ? v * v : v;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_sum2(const double *partial, int nblk, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  for (int i = 0; i < nblk; ++i) acc += partial[i];
  out[0] = acc;
}

constexpr int SUM_BLOCKS = 256;

// out = sum x (POW 1) or sum x^2 (POW 2), left on the device
template <int POW>
void dsum(hipStream_t st, const float *x, const double *xd, int64_t n, double *partial,
          double *out) {
  hipLaunchKernelGGL(k_sum1<POW>, dim3(SUM_BLOCKS), dim3(NT), 0, st, x, xd, n, partial);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(64), 0, st, partial, SUM_BLOCKS, out);
  SGW_HIP(hipGetLastError());
}

// Adam with bias-corrected moments; c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
__global__ void k_adam(float *theta, float *m, float *v, const float *grad, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// ---------------------------------------------------------------- network passes
struct Acts {
  float *xh, *a1, *a2, *g;
};

Acts activations(sgw_mlp *M, int64_t n) {
  Acts a;
  a.xh = M->buf("xh", sizeof(float) * n * M->din).as<float>();
  a.a1 = M->buf("a1", sizeof(float) * n * M->h1).as<float>();
  a.a2 = M->buf("a2", sizeof(float) * n * M->h2).as<float>();
  a.g = M->buf("g", sizeof(float) * n).as<float>();
  return a;
}

// g = network(x) for n samples (x [n][din]); activations kept in `a`
void forward(sgw_mlp *M, const float *x, int64_t n, const Acts &a) {
  const float *th = M->theta.as<float>();
  hipStream_t st = M->stream;
  hipLaunchKernelGGL(k_standardize, dim3(blocks(n * M->din)), dim3(NT), 0, st, x,
                     M->mean.as<float>(), M->inv_std.as<float>(), M->din, n, a.xh);
  SGW_HIP(hipGetLastError());
  GemmArgs g{};
  // a1[s][j] = tanh(sum_k W1[j][k] xh[s][k] + b1[j])
  g.a = th + M->oW1(); g.sam = M->din; g.sak = 1;
  g.b = a.xh; g.sbk = 1; g.sbn = M->din;
  g.c = a.a1; g.scm = 1; g.scn = M->h1;
  g.bias = th + M->ob1(); g.M = M->h1; g.N = (int)n; g.K = M->din;
  gemm<EPI_TANH_BIAS>(st, g);
  // a2[s][j] = tanh(sum_k W2[j][k] a1[s][k] + b2[j])
  g.a = th + M->oW2(); g.sam = M->h1; g.sak = 1;
  g.b = a.a1; g.sbk = 1; g.sbn = M->h1;
  g.c = a.a2; g.scm = 1; g.scn = M->h2;
  g.bias = th + M->ob2(); g.M = M->h2; g.K = M->h1;
  gemm<EPI_TANH_BIAS>(st, g);
  hipLaunchKernelGGL(k_output, dim3(blocks(n)), dim3(NT), 0, st, a.a2, th + M->ow3(),
                     th + M->ob3(), M->h2, n, a.g);
  SGW_HIP(hipGetLastError());
}

// gradient of L = (1/n) sum (g - y)^2 into M->grad; the loss (FP64) into *d_loss
void backward(sgw_mlp *M, const float *y, int64_t n, const Acts &a, double *d_loss) {
  const float *th = M->theta.as<float>();
  float *gr = M->grad.as<float>();
  hipStream_t st = M->stream;
  float *dg = M->buf("dg", sizeof(float) * n).as<float>();
  double *e2 = M->buf("e2", sizeof(double) * n).as<double>();
  double *part = M->buf("part", sizeof(double) * SUM_BLOCKS).as<double>();
  float *d2 = M->buf("d2", sizeof(float) * n * M->h2).as<float>();
  float *d1 = M->buf("d1", sizeof(float) * n * M->h1).as<float>();
  hipLaunchKernelGGL(k_residual, dim3(blocks(n)), dim3(NT), 0, st, a.g, y, n, dg, e2);
  SGW_HIP(hipGetLastError());
  dsum<1>(st, nullptr, e2, n, part, d_loss);
  // dw3 = sum_s dg[s] a2[s], db3 = sum_s dg[s]
  hipLaunchKernelGGL(k_colsum, dim3(blocks(M->h2)), dim3(NT), 0, st, a.a2, dg, M->h2, n,
                     gr + M->ow3());
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(NT), 0, st, dg, nullptr, 1, n, gr + M->ob3());
  hipLaunchKernelGGL(k_back_out, dim3(blocks(n * M->h2)), dim3(NT), 0, st, dg, th + M->ow3(),
                     a.a2, M->h2, n, d2);
  SGW_HIP(hipGetLastError());
  GemmArgs g{};
  // dW2[j][k] = sum_s d2[s][j] a1[s][k]
  g.a = d2; g.sam = 1; g.sak = M->h2;
  g.b = a.a1; g.sbk = M->h1; g.sbn = 1;
  g.c = gr + M->oW2(); g.scm = M->h1; g.scn = 1;
  g.M = M->h2; g.N = M->h1; g.K = (int)n;
  gemm<EPI_STORE>(st, g);
  hipLaunchKernelGGL(k_colsum, dim3(blocks(M->h2)), dim3(NT), 0, st, d2, nullptr, M->h2, n,
                     gr + M->ob2());
  // d1[s][k] = (sum_j W2[j][k] d2[s][j]) (1 - a1[s][k]^2)
  g = GemmArgs{};
  g.a = th + M->oW2(); g.sam = 1; g.sak = M->h1;
  g.b = d2; g.sbk = 1; g.sbn = M->h2;
  g.c = d1; g.scm = 1; g.scn = M->h1;
  g.aux = a.a1; g.M = M->h1; g.N = (int)n; g.K = M->h2;
  gemm<EPI_DTANH>(st, g);
  // dW1[j][k] = sum_s d1[s][j] xh[s][k]
  g = GemmArgs{};
  g.a = d1; g.sam = 1; g.sak = M->h1;
  g.b = a.xh; g.sbk = M->din; g.sbn = 1;
  g.c = gr + M->oW1(); g.scm = M->din; g.scn = 1;
  g.M = M->h1; g.N = M->din; g.K = (int)n;
  gemm<EPI_STORE>(st, g);
  hipLaunchKernelGGL(k_colsum, dim3(blocks(M->h1)), dim3(NT), 0, st, d1, nullptr, M->h1, n,
                     gr + M->ob1());
  SGW_HIP(hipGetLastError());
}

void adam(sgw_mlp *M, double lr, double b1, double b2, double eps) {
  M->t += 1;
  const double c1 = 1.0 / (1.0 - std::pow(b1, (double)M->t));
  const double c2 = 1.0 / (1.0 - std::pow(b2, (double)M->t));
  hipLaunchKernelGGL(k_adam, dim3(blocks(M->nparam)), dim3(NT), 0, M->stream,
                     M->theta.as<float>(), M->m.as<float>(), M->v.as<float>(),
                     M->grad.as<float>(), M->nparam, (float)lr, (float)b1, (float)b2,
                     (float)eps, (float)c1, (float)c2);
  SGW_HIP(hipGetLastError());
}

void check_n(int64_t n) {
  SGW_REQUIRE(n > 0 && n <= (int64_t)1 << 30, SGW_EINVAL, "sample count out of range");
}

}  // namespace

// =================================================================== ABI
extern "C" {

const char *sgw_mlp_last_error(const sgw_mlp *m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

sgw_status sgw_cv_features(sgw_ctx *ctx, const float *phi, int32_t K, int64_t ld_phi,
                           uint64_t seed, int64_t first_sample, int64_t nsamp, float *x) {
  if (!ctx) return SGW_EINVAL;
  return guard_ctx(ctx, [&] {
    SGW_REQUIRE(phi && x, SGW_EINVAL, "NULL argument");
    SGW_REQUIRE(K >= 1 && K <= 64, SGW_EINVAL, "K must be in 1..64");
    SGW_REQUIRE(ld_phi >= ctx->N, SGW_EINVAL, "ld_phi < number of grid points");
    SGW_REQUIRE(nsamp >= 0 && first_sample >= 0 && first_sample + nsamp <= ((int64_t)1 << 20),
                SGW_EINVAL, "sample indices must lie in [0, 2^20)");
    SGW_REQUIRE(ctx->N % 64 == 0, SGW_EUNSUPPORTED, "features need N divisible by 64");
    if (nsamp == 0) return;
    features(ctx, phi, K, ld_phi, seed, first_sample, nsamp, x);
  });
}

sgw_status sgw_cv_features_eta(sgw_ctx *ctx, const float *phi, int32_t K, int64_t ld_phi,
                               uint64_t seed, int64_t first_sample, int64_t nsamp,
                               int32_t n_eta, float *x, int64_t ldx) {
  if (!ctx) return SGW_EINVAL;
  return guard_ctx(ctx, [&] {
    SGW_REQUIRE(phi && x, SGW_EINVAL, "NULL argument");
    SGW_REQUIRE(K >= 1 && K <= 64, SGW_EINVAL, "K must be in 1..64");
    SGW_REQUIRE(n_eta >= 1 && n_eta < (1 << 20), SGW_EINVAL, "n_eta must be in 1..2^20-1");
    SGW_REQUIRE(ldx >= K, SGW_EINVAL, "ldx < K");
    SGW_REQUIRE(ld_phi >= ctx->N, SGW_EINVAL, "ld_phi < number of grid points");
    SGW_REQUIRE(nsamp >= 0 && first_sample >= 0 && first_sample + nsamp <= ((int64_t)1 << 20),
                SGW_EINVAL, "sample indices must lie in [0, 2^20)");
    SGW_REQUIRE(ctx->N % 64 == 0, SGW_EUNSUPPORTED, "features need N divisible by 64");
    if (nsamp == 0) return;
    features(ctx, phi, K, ld_phi, seed, first_sample, nsamp, x, n_eta, ldx);
  });
}

sgw_status sgw_mlp_create(int32_t din, int32_t h1, int32_t h2, const double *theta0,
                          void *hip_stream, sgw_mlp **out) {
  if (out) *out = nullptr;
  sgw_mlp *res = nullptr;
  const sgw_status st = guard_mlp(nullptr, [&] {
    SGW_REQUIRE(out && theta0, SGW_EINVAL, "NULL argument");
    SGW_REQUIRE(din >= 1 && h1 >= 1 && h2 >= 1 && din <= 4096 && h1 <= 4096 && h2 <= 4096,
                SGW_EINVAL, "layer sizes must be in 1..4096");
    std::unique_ptr<sgw_mlp> M(new sgw_mlp());
    M->din = din; M->h1 = h1; M->h2 = h2;
    M->stream = static_cast<hipStream_t>(hip_stream);
    M->nparam = M->ob3() + 1;
    std::vector<float> f(M->nparam);
    for (int64_t i = 0; i < M->nparam; ++i) {
      SGW_REQUIRE(std::isfinite(theta0[i]), SGW_EINVAL, "theta0 has a non-finite value");
      f[i] = (float)theta0[i];
    }
    M->theta.ensure(4 * M->nparam);
    M->m.ensure(4 * M->nparam);
    M->v.ensure(4 * M->nparam);
    M->grad.ensure(4 * M->nparam);
    SGW_HIP(hipMemcpy(M->theta.p, f.data(), 4 * M->nparam, hipMemcpyHostToDevice));
    SGW_HIP(hipMemset(M->m.p, 0, 4 * M->nparam));
    SGW_HIP(hipMemset(M->v.p, 0, 4 * M->nparam));
    SGW_HIP(hipMemset(M->grad.p, 0, 4 * M->nparam));
    std::vector<float> zero(din, 0.f), one(din, 1.f);
    M->mean.ensure(4 * din);
    M->inv_std.ensure(4 * din);
    SGW_HIP(hipMemcpy(M->mean.p, zero.data(), 4 * din, hipMemcpyHostToDevice));
    SGW_HIP(hipMemcpy(M->inv_std.p, one.data(), 4 * din, hipMemcpyHostToDevice));
    res = M.release();
  });
  if (st == SGW_OK) *out = res;
  return st;
}

void sgw_mlp_destroy(sgw_mlp *m) { delete m; }

sgw_status sgw_mlp_set_standardization(sgw_mlp *M, const double *mean, const double *std) {
  if (!M) return SGW_EINVAL;
  return guard_mlp(M, [&] {
    SGW_REQUIRE(mean && std, SGW_EINVAL, "NULL argument");
    std::vector<float> mf(M->din), sf(M->din);
    for (int k = 0; k < M->din; ++k) {
      SGW_REQUIRE(std::isfinite(mean[k]) && std[k] > 0 && std::isfinite(std[k]), SGW_EINVAL,
                  "standardization needs finite means and positive deviations");
      mf[k] = (float)mean[k];
      sf[k] = (float)(1.0 / std[k]);
    }
    SGW_HIP(hipMemcpyAsync(M->mean.p, mf.data(), 4 * M->din, hipMemcpyHostToDevice, M->stream));
    SGW_HIP(hipMemcpyAsync(M->inv_std.p, sf.data(), 4 * M->din, hipMemcpyHostToDevice, M->stream));
    SGW_HIP(hipStreamSynchronize(M->stream));
  });
}

sgw_status sgw_mlp_get_params(sgw_mlp *M, double *theta) {
  if (!M) return SGW_EINVAL;
  return guard_mlp(M, [&] {
    SGW_REQUIRE(theta, SGW_EINVAL, "NULL argument");
    std::vector<float> f(M->nparam);
    SGW_HIP(hipMemcpyAsync(f.data(), M->theta.p, 4 * M->nparam, hipMemcpyDeviceToHost, M->stream));
    SGW_HIP(hipStreamSynchronize(M->stream));
    for (int64_t i = 0; i < M->nparam; ++i) theta[i] = f[i];
  });
}

sgw_status sgw_mlp_forward(sgw_mlp *M, const float *x, int64_t n, float *g) {
  if (!M) return SGW_EINVAL;
  return guard_mlp(M, [&] {
    SGW_REQUIRE(x && g, SGW_EINVAL, "NULL argument");
    check_n(n);
    const Acts a = activations(M, n);
    forward(M, x, n, a);
    SGW_HIP(hipMemcpyAsync(g, a.g, 4 * n, hipMemcpyDeviceToDevice, M->stream));
  });
}

sgw_status sgw_mlp_gradient(sgw_mlp *M, const float *x, const float *y, int64_t n, double *loss,
                            double *grad) {
  if (!M) return SGW_EINVAL;
  return guard_mlp(M, [&] {
    SGW_REQUIRE(x && y && loss && grad, SGW_EINVAL, "NULL argument");
    check_n(n);
    const Acts a = activations(M, n);
    double *d_loss = M->buf("loss1", sizeof(double)).as<double>();
    forward(M, x, n, a);
    backward(M, y, n, a, d_loss);
    std::vector<float> f(M->nparam);
    double L = 0;
    SGW_HIP(hipMemcpyAsync(f.data(), M->grad.p, 4 * M->nparam, hipMemcpyDeviceToHost, M->stream));
    SGW_HIP(hipMemcpyAsync(&L, d_loss, sizeof(double), hipMemcpyDeviceToHost, M->stream));
    SGW_HIP(hipStreamSynchronize(M->stream));
    *loss = L / (double)n;
    for (int64_t i = 0; i < M->nparam; ++i) grad[i] = f[i];
  });
}

sgw_status sgw_mlp_adam(sgw_mlp *M, const double *grad, double lr, double b1, double b2,
                        double eps) {
  if (!M) return SGW_EINVAL;
  return guard_mlp(M, [&] {
    SGW_REQUIRE(lr > 0 && b1 >= 0 && b1 < 1 && b2 >= 0 && b2 < 1 && eps > 0, SGW_EINVAL,
                "Adam hyper-parameters out of range");
    if (grad) {
      std::vector<float> f(M->nparam);
      for (int64_t i = 0; i < M->nparam; ++i) f[i] = (float)grad[i];
      SGW_HIP(hipMemcpyAsync(M->grad.p, f.data(), 4 * M->nparam, hipMemcpyHostToDevice,
                             M->stream));
      adam(M, lr, b1, b2, eps);
      SGW_HIP(hipStreamSynchronize(M->stream));
    } else {
      adam(M, lr, b1, b2, eps);
    }
  });
}

sgw_status sgw_mlp_train(sgw_mlp *M, const float *x, const float *y, int64_t n, int32_t steps,
                         double lr, double *loss_hist) {
  if (!M) return SGW_EINVAL;
  return guard_mlp(M, [&] {
    SGW_REQUIRE(x && y, SGW_EINVAL, "NULL argument");
    SGW_REQUIRE(steps >= 0 && lr > 0, SGW_EINVAL, "steps >= 0 and lr > 0 required");
    check_n(n);
    const Acts a = activations(M, n);
    double *d_hist = M->buf("hist", sizeof(double) * std::max(1, (int)steps)).as<double>();
    for (int s = 0; s < steps; ++s) {
      forward(M, x, n, a);
      backward(M, y, n, a, d_hist + s);
      adam(M, lr, 0.9, 0.999, 1e-8);
    }
    if (loss_hist && steps > 0) {
      std::vector<double> h(steps);
      SGW_HIP(hipMemcpyAsync(h.data(), d_hist, sizeof(double) * steps, hipMemcpyDeviceToHost,
                             M->stream));
      SGW_HIP(hipStreamSynchronize(M->stream));
      for (int s = 0; s < steps; ++s) loss_hist[s] = h[s] / (double)n;
    }
  });
}

sgw_status sgw_cv_cheap_moments(sgw_ctx *ctx, sgw_mlp *M, const float *phi, int32_t K,
                                int64_t ld_phi, uint64_t seed, int64_t first_sample, int64_t count,
                                int64_t chunk, double *mean, double *var) {
  if (!ctx || !M) return SGW_EINVAL;
  return guard_ctx(ctx, [&] {
    SGW_REQUIRE(phi && mean && var, SGW_EINVAL, "NULL argument");
    SGW_REQUIRE(K == M->din, SGW_EINVAL, "K must equal the network's input size");
    SGW_REQUIRE(count >= 2 && chunk >= 1, SGW_EINVAL, "count >= 2 and chunk >= 1 required");
    SGW_REQUIRE(first_sample >= 0 && first_sample + count <= ((int64_t)1 << 20), SGW_EINVAL,
                "sample indices must lie in [0, 2^20)");
    SGW_REQUIRE(ctx->N % 64 == 0, SGW_EUNSUPPORTED, "features need N divisible by 64");
    SGW_REQUIRE(ctx->stream == M->stream, SGW_EINVAL, "context and network need one stream");
    chunk = std::min(chunk, count);
    float *xf = ctx->buf("cv_x", sizeof(float) * chunk * K).as<float>();
    const Acts a = activations(M, chunk);
    double *part = ctx->buf("cv_part", sizeof(double) * SUM_BLOCKS).as<double>();
    const int64_t nch = (count + chunk - 1) / chunk;
    double *sums = ctx->buf("cv_sums", sizeof(double) * 2 * nch).as<double>();
    for (int64_t c = 0; c < nch; ++c) {
      const int64_t s0 = first_sample + c * chunk, n = std::min(chunk, count - c * chunk);
      features(ctx, phi, K, ld_phi, seed, s0, n, xf);
      forward(M, xf, n, a);
      dsum<1>(ctx->stream, a.g, nullptr, n, part, sums + 2 * c);
      dsum<2>(ctx->stream, a.g, nullptr, n, part, sums + 2 * c + 1);
    }
    std::vector<double> h(2 * nch);
    SGW_HIP(hipMemcpyAsync(h.data(), sums, sizeof(double) * 2 * nch, hipMemcpyDeviceToHost,
                           ctx->stream));
    SGW_HIP(hipStreamSynchronize(ctx->stream));
    double s1 = 0, s2 = 0;
    for (int64_t c = 0; c < nch; ++c) { s1 += h[2 * c]; s2 += h[2 * c + 1]; }
    const double m = s1 / (double)count;
    *mean = m;
    *var = std::max(0.0, (s2 - (double)count * m * m) / (double)(count - 1));
  });
}

sgw_status sgw_cv_cheap_moments_mixed(sgw_ctx *ctx, sgw_mlp *M, const float *phi_z, int32_t Kz,
                                      const float *phi_e, int32_t Ke, int64_t ld_phi,
                                      uint64_t seed, int32_t n_eta, int64_t first_sample,
                                      int64_t count, int64_t chunk, double *mean, double *var) {
  if (!ctx || !M) return SGW_EINVAL;
  return guard_ctx(ctx, [&] {
    SGW_REQUIRE(mean && var && (Kz == 0 || phi_z) && (Ke == 0 || phi_e), SGW_EINVAL,
                "NULL argument");
    SGW_REQUIRE(Kz >= 0 && Kz <= 64 && Ke >= 0 && Ke <= 64 && Kz + Ke >= 1, SGW_EINVAL,
                "Kz and Ke must be in 0..64, not both 0");
    SGW_REQUIRE(Kz + Ke == M->din, SGW_EINVAL, "Kz + Ke must equal the network's input size");
    SGW_REQUIRE(Ke == 0 || (n_eta >= 1 && n_eta < (1 << 20)), SGW_EINVAL,
                "n_eta must be in 1..2^20-1");
    SGW_REQUIRE(count >= 2 && chunk >= 1, SGW_EINVAL, "count >= 2 and chunk >= 1 required");
    SGW_REQUIRE(ld_phi >= ctx->N, SGW_EINVAL, "ld_phi < number of grid points");
    SGW_REQUIRE(first_sample >= 0 && first_sample + count <= ((int64_t)1 << 20), SGW_EINVAL,
                "sample indices must lie in [0, 2^20)");
    SGW_REQUIRE(ctx->N % 64 == 0, SGW_EUNSUPPORTED, "features need N divisible by 64");
    SGW_REQUIRE(ctx->stream == M->stream, SGW_EINVAL, "context and network need one stream");
    const int K = Kz + Ke;
    chunk = std::min(chunk, count);
    float *xf = ctx->buf("cv_x", sizeof(float) * chunk * K).as<float>();
    const Acts a = activations(M, chunk);
    double *part = ctx->buf("cv_part", sizeof(double) * SUM_BLOCKS).as<double>();
    const int64_t nch = (count + chunk - 1) / chunk;
    double *sums = ctx->buf("cv_sums", sizeof(double) * 2 * nch).as<double>();
    for (int64_t c = 0; c < nch; ++c) {
      const int64_t s0 = first_sample + c * chunk, n = std::min(chunk, count - c * chunk);
      if (Kz > 0) features(ctx, phi_z, Kz, ld_phi, seed, s0, n, xf, 0, K);
      if (Ke > 0) features(ctx, phi_e, Ke, ld_phi, seed, s0, n, xf + Kz, n_eta, K);
      forward(M, xf, n, a);
      dsum<1>(ctx->stream, a.g, nullptr, n, part, sums + 2 * c);
      dsum<2>(ctx->stream, a.g, nullptr, n, part, sums + 2 * c + 1);
    }
    std::vector<double> h(2 * nch);
    SGW_HIP(hipMemcpyAsync(h.data(), sums, sizeof(double) * 2 * nch, hipMemcpyDeviceToHost,
                           ctx->stream));
    SGW_HIP(hipStreamSynchronize(ctx->stream));
    double s1 = 0, s2 = 0;
    for (int64_t c = 0; c < nch; ++c) { s1 += h[2 * c]; s2 += h[2 * c + 1]; }
    const double m = s1 / (double)count;
    *mean = m;
    *var = std::max(0.0, (s2 - (double)count * m * m) / (double)(count - 1));
  });
}

sgw_status sgw_cv_estimate(const double *yA, const double *gA, int64_t nA, const double *yB,
                           const double *gB, int64_t nB, double gM_mean, double gM_var,
                           int64_t M, sgw_cv_result *out) {
  if (!yA || !gA || !yB || !gB || !out || nA < 2 || nB < 2 || M < 2) return SGW_EINVAL;
  if (!std::isfinite(gM_mean) || !(gM_var >= 0)) return SGW_EINVAL;
  auto mean = [](const double *a, int64_t n) {
    double s = 0; for (int64_t i = 0; i < n; ++i) s += a[i]; return s / (double)n;
  };
  const double my = mean(yA, nA), mg = mean(gA, nA);
  double cyg = 0, vg = 0, vy = 0;
  for (int64_t i = 0; i < nA; ++i) {
    cyg += (yA[i] - my) * (gA[i] - mg);
    vg += (gA[i] - mg) * (gA[i] - mg);
    vy += (yA[i] - my) * (yA[i] - my);
  }
  const double c = vg > 0 ? cyg / vg : 0.0;
  double mr = 0;
  for (int64_t i = 0; i < nB; ++i) mr += yB[i] - c * gB[i];
  mr /= (double)nB;
  double vr = 0;
  for (int64_t i = 0; i < nB; ++i) {
    const double d = yB[i] - c * gB[i] - mr;
    vr += d * d;
  }
  vr /= (double)(nB - 1);
  const double est = mr + c * gM_mean;
  const double var_cv = vr / (double)nB + c * c * gM_var / (double)M;
  double sy = 0;
  for (int64_t i = 0; i < nA; ++i) sy += yA[i];
  for (int64_t i = 0; i < nB; ++i) sy += yB[i];
  const int64_t nt = nA + nB;
  const double plain = sy / (double)nt;
  double vp = 0;
  for (int64_t i = 0; i < nA; ++i) vp += (yA[i] - plain) * (yA[i] - plain);
  for (int64_t i = 0; i < nB; ++i) vp += (yB[i] - plain) * (yB[i] - plain);
  const double var_plain = vp / (double)(nt - 1) / (double)nt;
  out->c = c;
  out->rho2 = (vg > 0 && vy > 0) ? cyg * cyg / (vg * vy) : 0.0;
  out->plain = plain;
  out->sigma_plain = std::sqrt(var_plain);
  out->sigma_cv = std::sqrt(var_cv);
  out->fallback = std::fabs(est - plain) > 3.0 * std::sqrt(var_cv + var_plain) ? 1 : 0;
  out->estimate = out->fallback ? plain : est;
  out->sigma = out->fallback ? out->sigma_plain : out->sigma_cv;
  return SGW_OK;
}

}  // extern "C"
