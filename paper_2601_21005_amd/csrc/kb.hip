// Kleinman-Bylander projector contraction (the separable pseudopotential
// part, applied in the paper with atomic adds where neighbouring projector
// spheres overlap, Sec. 3).  Here the work is owned by 8x8x8 grid tiles:
//   gather   partial[e][v] = dV sum_{r in tile} beta_e(r) psi_v(r)   per
//            (tile, projector) entry e -- the tile of NV vectors sits in LDS;
//   reduce   C[p][v] = sum of the partials of projector p, in a fixed order
//            (optionally times E_p);
//   mix      C'[p][v] = sum_q K[p][q] C[q][v]  (dense, for exp(-i tau V_NL));
//   scatter  dst_v(r) += s1 sum_e beta_e(r) C'[p(e)][v] on each tile's own
//            points -- every point is written by exactly one workgroup, so
//            no atomics and bitwise reproducible results.
#include "common.h"
#include "kernels.h"

namespace sgw {

constexpr int NTK = 256;
constexpr int KB_MAXE = 256;   // max projector entries per tile

template <typename R> struct KBV;
template <> struct KBV<float> { static constexpr int NV = 8; };
template <> struct KBV<double> { static constexpr int NV = 4; };

// flat grid index of point p of a tile whose x and y extents are 2^lx, 2^ly
__device__ __forceinline__ int64_t tile_point(int base, int p, int nx, int ny, int lx, int ly) {
  const int x = p & ((1 << lx) - 1), y = (p >> lx) & ((1 << ly) - 1), z = p >> (lx + ly);
  return (int64_t)base + x + (int64_t)nx * (y + (int64_t)ny * z);
}

template <typename T> __device__ __forceinline__ T wsum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <typename R>
__global__ __launch_bounds__(NTK) void k_kb_gather(const cplx<R> *psi, int64_t ld, int64_t nvec,
                                                   const int *tile_base, const int *tile_off,
                                                   const R *beta, cplx<R> *partial, int nx,
                                                   int ny, int lx, int ly, R dV) {
  constexpr int NV = KBV<R>::NV;
  using C = cplx<R>;
  __shared__ C s[KB_TP * NV];
  const int t = blockIdx.y;
  const int64_t v0 = (int64_t)blockIdx.x * NV;
  const int base = tile_base[t];
  for (int idx = threadIdx.x; idx < KB_TP * NV; idx += NTK) {
    const int vl = idx / KB_TP, p = idx % KB_TP;
    C val = cmake<C>(0, 0);
    if (v0 + vl < nvec) val = psi[(v0 + vl) * ld + tile_point(base, p, nx, ny, lx, ly)];
    s[p * NV + vl] = val;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e1 = tile_off[t + 1];
  for (int e = tile_off[t] + w; e < e1; e += NTK / 64) {
    R ar[NV], ai[NV];
#pragma unroll
    for (int vl = 0; vl < NV; ++vl) { ar[vl] = 0; ai[vl] = 0; }
    const R *b = beta + (int64_t)e * KB_TP;
#pragma unroll
    for (int q = 0; q < KB_TP / 64; ++q) {
      const int p = lane + 64 * q;
      const R bv = b[p];
#pragma unroll
      for (int vl = 0; vl < NV; ++vl) {
        const C x = s[p * NV + vl];
        ar[vl] += bv * x.x;
        ai[vl] += bv * x.y;
      }
    }
#pragma unroll
    for (int vl = 0; vl < NV; ++vl) {
      ar[vl] = wsum(ar[vl]);
      ai[vl] = wsum(ai[vl]);
    }
    if (lane == 0) {
#pragma unroll
      for (int vl = 0; vl < NV; ++vl)
        if (v0 + vl < nvec) partial[(int64_t)e * nvec + v0 + vl] = cmake<C>(dV * ar[vl], dV * ai[vl]);
    }
  }
}

template <typename R>
__global__ void k_kb_reduce(const cplx<R> *partial, const int *proj_off, const int *proj_entries,
                            const double *ekb, int use_e, int64_t nvec, cplx<R> *out) {
  const int64_t v = (int64_t)blockIdx.x * NTK + threadIdx.x;
  const int p = blockIdx.y;
  if (v >= nvec) return;
  double sr = 0, si = 0;
  for (int k = proj_off[p]; k < proj_off[p + 1]; ++k) {
    const cplx<R> c = partial[(int64_t)proj_entries[k] * nvec + v];
    sr += c.x;
    si += c.y;
  }
  if (use_e) { sr *= ekb[p]; si *= ekb[p]; }
  out[(int64_t)p * nvec + v] = cmake<cplx<R>>(sr, si);
}

template <typename R>
__global__ void k_kb_mix(const cplx<R> *K, const cplx<R> *in, cplx<R> *out, int np,
                         int64_t nvec) {
  const int64_t v = (int64_t)blockIdx.x * NTK + threadIdx.x;
  const int p = blockIdx.y;
  if (v >= nvec) return;
  double sr = 0, si = 0;
  const cplx<R> *k = K + (int64_t)p * np;
  for (int q = 0; q < np; ++q) {
    const cplx<R> a = k[q], b = in[(int64_t)q * nvec + v];
    sr += (double)a.x * b.x - (double)a.y * b.y;
    si += (double)a.x * b.y + (double)a.y * b.x;
  }
  out[(int64_t)p * nvec + v] = cmake<cplx<R>>(sr, si);
}

template <typename R>
__global__ __launch_bounds__(NTK) void k_kb_scatter(const cplx<R> *coef, int64_t nvec,
                                                    const int *tile_base, const int *tile_off,
                                                    const int *entry_proj, const R *beta,
                                                    cplx<R> *dst, int64_t ld, R s1r, R s1i,
                                                    cplx<R> *dst2, R s2r, R s2i, int nx,
                                                    int ny, int lx, int ly) {
  constexpr int NV = KBV<R>::NV;
  using C = cplx<R>;
  __shared__ C c[KB_MAXE * NV];
  const int t = blockIdx.y;
  const int64_t v0 = (int64_t)blockIdx.x * NV;
  const int off = tile_off[t], ne = tile_off[t + 1] - off;
  const int base = tile_base[t];
  for (int idx = threadIdx.x; idx < ne * NV; idx += NTK) {
    const int el = idx / NV, vl = idx % NV;
    C val = cmake<C>(0, 0);
    if (v0 + vl < nvec) val = coef[(int64_t)entry_proj[off + el] * nvec + v0 + vl];
    c[idx] = val;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < KB_TP; p += NTK) {
    R ar[NV], ai[NV];
#pragma unroll
    for (int vl = 0; vl < NV; ++vl) { ar[vl] = 0; ai[vl] = 0; }
    for (int el = 0; el < ne; ++el) {
      const R bv = beta[(int64_t)(off + el) * KB_TP + p];
#pragma unroll
      for (int vl = 0; vl < NV; ++vl) {
        const C x = c[el * NV + vl];
        ar[vl] += bv * x.x;
        ai[vl] += bv * x.y;
      }
    }
    const int64_t r = tile_point(base, p, nx, ny, lx, ly);
#pragma unroll
    for (int vl = 0; vl < NV; ++vl) {
      if (v0 + vl >= nvec) break;
      C *d = dst + (v0 + vl) * ld + r;
      C o = *d;
      o.x += s1r * ar[vl] - s1i * ai[vl];
      o.y += s1r * ai[vl] + s1i * ar[vl];
      *d = o;
      if (dst2) {
        C *d2 = dst2 + (v0 + vl) * ld + r;
        C o2 = *d2;
        o2.x += s2r * ar[vl] - s2i * ai[vl];
        o2.y += s2r * ai[vl] + s2i * ar[vl];
        *d2 = o2;
      }
    }
  }
}

// ---------------------------------------------------------------- MFMA (FP32)
// Per tile the gather is the GEMM  C[e][j] = sum_p beta[e][p] Psi[p][j]
// (M = projector entries, K = 512 points, N = 2 NVB real columns = NVB
// complex vectors) and the scatter  D[p][j] = sum_e beta[e][p] C'[e][j]
// (M = 512 points, K = entries).  Both run on v_mfma_f32_16x16x4f32: lane l
// supplies A[l % 16][k] and B[k][l % 16] for the lane's K slot k, and holds
// D[4 (l / 16) + r][l % 16] in accumulator register r.  Within a group of 4
// MFMA steps lane l takes the K slots 4 (l / 16) + s, s = 0..3, so that its
// four A values are 16 contiguous bytes.  The four waves of a workgroup split
// K (the gather: 128 points each, summed in wave order) or M (the scatter), so
// every variant below adds the same products in the same order: the choice of
// NVB and MT changes the speed, not a single bit of the result.
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int NVB, int MT>
__global__ __launch_bounds__(NTK) void k_kb_gather_mfma(
    const float2 *psi, int64_t ld, int64_t nvec, const int *tile_base, const int *tile_off,
    const float *beta, float2 *partial, int nx, int ny, int lx, int ly, float dV) {
  constexpr int COLS = 2 * NVB + 1, NTL = NVB / 8;   // padded pitch: no bank conflicts
  static_assert(4 * MT * NTL * 256 <= KB_TP * COLS, "reduction buffer exceeds the Psi tile");
  __shared__ float sp[KB_TP * COLS];               // Psi tile [p][j], then the reduction
  const int t = blockIdx.y;
  const int64_t v0 = (int64_t)blockIdx.x * NVB;
  const int base = tile_base[t];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int off = tile_off[t], ne = tile_off[t + 1] - off;
  const int q = lane >> 4, col = lane & 15;
  for (int mg = 0; mg < ne; mg += 16 * MT) {
    for (int idx = tid; idx < KB_TP * NVB; idx += NTK) {
      const int vl = idx / KB_TP, p = idx % KB_TP;
      float2 val = make_float2(0.f, 0.f);
      if (v0 + vl < nvec) val = psi[(v0 + vl) * ld + tile_point(base, p, nx, ny, lx, ly)];
      sp[p * COLS + 2 * vl] = val.x;
      sp[p * COLS + 2 * vl + 1] = val.y;
    }
    __syncthreads();
    f32x4 acc[MT][NTL];
#pragma unroll
    for (int j = 0; j < MT; ++j)
#pragma unroll
      for (int n = 0; n < NTL; ++n) acc[j][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 128 * w; k0 < 128 * w + 128; k0 += 16) {
      const int kq = k0 + 4 * q;                     // this lane's 4 K slots
      float b[NTL][4];
#pragma unroll
      for (int n = 0; n < NTL; ++n)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) b[n][s4] = sp[(kq + s4) * COLS + 16 * n + col];
#pragma unroll
      for (int j = 0; j < MT; ++j) {
        if (mg + 16 * j < ne) {
          const int e = mg + 16 * j + col;           // A row = lane % 16
          f32x4 a = f32x4{0.f, 0.f, 0.f, 0.f};
          if (e < ne) a = *reinterpret_cast<const f32x4 *>(beta + (int64_t)(off + e) * KB_TP + kq);
#pragma unroll
          for (int n = 0; n < NTL; ++n)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
              acc[j][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s4], b[n][s4], acc[j][n], 0, 0, 0);
        }
      }
    }
    __syncthreads();                                 // every wave is done with Psi
    float *red = sp;                                 // [w][j][n][lane][4]
#pragma unroll
    for (int j = 0; j < MT; ++j)
#pragma unroll
      for (int n = 0; n < NTL; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          red[(((w * MT + j) * NTL + n) * 64 + lane) * 4 + r] = acc[j][n][r];
    __syncthreads();
    for (int o = tid; o < MT * NTL * 256; o += NTK) {
      const int jn = o / 256, l = (o / 4) % 64, r = o % 4;
      const int j = jn / NTL, n = jn % NTL;
      const int e = mg + 16 * j + 4 * (l >> 4) + r;  // D row
      const int c = 16 * n + (l & 15);               // D column
      float sum = 0.f;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) sum += red[(((ww * MT + j) * NTL + n) * 64 + l) * 4 + r];
      const int vl = c >> 1;
      if (e < ne && v0 + vl < nvec)
        reinterpret_cast<float *>(partial + (int64_t)(off + e) * nvec + v0 + vl)[c & 1] = dV * sum;
    }
    __syncthreads();
  }
}

// dst_v(r) += s1 * sum_e beta_e(r) C[p(e)][v]  (s1 real)
template <int NVB>
__global__ __launch_bounds__(NTK) void k_kb_scatter_mfma(
    const float2 *coef, int64_t nvec, const int *tile_base, const int *tile_off,
    const int *entry_proj, const float *beta, float2 *dst, int64_t ld, float s1, int nx,
    int ny, int lx, int ly) {
  constexpr int COLS = 2 * NVB + 1, NTL = NVB / 8;
  constexpr int SC = KB_MAXE * COLS > KB_TP * COLS ? KB_MAXE * COLS : KB_TP * COLS;
  __shared__ float sm[SC];                         // C' [e][j], then D staging [p][j]
  const int t = blockIdx.y;
  const int64_t v0 = (int64_t)blockIdx.x * NVB;
  const int off = tile_off[t], ne = tile_off[t + 1] - off;
  const int nek = (ne + 3) & ~3;                   // K padded to the MFMA step
  const int base = tile_base[t];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int idx = tid; idx < nek * NVB; idx += NTK) {
    const int el = idx / NVB, vl = idx % NVB;
    float2 val = make_float2(0.f, 0.f);
    if (el < ne && v0 + vl < nvec) val = coef[(int64_t)entry_proj[off + el] * nvec + v0 + vl];
    sm[el * COLS + 2 * vl] = val.x;
    sm[el * COLS + 2 * vl + 1] = val.y;
  }
  __syncthreads();
  const int q = lane >> 4, col = lane & 15;
  // wave w: M tiles (16 points each) 8 w .. 8 w + 7
  f32x4 acc[8][NTL];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int n = 0; n < NTL; ++n) acc[j][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  // K loop with the next step's operands loaded ahead of this step's MFMAs
  float a_cur[8], a_nxt[8], b_cur[NTL], b_nxt[NTL];
  auto load_step = [&](int k0, float *a, float *b) {
    const int e = k0 + q;                          // this lane's K slot
#pragma unroll
    for (int n = 0; n < NTL; ++n) b[n] = sm[e * COLS + 16 * n + col];
    const float *brow = beta + (int64_t)(off + (e < ne ? e : 0)) * KB_TP;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = e < ne ? brow[16 * (8 * w + j) + col] : 0.f;  // A row = point
  };
  load_step(0, a_cur, b_cur);
  for (int k0 = 0; k0 < nek; k0 += 4) {
    if (k0 + 4 < nek) load_step(k0 + 4, a_nxt, b_nxt);
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int n = 0; n < NTL; ++n)
        acc[j][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_cur[j], b_cur[n], acc[j][n], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 8; ++j) a_cur[j] = a_nxt[j];
#pragma unroll
    for (int n = 0; n < NTL; ++n) b_cur[n] = b_nxt[n];
  }
  __syncthreads();                                 // C' no longer needed
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int n = 0; n < NTL; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = 16 * (8 * w + j) + 4 * q + r;
        sm[p * COLS + 16 * n + col] = acc[j][n][r];
      }
  __syncthreads();
  for (int idx = tid; idx < KB_TP * NVB; idx += NTK) {
    const int vl = idx / KB_TP, p = idx % KB_TP;
    if (v0 + vl >= nvec) continue;
    float2 *d = dst + (v0 + vl) * ld + tile_point(base, p, nx, ny, lx, ly);
    float2 o = *d;
    o.x += s1 * sm[p * COLS + 2 * vl];
    o.y += s1 * sm[p * COLS + 2 * vl + 1];
    *d = o;
  }
}

// variants (autotuned per context and batch size)
struct GatherVariant { int nvb, mt; };
static const GatherVariant kGather[] = {{8, 2}, {8, 4}, {8, 8}, {16, 2}, {16, 4}, {16, 8}};
static const int kScatterNvb[] = {8, 16};
constexpr int NGATHER = 6, NSCATTER = 2;

static void launch_gather_variant(int vi, dim3 g, hipStream_t st, const float2 *psi, int64_t ld,
                                  int64_t nvec, const int *tb, const int *to, const float *beta,
                                  float2 *partial, int nx, int ny, int lx, int ly, float dV) {
  switch (vi) {
#define SGW_G(I, A, B) case I: hipLaunchKernelGGL((k_kb_gather_mfma<A, B>), g, dim3(NTK), 0, st, psi, ld, nvec, tb, to, beta, partial, nx, ny, lx, ly, dV); break;
    SGW_G(0, 8, 2) SGW_G(1, 8, 4) SGW_G(2, 8, 8) SGW_G(3, 16, 2) SGW_G(4, 16, 4) SGW_G(5, 16, 8)
#undef SGW_G
  }
}

static void launch_scatter_variant(int vi, dim3 g, hipStream_t st, const float2 *coef,
                                   int64_t nvec, const int *tb, const int *to, const int *ep,
                                   const float *beta, float2 *dst, int64_t ld, float s1, int nx,
                                   int ny, int lx, int ly) {
  if (vi == 0)
    hipLaunchKernelGGL((k_kb_scatter_mfma<8>), g, dim3(NTK), 0, st, coef, nvec, tb, to, ep, beta,
                       dst, ld, s1, nx, ny, lx, ly);
  else
    hipLaunchKernelGGL((k_kb_scatter_mfma<16>), g, dim3(NTK), 0, st, coef, nvec, tb, to, ep, beta,
                       dst, ld, s1, nx, ny, lx, ly);
}

// ---------------------------------------------------------------- launchers
template <typename R>
static void gather_t(sgw_ctx *ctx, const void *psi, int64_t nvec, int64_t ld, void *out,
                     bool use_e) {
  constexpr int NV = KBV<R>::NV;
  using C = cplx<R>;
  C *partial = ctx->buf("kb_partial", sizeof(C) * (size_t)ctx->kb_nentry * nvec).as<C>();
  SGW_REQUIRE(ctx->kb_ntile <= 65535, SGW_EUNSUPPORTED, "KB gather: too many tiles");
  if constexpr (sizeof(R) == 4) {
    auto run = [&](int vi) {
      const int64_t nvb = (nvec + kGather[vi].nvb - 1) / kGather[vi].nvb;
      launch_gather_variant(vi, dim3(nvb, ctx->kb_ntile), ctx->stream,
                            static_cast<const float2 *>(psi), ld, nvec,
                            ctx->d_kb_tile_base.as<int>(), ctx->d_kb_tile_off.as<int>(),
                            ctx->d_kb_beta.as<float>(), reinterpret_cast<float2 *>(partial),
                            ctx->nx, ctx->ny, ctx->kb_lx, ctx->kb_ly, (float)ctx->dV);
    };
    run(ctx->tune("kb_gather", nvec, NGATHER, run));   // the gather overwrites: trials are harmless
  } else {
    const int64_t nvb = (nvec + NV - 1) / NV;
    hipLaunchKernelGGL(k_kb_gather<R>, dim3(nvb, ctx->kb_ntile), dim3(NTK), 0, ctx->stream,
                       static_cast<const C *>(psi), ld, nvec, ctx->d_kb_tile_base.as<int>(),
                       ctx->d_kb_tile_off.as<int>(), ctx->d_kb_beta.as<R>(), partial, ctx->nx,
                       ctx->ny, ctx->kb_lx, ctx->kb_ly, (R)ctx->dV);
  }
  SGW_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_kb_reduce<R>, dim3((nvec + NTK - 1) / NTK, ctx->kb.nproj), dim3(NTK), 0,
                     ctx->stream, partial, ctx->d_kb_proj_off.as<int>(),
                     ctx->d_kb_proj_entries.as<int>(), ctx->d_kb_ekb.as<double>(), use_e ? 1 : 0,
                     nvec, static_cast<C *>(out));
  SGW_HIP(hipGetLastError());
}

void kb_gather(sgw_ctx *ctx, const void *psi, int64_t nvec, int64_t ld, void *coef_out) {
  if (ctx->dbl) gather_t<double>(ctx, psi, nvec, ld, coef_out, false);
  else gather_t<float>(ctx, psi, nvec, ld, coef_out, false);
}

void kb_gather_e(sgw_ctx *ctx, const void *psi, int64_t nvec, int64_t ld, void *coef_out) {
  if (ctx->dbl) gather_t<double>(ctx, psi, nvec, ld, coef_out, true);
  else gather_t<float>(ctx, psi, nvec, ld, coef_out, true);
}

void kb_mix_dense(sgw_ctx *ctx, const void *K, const void *coef_in, void *coef_out,
                  int64_t nvec) {
  const dim3 g((nvec + NTK - 1) / NTK, ctx->kb.nproj);
  if (ctx->dbl)
    hipLaunchKernelGGL(k_kb_mix<double>, g, dim3(NTK), 0, ctx->stream,
                       static_cast<const double2 *>(K), static_cast<const double2 *>(coef_in),
                       static_cast<double2 *>(coef_out), ctx->kb.nproj, nvec);
  else
    hipLaunchKernelGGL(k_kb_mix<float>, g, dim3(NTK), 0, ctx->stream,
                       static_cast<const float2 *>(K), static_cast<const float2 *>(coef_in),
                       static_cast<float2 *>(coef_out), ctx->kb.nproj, nvec);
  SGW_HIP(hipGetLastError());
}

template <typename R>
static void scatter_t(sgw_ctx *ctx, const void *coef, int64_t nvec, void *dst, int64_t ld,
                      double s1re, double s1im, void *dst2, double s2re, double s2im) {
  constexpr int NV = KBV<R>::NV;
  using C = cplx<R>;
  SGW_REQUIRE(ctx->kb_ntile <= 65535, SGW_EUNSUPPORTED, "KB scatter: too many tiles");
  if constexpr (sizeof(R) == 4) {
    if (dst2 == nullptr && s1im == 0.0) {
      auto run = [&](int vi) {
        const int64_t nvb = (nvec + kScatterNvb[vi] - 1) / kScatterNvb[vi];
        launch_scatter_variant(vi, dim3(nvb, ctx->kb_ntile), ctx->stream,
                               static_cast<const float2 *>(coef), nvec,
                               ctx->d_kb_tile_base.as<int>(), ctx->d_kb_tile_off.as<int>(),
                               ctx->d_kb_entry_proj.as<int>(), ctx->d_kb_beta.as<float>(),
                               static_cast<float2 *>(dst), ld, (float)s1re, ctx->nx, ctx->ny,
                               ctx->kb_lx, ctx->kb_ly);
      };
      // trials add 0 * (B C) to dst, which leaves it unchanged
      const int vi = ctx->tune("kb_scatter", nvec, NSCATTER, [&](int i) {
        const int64_t nvb = (nvec + kScatterNvb[i] - 1) / kScatterNvb[i];
        launch_scatter_variant(i, dim3(nvb, ctx->kb_ntile), ctx->stream,
                               static_cast<const float2 *>(coef), nvec,
                               ctx->d_kb_tile_base.as<int>(), ctx->d_kb_tile_off.as<int>(),
                               ctx->d_kb_entry_proj.as<int>(), ctx->d_kb_beta.as<float>(),
                               static_cast<float2 *>(dst), ld, 0.0f, ctx->nx, ctx->ny,
                               ctx->kb_lx, ctx->kb_ly);
      });
      run(vi);
      SGW_HIP(hipGetLastError());
      return;
    }
  }
  const int64_t nvb = (nvec + NV - 1) / NV;
  hipLaunchKernelGGL(k_kb_scatter<R>, dim3(nvb, ctx->kb_ntile), dim3(NTK), 0, ctx->stream,
                     static_cast<const C *>(coef), nvec, ctx->d_kb_tile_base.as<int>(),
                     ctx->d_kb_tile_off.as<int>(), ctx->d_kb_entry_proj.as<int>(),
                     ctx->d_kb_beta.as<R>(), static_cast<C *>(dst), ld, (R)s1re, (R)s1im,
                     static_cast<C *>(dst2), (R)s2re, (R)s2im, ctx->nx, ctx->ny, ctx->kb_lx,
                     ctx->kb_ly);
  SGW_HIP(hipGetLastError());
}

void kb_scatter(sgw_ctx *ctx, const void *coef, int64_t nvec, void *dst, int64_t ld,
                double s1re, double s1im, void *dst2, double s2re, double s2im) {
  if (ctx->dbl) scatter_t<double>(ctx, coef, nvec, dst, ld, s1re, s1im, dst2, s2re, s2im);
  else scatter_t<float>(ctx, coef, nvec, dst, ld, s1re, s1im, dst2, s2re, s2im);
}

}  // namespace sgw
