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

__device__ __forceinline__ int64_t tile_point(int base, int p, int nx, int ny) {
  return (int64_t)base + (p & 7) + (int64_t)nx * (((p >> 3) & 7) + (int64_t)ny * (p >> 6));
}

template <typename T> __device__ __forceinline__ T wsum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <typename R>
__global__ __launch_bounds__(NTK) void k_kb_gather(const cplx<R> *psi, int64_t ld, int64_t nvec,
                                                   const int *tile_base, const int *tile_off,
                                                   const R *beta, cplx<R> *partial, int nx,
                                                   int ny, R dV) {
  constexpr int NV = KBV<R>::NV;
  using C = cplx<R>;
  __shared__ C s[KB_TP * NV];
  const int t = blockIdx.y;
  const int64_t v0 = (int64_t)blockIdx.x * NV;
  const int base = tile_base[t];
  for (int idx = threadIdx.x; idx < KB_TP * NV; idx += NTK) {
    const int vl = idx / KB_TP, p = idx % KB_TP;
    C val = cmake<C>(0, 0);
    if (v0 + vl < nvec) val = psi[(v0 + vl) * ld + tile_point(base, p, nx, ny)];
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
                                                    int ny) {
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
    const int64_t r = tile_point(base, p, nx, ny);
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

// ---------------------------------------------------------------- launchers
template <typename R>
static void gather_t(sgw_ctx *ctx, const void *psi, int64_t nvec, int64_t ld, void *out,
                     bool use_e) {
  constexpr int NV = KBV<R>::NV;
  using C = cplx<R>;
  C *partial = ctx->buf("kb_partial", sizeof(C) * (size_t)ctx->kb_nentry * nvec).as<C>();
  const int64_t nvb = (nvec + NV - 1) / NV;
  SGW_REQUIRE(ctx->kb_ntile <= 65535, SGW_EUNSUPPORTED, "KB gather: too many tiles");
  hipLaunchKernelGGL(k_kb_gather<R>, dim3(nvb, ctx->kb_ntile), dim3(NTK), 0, ctx->stream,
                     static_cast<const C *>(psi), ld, nvec, ctx->d_kb_tile_base.as<int>(),
                     ctx->d_kb_tile_off.as<int>(), ctx->d_kb_beta.as<R>(), partial, ctx->nx,
                     ctx->ny, (R)ctx->dV);
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
  const int64_t nvb = (nvec + NV - 1) / NV;
  SGW_REQUIRE(ctx->kb_ntile <= 65535, SGW_EUNSUPPORTED, "KB scatter: too many tiles");
  hipLaunchKernelGGL(k_kb_scatter<R>, dim3(nvb, ctx->kb_ntile), dim3(NTK), 0, ctx->stream,
                     static_cast<const C *>(coef), nvec, ctx->d_kb_tile_base.as<int>(),
                     ctx->d_kb_tile_off.as<int>(), ctx->d_kb_entry_proj.as<int>(),
                     ctx->d_kb_beta.as<R>(), static_cast<C *>(dst), ld, (R)s1re, (R)s1im,
                     static_cast<C *>(dst2), (R)s2re, (R)s2im, ctx->nx, ctx->ny);
  SGW_HIP(hipGetLastError());
}

void kb_scatter(sgw_ctx *ctx, const void *coef, int64_t nvec, void *dst, int64_t ld,
                double s1re, double s1im, void *dst2, double s2re, double s2im) {
  if (ctx->dbl) scatter_t<double>(ctx, coef, nvec, dst, ld, s1re, s1im, dst2, s2re, s2im);
  else scatter_t<float>(ctx, coef, nvec, dst, ld, s1re, s1im, dst2, s2re, s2im);
}

}  // namespace sgw
