// Elementwise, reduction, TDH and sROI kernels.
#include "fft_lds.h"
#include "kernels.h"
#include "rng.h"

namespace sgw {

constexpr int NT = 256;

static inline dim3 grid1(int64_t n, int64_t y = 1) {
  return dim3((unsigned)((n + NT - 1) / NT), (unsigned)y);
}

// ============================================================ vectors
template <typename R>
__global__ void k_scale_copy(const cplx<R> *x, int64_t ldx, cplx<R> *acc, int64_t lda,
                             int64_t N, R cre, R cim) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (r >= N) return;
  const cplx<R> a = x[v * ldx + r];
  cplx<R> o;
  o.x = cre * a.x - cim * a.y;
  o.y = cre * a.y + cim * a.x;
  acc[v * lda + r] = o;
}

void launch_scale_copy(sgw_ctx *ctx, const void *x, int64_t ldx, void *acc, int64_t lda,
                       int64_t nvec, double cre, double cim) {
  for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
    const int64_t nv = std::min<int64_t>(65535, nvec - v0);
    if (ctx->dbl)
      hipLaunchKernelGGL(k_scale_copy<double>, grid1(ctx->N, nv), dim3(NT), 0, ctx->stream,
                         static_cast<const double2 *>(x) + v0 * ldx, ldx,
                         static_cast<double2 *>(acc) + v0 * lda, lda, ctx->N, cre, cim);
    else
      hipLaunchKernelGGL(k_scale_copy<float>, grid1(ctx->N, nv), dim3(NT), 0, ctx->stream,
                         static_cast<const float2 *>(x) + v0 * ldx, ldx,
                         static_cast<float2 *>(acc) + v0 * lda, lda, ctx->N, (float)cre,
                         (float)cim);
  }
  SGW_HIP(hipGetLastError());
}

template <typename R>
__global__ void k_axpy(const cplx<R> *x, int64_t ldx, cplx<R> *acc, int64_t lda, int64_t N,
                       R cre, R cim) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (r >= N) return;
  const cplx<R> a = x[v * ldx + r];
  cplx<R> o = acc[v * lda + r];
  o.x += cre * a.x - cim * a.y;
  o.y += cre * a.y + cim * a.x;
  acc[v * lda + r] = o;
}

void launch_axpy(sgw_ctx *ctx, const void *x, int64_t ldx, void *acc, int64_t lda,
                 int64_t nvec, double cre, double cim) {
  for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
    const int64_t nv = std::min<int64_t>(65535, nvec - v0);
    if (ctx->dbl)
      hipLaunchKernelGGL(k_axpy<double>, grid1(ctx->N, nv), dim3(NT), 0, ctx->stream,
                         static_cast<const double2 *>(x) + v0 * ldx, ldx,
                         static_cast<double2 *>(acc) + v0 * lda, lda, ctx->N, cre, cim);
    else
      hipLaunchKernelGGL(k_axpy<float>, grid1(ctx->N, nv), dim3(NT), 0, ctx->stream,
                         static_cast<const float2 *>(x) + v0 * ldx, ldx,
                         static_cast<float2 *>(acc) + v0 * lda, lda, ctx->N, (float)cre,
                         (float)cim);
  }
  SGW_HIP(hipGetLastError());
}

// acc (= when assign, else +=) c0 a + c1 b, in that order
template <typename R>
__global__ void k_axpy2(const cplx<R> *a, const cplx<R> *b, int64_t ld, cplx<R> *acc, int64_t N,
                        R c0r, R c0i, R c1r, R c1i, int assign) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (r >= N) return;
  const cplx<R> x = a[v * ld + r], y = b[v * ld + r];
  cplx<R> o;
  o.x = o.y = 0;
  if (!assign) o = acc[v * ld + r];
  o.x += c0r * x.x - c0i * x.y;
  o.y += c0r * x.y + c0i * x.x;
  o.x += c1r * y.x - c1i * y.y;
  o.y += c1r * y.y + c1i * y.x;
  acc[v * ld + r] = o;
}

void launch_axpy2(sgw_ctx *ctx, const void *a, const void *b, int64_t ld, void *acc,
                  int64_t nvec, double c0r, double c0i, double c1r, double c1i, bool assign) {
  for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
    const int64_t nv = std::min<int64_t>(65535, nvec - v0);
    if (ctx->dbl)
      hipLaunchKernelGGL(k_axpy2<double>, grid1(ctx->N, nv), dim3(NT), 0, ctx->stream,
                         static_cast<const double2 *>(a) + v0 * ld,
                         static_cast<const double2 *>(b) + v0 * ld, ld,
                         static_cast<double2 *>(acc) + v0 * ld, ctx->N, c0r, c0i, c1r, c1i,
                         assign ? 1 : 0);
    else
      hipLaunchKernelGGL(k_axpy2<float>, grid1(ctx->N, nv), dim3(NT), 0, ctx->stream,
                         static_cast<const float2 *>(a) + v0 * ld,
                         static_cast<const float2 *>(b) + v0 * ld, ld,
                         static_cast<float2 *>(acc) + v0 * ld, ctx->N, (float)c0r, (float)c0i,
                         (float)c1r, (float)c1i, assign ? 1 : 0);
  }
  SGW_HIP(hipGetLastError());
}

// Several Chebyshev sums over one recurrence: acc_g (= when assign, else +=)
// sum_j c_g,j x_j for g < G over a group of nterm terms, added in order of j.
// The group's terms are read once (all loads first) for all G accumulators,
// which are G-major, acc + (g nvec + v) N.
template <typename R>
__global__ void k_cheb_accs(ChebAccTerms t, int nterm, cplx<R> *acc, int64_t N, int64_t nvec,
                            int G, int assign) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (r >= N) return;
  cplx<R> x[kSweepGroup];
#pragma unroll
  for (int j = 0; j < kSweepGroup; ++j)
    if (j < nterm) x[j] = static_cast<const cplx<R> *>(t.x[j])[v * N + r];
#pragma unroll
  for (int g = 0; g < kMaxSweep; ++g) {
    if (g < G) {
      cplx<R> *o = acc + ((int64_t)g * nvec + v) * N + r;
      cplx<R> s;
      s.x = s.y = 0;
      if (!assign) s = *o;
#pragma unroll
      for (int j = 0; j < kSweepGroup; ++j) {
        if (j < nterm) {
          const R cr = (R)t.c[g][2 * j], ci = (R)t.c[g][2 * j + 1];
          s.x += cr * x[j].x - ci * x[j].y;
          s.y += cr * x[j].y + ci * x[j].x;
        }
      }
      *o = s;
    }
  }
}

void launch_cheb_accs(sgw_ctx *ctx, const ChebAccTerms &t, int nterm, void *acc, int64_t nvec,
                      int G, bool assign) {
  SGW_REQUIRE(G >= 1 && G <= kMaxSweep && nterm >= 0 && nterm <= kSweepGroup && nvec <= 65535,
              SGW_EINVAL, "cheb_accs: bad sizes");
  if (nvec == 0) return;
  if (ctx->dbl)
    hipLaunchKernelGGL(k_cheb_accs<double>, grid1(ctx->N, nvec), dim3(NT), 0, ctx->stream, t,
                       nterm, static_cast<double2 *>(acc), ctx->N, nvec, G, assign ? 1 : 0);
  else
    hipLaunchKernelGGL(k_cheb_accs<float>, grid1(ctx->N, nvec), dim3(NT), 0, ctx->stream, t,
                       nterm, static_cast<float2 *>(acc), ctx->N, nvec, G, assign ? 1 : 0);
  SGW_HIP(hipGetLastError());
}

void launch_copy(sgw_ctx *ctx, const void *src, int64_t lds, void *dst, int64_t ldd,
                 int64_t nvec) {
  SGW_HIP(hipMemcpy2DAsync(dst, ldd * ctx->csize(), src, lds * ctx->csize(),
                           ctx->N * ctx->csize(), nvec, hipMemcpyDeviceToDevice,
                           ctx->stream));
}

// ============================================================ reductions
// Two-stage deterministic sums in FP64: stage 1 writes one partial per
// (item, block of RCHUNK points) from a fixed-order LDS tree, stage 2 adds
// the partials of each item in order.
constexpr int RCHUNK = NT * 16;

__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

enum RedOp { RED_NORM2 = 0, RED_REDOT = 1 };

template <typename R, int OP>
__global__ void k_reduce1(const cplx<R> *a, const cplx<R> *b, int64_t ld, int64_t N,
                          double *partial, int nblk) {
  __shared__ double sh[NT];
  const int64_t item = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * RCHUNK;
  const int64_t r1 = std::min<int64_t>(N, r0 + RCHUNK);
  double acc = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += NT) {
    const cplx<R> x = a[item * ld + r];
    if (OP == RED_NORM2) {
      acc += (double)x.x * x.x + (double)x.y * x.y;
    } else {
      const cplx<R> y = b[item * ld + r];
      acc += (double)x.x * y.x + (double)x.y * y.y;
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[item * nblk + blockIdx.x] = s;
}

__global__ void k_reduce2(const double *partial, int nblk, int64_t nitems, double *out) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= nitems) return;
  double s = 0;
  for (int k = 0; k < nblk; ++k) s += partial[i * nblk + k];
  out[i] = s;
}

template <int OP>
static void reduce(sgw_ctx *ctx, const void *a, const void *b, int64_t ld, int64_t n,
                   double *d_out) {
  const int nblk = (int)((ctx->N + RCHUNK - 1) / RCHUNK);
  double *partial = ctx->buf("red_partial", sizeof(double) * nblk * std::max<int64_t>(n, 1)).as<double>();
  for (int64_t v0 = 0; v0 < n; v0 += 65535) {
    const int64_t nv = std::min<int64_t>(65535, n - v0);
    if (ctx->dbl)
      hipLaunchKernelGGL((k_reduce1<double, OP>), dim3(nblk, nv), dim3(NT), 0, ctx->stream,
                         static_cast<const double2 *>(a) + v0 * ld,
                         b ? static_cast<const double2 *>(b) + v0 * ld : nullptr, ld, ctx->N,
                         partial + v0 * nblk, nblk);
    else
      hipLaunchKernelGGL((k_reduce1<float, OP>), dim3(nblk, nv), dim3(NT), 0, ctx->stream,
                         static_cast<const float2 *>(a) + v0 * ld,
                         b ? static_cast<const float2 *>(b) + v0 * ld : nullptr, ld, ctx->N,
                         partial + v0 * nblk, nblk);
  }
  hipLaunchKernelGGL(k_reduce2, grid1(n), dim3(NT), 0, ctx->stream, partial, nblk, n, d_out);
  SGW_HIP(hipGetLastError());
}

void launch_norm2(sgw_ctx *ctx, const void *x, int64_t ld, int64_t nvec, double *d_out) {
  reduce<RED_NORM2>(ctx, x, nullptr, ld, nvec, d_out);
}
void launch_redot(sgw_ctx *ctx, const void *a, const void *b, int64_t ld, int64_t nf,
                  double *d_out) {
  reduce<RED_REDOT>(ctx, a, b, ld, nf, d_out);
}

// ============================================================ white noise
template <typename R>
__global__ void k_fill_noise(const uint64_t *keys, int64_t nr, int64_t N, R amp,
                             cplx<R> *out) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t k = blockIdx.y;
  if (r >= N) return;
  cplx<R> o;
  o.x = noise_bit(keys[2 * k], r) ? -amp : amp;
  o.y = (2 * k + 1 < nr) ? (noise_bit(keys[2 * k + 1], r) ? -amp : amp) : (R)0;
  out[k * N + r] = o;
}

void launch_fill_noise(sgw_ctx *ctx, const uint64_t *d_keys, int64_t nr, void *out) {
  const int64_t nc = (nr + 1) / 2;
  const double amp = 1.0 / std::sqrt(ctx->dV);
  for (int64_t k0 = 0; k0 < nc; k0 += 65535) {
    const int64_t nk = std::min<int64_t>(65535, nc - k0);
    if (ctx->dbl)
      hipLaunchKernelGGL(k_fill_noise<double>, grid1(ctx->N, nk), dim3(NT), 0, ctx->stream,
                         d_keys + 2 * k0, nr - 2 * k0, ctx->N, amp,
                         static_cast<double2 *>(out) + k0 * ctx->N);
    else
      hipLaunchKernelGGL(k_fill_noise<float>, grid1(ctx->N, nk), dim3(NT), 0, ctx->stream,
                         d_keys + 2 * k0, nr - 2 * k0, ctx->N, (float)amp,
                         static_cast<float2 *>(out) + k0 * ctx->N);
  }
  SGW_HIP(hipGetLastError());
}

template <typename R>
__device__ __forceinline__ R real_component(const cplx<R> *filt, int64_t q, int64_t N,
                                            int64_t r) {
  const cplx<R> c = filt[(q >> 1) * N + r];
  return (q & 1) ? c.y : c.x;
}

template <typename R>
__global__ void k_unpack(UnpackArgs a, int64_t N, R amp) {
  using C = cplx<R>;
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t s = blockIdx.y;
  if (r >= N) return;
  const C *filt = static_cast<const C *>(a.filt);
  const int64_t q0 = s * (1 + a.neta);
  const R zocc = real_component<R>(filt, q0, N, r);
  const R zb = noise_bit(a.keys[q0], r) ? -amp : amp;
  const R ph = static_cast<const R *>(a.phi)[r];
  if (a.zeta) {
    C *zeta = static_cast<C *>(a.zeta) + s * 2 * N;
    zeta[r] = cmake<C>(zb - zocc, 0);
    zeta[N + r] = cmake<C>(zocc, 0);
  }
  static_cast<C *>(a.kick)[s * N + r] = cmake<C>(ph * zb, 0);
  const int64_t lp = a.ldp > 0 ? a.ldp : N;
  C *psi = a.psi ? static_cast<C *>(a.psi) + s * a.ncopy * a.neta * lp : nullptr;
  C *xs = static_cast<C *>(a.xsrc) + s * (a.neta / 2) * N;
  for (int l = 0; l < a.neta; l += 2) {
    const R e0 = real_component<R>(filt, q0 + 1 + l, N, r);
    const R e1 = real_component<R>(filt, q0 + 2 + l, N, r);
    if (psi) {
      psi[(int64_t)l * lp + r] = cmake<C>(e0, 0);
      psi[(int64_t)(l + 1) * lp + r] = cmake<C>(e1, 0);
    }
    xs[(int64_t)(l / 2) * N + r] = cmake<C>(ph * e0, ph * e1);
  }
}

void launch_unpack(sgw_ctx *ctx, const UnpackArgs &a) {
  const double amp = 1.0 / std::sqrt(ctx->dV);
  if (ctx->dbl)
    hipLaunchKernelGGL(k_unpack<double>, grid1(ctx->N, a.S), dim3(NT), 0, ctx->stream, a,
                       ctx->N, amp);
  else
    hipLaunchKernelGGL(k_unpack<float>, grid1(ctx->N, a.S), dim3(NT), 0, ctx->stream, a,
                       ctx->N, (float)amp);
  SGW_HIP(hipGetLastError());
}

// ============================================================ TDH
// A sample's block holds 1 + K copies of its N_eta orbitals, psi[s][c][l]
// (vectors ld apart): c = 0 the unperturbed eta, c = 1 + k the tangent
// delta-eta of state k, whose response field is u[k][s].  K = 1 is the
// single-state layout.

// psi[s][1 + k][l] = -i dv[k][s] psi[s][0][l]
template <typename R>
__global__ void k_tdh_tangent(cplx<R> *psi, const R *dv, int neta, int nk, int64_t N,
                              int64_t ld) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t s = blockIdx.y, S = gridDim.y;
  if (r >= N) return;
  cplx<R> *p0 = psi + s * (1 + nk) * neta * ld;
  for (int k = 0; k < nk; ++k) {
    const R d = dv[(k * S + s) * N + r];
    cplx<R> *p1 = p0 + (int64_t)(1 + k) * neta * ld;
    for (int l = 0; l < neta; ++l) {
      const cplx<R> e = p0[(int64_t)l * ld + r];
      p1[(int64_t)l * ld + r] = cmake<cplx<R>>(d * e.y, -d * e.x);
    }
  }
}

// Local step of length a:  eta <- e^{-i V a} eta,
// delta-eta_k <- e^{-i V a} (delta-eta_k - i a u_k eta)
template <typename R>
__global__ void k_tdh_local(cplx<R> *psi, const R *v, const R *u, int neta, int nk, int64_t N,
                            int64_t ld, R a) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t s = blockIdx.y, S = gridDim.y;
  if (r >= N) return;
  R sn, cs;
  const R ph = v[s * N + r] * a;
  if constexpr (sizeof(R) == 4) sincosf(ph, &sn, &cs);
  else sincos(ph, &sn, &cs);
  R au[SGW_MAX_STATES];
#pragma unroll
  for (int k = 0; k < SGW_MAX_STATES; ++k) au[k] = k < nk ? a * u[(k * S + s) * N + r] : (R)0;
  cplx<R> *p0 = psi + s * (1 + nk) * neta * ld;
#pragma unroll 4
  for (int l = 0; l < neta; ++l) {
    const cplx<R> e = p0[(int64_t)l * ld + r];
#pragma unroll
    for (int k = 0; k < SGW_MAX_STATES; ++k) {
      if (k < nk) {
        cplx<R> *p1 = p0 + (int64_t)(1 + k) * neta * ld;
        cplx<R> d = p1[(int64_t)l * ld + r];
        d.x += au[k] * e.y;      // - i a u eta
        d.y -= au[k] * e.x;
        // multiply by (cs - i sn)
        p1[(int64_t)l * ld + r] = cmake<cplx<R>>(cs * d.x + sn * d.y, cs * d.y - sn * d.x);
      }
    }
    p0[(int64_t)l * ld + r] = cmake<cplx<R>>(cs * e.x + sn * e.y, cs * e.y - sn * e.x);
  }
}

// n = w sum_l |eta_l|^2,  dn_k = 2 w sum_l Re(conj(eta_l) delta-eta_k,l), packed
// as complex fields for the Poisson solve: rho[0][s] = n + i dn_0 and, for
// b >= 1, rho[b][s] = dn_{2b-1} + i dn_{2b} (0 past the last state).
template <typename R>
__global__ void k_tdh_density(const cplx<R> *psi, cplx<R> *rho, int neta, int nk, int64_t N,
                              int64_t ld, R w) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t s = blockIdx.y, S = gridDim.y;
  if (r >= N) return;
  const cplx<R> *p0 = psi + s * (1 + nk) * neta * ld;
  R n = 0, dn[SGW_MAX_STATES];
#pragma unroll
  for (int k = 0; k < SGW_MAX_STATES; ++k) dn[k] = 0;
#pragma unroll 4
  for (int l = 0; l < neta; ++l) {
    const cplx<R> e = p0[(int64_t)l * ld + r];
    n += e.x * e.x + e.y * e.y;
#pragma unroll
    for (int k = 0; k < SGW_MAX_STATES; ++k) {
      if (k < nk) {
        const cplx<R> d = p0[(int64_t)((1 + k) * neta + l) * ld + r];
        dn[k] += e.x * d.x + e.y * d.y;
      }
    }
  }
  rho[s * N + r] = cmake<cplx<R>>(w * n, (R)2 * w * dn[0]);
#pragma unroll
  for (int b = 1; b <= SGW_MAX_STATES / 2; ++b) {
    if (2 * b - 1 < nk) {
      const R hi = 2 * b < nk ? (R)2 * w * dn[2 * b < SGW_MAX_STATES ? 2 * b : 0] : (R)0;
      rho[(b * S + s) * N + r] = cmake<cplx<R>>((R)2 * w * dn[2 * b - 1], hi);
    }
  }
}

template <typename R>
__global__ void k_bcast_real(const R *src, R *dst, int64_t N) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (r < N) dst[(int64_t)blockIdx.y * N + r] = src[r];
}

void launch_tdh_tangent(sgw_ctx *ctx, void *psi, int64_t ld, const void *dv, int S, int neta,
                        int nk) {
  if (ctx->dbl)
    hipLaunchKernelGGL(k_tdh_tangent<double>, grid1(ctx->N, S), dim3(NT), 0, ctx->stream,
                       static_cast<double2 *>(psi), static_cast<const double *>(dv), neta, nk,
                       ctx->N, ld);
  else
    hipLaunchKernelGGL(k_tdh_tangent<float>, grid1(ctx->N, S), dim3(NT), 0, ctx->stream,
                       static_cast<float2 *>(psi), static_cast<const float *>(dv), neta, nk,
                       ctx->N, ld);
  SGW_HIP(hipGetLastError());
}

void launch_tdh_local(sgw_ctx *ctx, void *psi, int64_t ld, const void *v, const void *u, int S,
                      int neta, int nk, double a) {
  if (ctx->dbl)
    hipLaunchKernelGGL(k_tdh_local<double>, grid1(ctx->N, S), dim3(NT), 0, ctx->stream,
                       static_cast<double2 *>(psi), static_cast<const double *>(v),
                       static_cast<const double *>(u), neta, nk, ctx->N, ld, a);
  else
    hipLaunchKernelGGL(k_tdh_local<float>, grid1(ctx->N, S), dim3(NT), 0, ctx->stream,
                       static_cast<float2 *>(psi), static_cast<const float *>(v),
                       static_cast<const float *>(u), neta, nk, ctx->N, ld, (float)a);
  SGW_HIP(hipGetLastError());
}

void launch_tdh_density(sgw_ctx *ctx, const void *psi, int64_t ld, void *rho, int S, int neta,
                        int nk, double w) {
  if (ctx->dbl)
    hipLaunchKernelGGL(k_tdh_density<double>, grid1(ctx->N, S), dim3(NT), 0, ctx->stream,
                       static_cast<const double2 *>(psi), static_cast<double2 *>(rho), neta, nk,
                       ctx->N, ld, w);
  else
    hipLaunchKernelGGL(k_tdh_density<float>, grid1(ctx->N, S), dim3(NT), 0, ctx->stream,
                       static_cast<const float2 *>(psi), static_cast<float2 *>(rho), neta, nk,
                       ctx->N, ld, (float)w);
  SGW_HIP(hipGetLastError());
}

void launch_bcast_real(sgw_ctx *ctx, const void *src, void *dst, int S) {
  if (ctx->dbl)
    hipLaunchKernelGGL(k_bcast_real<double>, grid1(ctx->N, S), dim3(NT), 0, ctx->stream,
                       static_cast<const double *>(src), static_cast<double *>(dst), ctx->N);
  else
    hipLaunchKernelGGL(k_bcast_real<float>, grid1(ctx->N, S), dim3(NT), 0, ctx->stream,
                       static_cast<const float *>(src), static_cast<float *>(dst), ctx->N);
  SGW_HIP(hipGetLastError());
}

// ============================================================ sROI
// Segment blocks of xi_m: draw word mod nblocks, replace a used block by the
// next free one (linear probing); one thread per (sample, m).
__global__ void k_xi_supports(const uint64_t *keys, int S, int n_xi, int nseg,
                              uint64_t nblocks, int *blocks) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t >= (int64_t)S * n_xi) return;
  const int s = (int)(t / n_xi);
  const int64_t m = t % n_xi;
  int *row = blocks + t * nseg;
  const uint64_t key = keys[s];
  for (int g = 0; g < nseg; ++g) {
    uint64_t b = sm64(key + (uint64_t)(m * nseg + g)) % nblocks;
    for (;;) {
      bool used = false;
      for (int q = 0; q < g; ++q) used |= ((uint64_t)row[q] == b);
      if (!used) break;
      b = (b + 1) % nblocks;
    }
    row[g] = (int)b;
  }
}

void launch_xi_supports(sgw_ctx *ctx, const uint64_t *d_keys, int S, int n_xi, int nseg,
                        int *blocks) {
  hipLaunchKernelGGL(k_xi_supports, grid1((int64_t)S * n_xi), dim3(NT), 0, ctx->stream,
                     d_keys, S, n_xi, nseg, (uint64_t)(ctx->N / 32), blocks);
  SGW_HIP(hipGetLastError());
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// one wavefront per xi_m: half-waves take alternate segments of 32 points
template <typename R>
__global__ __launch_bounds__(NT) void k_xi_real(const R *u, const int *blocks,
                                                const uint64_t *skeys, int n_xi, int nseg,
                                                int64_t N, R amp_dv, R *out,
                                                int64_t out_stride_s, int64_t out_off,
                                                const int *step_dev, int64_t step_stride) {
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  const int s = blockIdx.y;
  if (m >= n_xi) return;
  const int *row = blocks + ((int64_t)s * n_xi + m) * nseg;
  const uint64_t key = skeys[s];
  const R *us = u + (int64_t)s * N;
  const int p = lane & 31;
  R acc = 0;
  // the block indices of 64 segments at a time, one per lane, then passed
  // to the half-waves by lane exchange (no dependent load per segment); the
  // exchange runs on the whole wave, the segment on its half-wave.  Four
  // segments per half-wave are loaded before they are added (in order of g);
  // indices past the last segment repeat it (in bounds, not added).
  for (int g0 = 0; g0 < nseg; g0 += 64) {
    const int rowv = g0 + lane < nseg ? row[g0 + lane] : 0;
    const int g1 = min(nseg, g0 + 64);
    for (int gp = g0; gp < g1; gp += 8) {
      R val[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int g = gp + 2 * u + (lane >> 5);
        const int rb = __shfl(rowv, min(g, g1 - 1) - g0, 64);
        val[u] = us[(int64_t)rb * 32 + p];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int g = gp + 2 * u + (lane >> 5);
        if (g < g1) {
          const uint64_t w = sm64(key + (uint64_t)(m * nseg + g));
          acc += ((w >> p) & 1ull) ? -val[u] : val[u];
        }
      }
    }
  }
  acc = wave_sum(acc);
  const int64_t off = out_off + (step_dev ? (int64_t)step_dev[0] * step_stride : 0);
  if (lane == 0) out[s * out_stride_s + off + m] = amp_dv * acc;
}

template <typename R>
__global__ __launch_bounds__(NT) void k_xi_zeta(const cplx<R> *zeta, const R *phi,
                                                const int *blocks, const uint64_t *skeys,
                                                int n_xi, int nseg, int64_t N, R amp_dv,
                                                cplx<R> *dp, cplx<R> *dt) {
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  const int s = blockIdx.y;
  if (m >= n_xi) return;
  const int *row = blocks + ((int64_t)s * n_xi + m) * nseg;
  const uint64_t key = skeys[s];
  const cplx<R> *zp = zeta + (int64_t)s * 2 * N;
  const cplx<R> *zt = zp + N;
  const int p = lane & 31;
  R a0 = 0, a1 = 0, b0 = 0, b1 = 0;
  for (int g0 = 0; g0 < nseg; g0 += 64) {   // block indices and loads as in k_xi_real
    const int rowv = g0 + lane < nseg ? row[g0 + lane] : 0;
    const int g1 = min(nseg, g0 + 64);
    for (int gp = g0; gp < g1; gp += 8) {
      R fv[4];
      cplx<R> xv[4], yv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int g = gp + 2 * u + (lane >> 5);
        const int64_t r = (int64_t)__shfl(rowv, min(g, g1 - 1) - g0, 64) * 32 + p;
        fv[u] = phi[r];
        xv[u] = zp[r];
        yv[u] = zt[r];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int g = gp + 2 * u + (lane >> 5);
        if (g < g1) {
          const uint64_t w = sm64(key + (uint64_t)(m * nseg + g));
          R f = fv[u];
          if ((w >> p) & 1ull) f = -f;
          a0 += f * xv[u].x; a1 += f * xv[u].y;
          b0 += f * yv[u].x; b1 += f * yv[u].y;
        }
      }
    }
  }
  a0 = wave_sum(a0); a1 = wave_sum(a1); b0 = wave_sum(b0); b1 = wave_sum(b1);
  if (lane == 0) {
    dp[(int64_t)s * n_xi + m] = cmake<cplx<R>>(amp_dv * a0, amp_dv * a1);
    dt[(int64_t)s * n_xi + m] = cmake<cplx<R>>(amp_dv * b0, amp_dv * b1);
  }
}

void launch_xi_real(sgw_ctx *ctx, const void *u, const int *blocks, const uint64_t *d_sign_keys,
                    int S, int n_xi, int nseg, double amp_dv, void *out, int64_t out_stride_s,
                    int64_t out_off, const int *step_dev, int64_t step_stride) {
  const dim3 g((n_xi + 3) / 4, S);
  if (ctx->dbl)
    hipLaunchKernelGGL(k_xi_real<double>, g, dim3(NT), 0, ctx->stream,
                       static_cast<const double *>(u), blocks, d_sign_keys, n_xi, nseg, ctx->N,
                       amp_dv, static_cast<double *>(out), out_stride_s, out_off, step_dev,
                       step_stride);
  else
    hipLaunchKernelGGL(k_xi_real<float>, g, dim3(NT), 0, ctx->stream,
                       static_cast<const float *>(u), blocks, d_sign_keys, n_xi, nseg, ctx->N,
                       (float)amp_dv, static_cast<float *>(out), out_stride_s, out_off,
                       step_dev, step_stride);
  SGW_HIP(hipGetLastError());
}

void launch_xi_zeta(sgw_ctx *ctx, const void *zeta, const void *phi, const int *blocks,
                    const uint64_t *d_sign_keys, int S, int n_xi, int nseg, double amp_dv,
                    void *dp, void *dt) {
  const dim3 g((n_xi + 3) / 4, S);
  if (ctx->dbl)
    hipLaunchKernelGGL(k_xi_zeta<double>, g, dim3(NT), 0, ctx->stream,
                       static_cast<const double2 *>(zeta), static_cast<const double *>(phi),
                       blocks, d_sign_keys, n_xi, nseg, ctx->N, amp_dv,
                       static_cast<double2 *>(dp), static_cast<double2 *>(dt));
  else
    hipLaunchKernelGGL(k_xi_zeta<float>, g, dim3(NT), 0, ctx->stream,
                       static_cast<const float2 *>(zeta), static_cast<const float *>(phi),
                       blocks, d_sign_keys, n_xi, nseg, ctx->N, (float)amp_dv,
                       static_cast<float2 *>(dp), static_cast<float2 *>(dt));
  SGW_HIP(hipGetLastError());
}

// ============================================================ time ordering
// Row f_j (j < nt1, zero beyond), A = FFT(f).  For real f, conj(A_k) is the
// e^{+i omega t} transform at omega_k = 2 pi k / (NFT dt); it is kept for
// k <= NFT/2 (omega >= 0) and conjugated -- giving back A_k -- for k > NFT/2
// (omega < 0).  g = FFT(G) / NFT, g_j kept for j < nt1.
template <typename R, int NFT>
__global__ __launch_bounds__(NT) void k_time_order(const R *in, cplx<R> *out, int64_t n_inner,
                                                   int nt1, const cplx<R> *tw) {
  using C = cplx<R>;
  __shared__ C s[NFT];
  const int64_t row = blockIdx.x;
  const int64_t base = (row / n_inner) * nt1 * n_inner + row % n_inner;
  for (int j = threadIdx.x; j < NFT; j += NT)
    s[j] = cmake<C>(j < nt1 ? in[base + (int64_t)j * n_inner] : (R)0, 0);
  __syncthreads();
  lds_fft<C, NFT, 1, 0, 1, false, NT>(s, tw, threadIdx.x);
  for (int k = threadIdx.x; k <= NFT / 2; k += NT) s[k] = cconj(s[k]);
  __syncthreads();
  lds_fft<C, NFT, 1, 0, 1, false, NT>(s, tw, threadIdx.x);
  const R inv = (R)1 / (R)NFT;
  for (int j = threadIdx.x; j < nt1; j += NT) out[base + (int64_t)j * n_inner] = cscale(s[j], inv);
}

template <typename R>
static bool to_dispatch(sgw_ctx *ctx, const void *in, void *out, int64_t nrows, int64_t n_inner,
                        int nt1, int nft, const void *tw) {
  using C = cplx<R>;
  const R *i = static_cast<const R *>(in);
  C *o = static_cast<C *>(out);
  const C *t = static_cast<const C *>(tw);
  const dim3 g((unsigned)nrows);
  switch (nft) {
#define SGW_TO(N) case N: hipLaunchKernelGGL((k_time_order<R, N>), g, dim3(NT), 0, ctx->stream, i, o, n_inner, nt1, t); break;
    SGW_TO(16) SGW_TO(32) SGW_TO(64) SGW_TO(128) SGW_TO(256) SGW_TO(512) SGW_TO(1024)
    SGW_TO(2048)
#undef SGW_TO
    case 4096:
      if constexpr (sizeof(R) == 4) {
        hipLaunchKernelGGL((k_time_order<R, 4096>), g, dim3(NT), 0, ctx->stream, i, o, n_inner,
                           nt1, t);
        break;
      }
      return false;
    default: return false;
  }
  return true;
}

bool launch_time_order(sgw_ctx *ctx, const void *in, void *out, int64_t nrows, int64_t n_inner,
                       int nt1, int nft, const void *d_tw) {
  const bool ok = ctx->dbl ? to_dispatch<double>(ctx, in, out, nrows, n_inner, nt1, nft, d_tw)
                           : to_dispatch<float>(ctx, in, out, nrows, n_inner, nt1, nft, d_tw);
  SGW_HIP(hipGetLastError());
  return ok;
}

// ============================================================ contraction
// sig[(s nt1 + j) 4 + {0,1,2,3}] = (Sigma^+, Sigma^-) of step j, FP64 sums.
// One launch may cover several steps: step j0 + blockIdx.y reads its overlaps
// at dp, dt + blockIdx.y * dstride.
template <typename R>
__global__ __launch_bounds__(NT) void k_contract_xi(const cplx<R> *cto, const cplx<R> *dp,
                                                    const cplx<R> *dt, int n_xi, int nt1, int j0,
                                                    int64_t dstride, double *sig) {
  __shared__ double sh[NT];
  const int s = blockIdx.x;
  const int j = j0 + blockIdx.y;
  dp += blockIdx.y * dstride;
  dt += blockIdx.y * dstride;
  const cplx<R> *c = cto + ((int64_t)s * nt1 + j) * n_xi;
  const cplx<R> *a = dp + (int64_t)s * n_xi;
  const cplx<R> *b = dt + (int64_t)s * n_xi;
  double pr = 0, pi = 0, mr = 0, mi = 0;
  for (int m = threadIdx.x; m < n_xi; m += NT) {
    const double cr = c[m].x, ci = c[m].y;
    const double ar = a[m].x, ai = a[m].y;
    const double br = -b[m].x, bi = b[m].y;   // -conj(d~)
    pr += cr * ar - ci * ai;
    pi += cr * ai + ci * ar;
    mr += cr * br - ci * bi;
    mi += cr * bi + ci * br;
  }
  pr = block_sum(pr, sh);
  pi = block_sum(pi, sh);
  mr = block_sum(mr, sh);
  mi = block_sum(mi, sh);
  if (threadIdx.x == 0) {
    double *o = sig + ((int64_t)s * nt1 + j) * 4;
    o[0] = pr; o[1] = pi; o[2] = mr; o[3] = mi;
  }
}

void launch_contract_xi(sgw_ctx *ctx, const void *cto, const void *dp, const void *dt, int S,
                        int n_xi, int nt1, int j, double *d_sig, int nsteps, int64_t dstride) {
  SGW_REQUIRE(nsteps >= 1 && j + nsteps <= nt1 && nsteps <= 65535, SGW_EINVAL,
              "contract_xi: bad step range");
  const dim3 g(S, nsteps);
  if (ctx->dbl)
    hipLaunchKernelGGL(k_contract_xi<double>, g, dim3(NT), 0, ctx->stream,
                       static_cast<const double2 *>(cto), static_cast<const double2 *>(dp),
                       static_cast<const double2 *>(dt), n_xi, nt1, j, dstride, d_sig);
  else
    hipLaunchKernelGGL(k_contract_xi<float>, g, dim3(NT), 0, ctx->stream,
                       static_cast<const float2 *>(cto), static_cast<const float2 *>(dp),
                       static_cast<const float2 *>(dt), n_xi, nt1, j, dstride, d_sig);
  SGW_HIP(hipGetLastError());
}

template <typename R>
__global__ __launch_bounds__(NT) void k_contract_exact1(const cplx<R> *uto, const cplx<R> *zeta,
                                                        const R *phi, int nt1, int j, int64_t N,
                                                        double *partial, int nblk) {
  __shared__ double sh[NT];
  const int s = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * RCHUNK;
  const int64_t r1 = std::min<int64_t>(N, r0 + RCHUNK);
  const cplx<R> *u = uto + ((int64_t)s * nt1 + j) * N;
  const cplx<R> *zp = zeta + (int64_t)s * 2 * N;
  const cplx<R> *zt = zp + N;
  double pr = 0, pi = 0, mr = 0, mi = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += NT) {
    const double f = phi[r];
    const double ur = u[r].x, ui = u[r].y;
    const double ar = f * zp[r].x, ai = f * zp[r].y;
    const double br = -f * zt[r].x, bi = f * zt[r].y;   // -phi conj(z~)
    pr += ar * ur - ai * ui;
    pi += ar * ui + ai * ur;
    mr += br * ur - bi * ui;
    mi += br * ui + bi * ur;
  }
  pr = block_sum(pr, sh);
  pi = block_sum(pi, sh);
  mr = block_sum(mr, sh);
  mi = block_sum(mi, sh);
  if (threadIdx.x == 0) {
    double *o = partial + ((int64_t)s * nblk + blockIdx.x) * 4;
    o[0] = pr; o[1] = pi; o[2] = mr; o[3] = mi;
  }
}

__global__ void k_contract_exact2(const double *partial, int nblk, int S, int nt1, int j,
                                  double dV, double *sig) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= S * 4) return;
  const int s = t / 4, c = t % 4;
  double acc = 0;
  for (int b = 0; b < nblk; ++b) acc += partial[((int64_t)s * nblk + b) * 4 + c];
  sig[((int64_t)s * nt1 + j) * 4 + c] = dV * acc;
}

void launch_contract_exact(sgw_ctx *ctx, const void *uto, const void *zeta, const void *phi,
                           int S, int nt1, int j, double *d_partial, double *d_sig) {
  const int nblk = (int)((ctx->N + RCHUNK - 1) / RCHUNK);
  if (ctx->dbl)
    hipLaunchKernelGGL(k_contract_exact1<double>, dim3(nblk, S), dim3(NT), 0, ctx->stream,
                       static_cast<const double2 *>(uto), static_cast<const double2 *>(zeta),
                       static_cast<const double *>(phi), nt1, j, ctx->N, d_partial, nblk);
  else
    hipLaunchKernelGGL(k_contract_exact1<float>, dim3(nblk, S), dim3(NT), 0, ctx->stream,
                       static_cast<const float2 *>(uto), static_cast<const float2 *>(zeta),
                       static_cast<const float *>(phi), nt1, j, ctx->N, d_partial, nblk);
  hipLaunchKernelGGL(k_contract_exact2, dim3((S * 4 + NT - 1) / NT), dim3(NT), 0, ctx->stream,
                     d_partial, nblk, S, nt1, j, ctx->dV, d_sig);
  SGW_HIP(hipGetLastError());
}

}  // namespace sgw

namespace sgw {

// device step counters of replayed graphs (vector stores from one lane)
__global__ void k_counter(int *c, int idx, int value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[idx] = add ? c[idx] + value : value;
}

void launch_counter(sgw_ctx *ctx, int idx, int value, bool add) {
  hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, ctx->stream,
                     ctx->d_counter.as<int>(), idx, value, add ? 1 : 0);
  SGW_HIP(hipGetLastError());
}

}  // namespace sgw
