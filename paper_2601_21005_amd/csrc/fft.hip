// 3D FFT passes for H|psi> and the split-operator steps (Sec. 2.2: FFT pairs
// switch between the position representation, where V is diagonal, and the
// momentum representation, where T is diagonal).
//
// Passes over a batch of vectors (x fastest):
//   plane   one xy plane of one vector per workgroup, x then y transform in
//           LDS, with fused epilogues on the inverse pass (V psi, Chebyshev
//           update, Poisson outputs) -- used when the plane fits in LDS;
//   pencil  TX neighbouring x columns along y or z per workgroup (coalesced
//           rows of TX complex), optionally forward z -> k-space multiplier
//           -> inverse z in one pass;
//   xlines  whole x lines (fallback for planes too big for LDS).
#include "fft_lds.h"

namespace sgw {

constexpr int NT_FFT = 256;

struct PassArgs {
  const void *src = nullptr;
  void *dst = nullptr;
  int64_t ld_src = 0, ld_dst = 0, ld_x = 0;
  const void *tw0 = nullptr, *tw1 = nullptr;   // twiddles of the two axes used
  const void *k2x = nullptr, *k2y = nullptr, *k2z = nullptr;
  int nx = 0, ny = 0, nz = 0;
  int mode = 0;          // PlaneMode (inverse passes) / 0 forward
  int inverse = 0;
  int mul = 0;           // MulMode (pencil z)
  int axis = 2;          // pencil: 1 = y, 2 = z
  int rev = 0;           // 1: vectors in descending order of blockIdx.y
  double tau = 0, ecut = 0, invN = 0;
  int64_t N = 0;
  EpiArgs e;
};

// ----------------------------------------------------------------- epilogue
template <typename R, int MODE>
__device__ __forceinline__ void epilogue(const PassArgs &a, int64_t v, int64_t r,
                                         cplx<R> val) {
  using C = cplx<R>;
  switch (MODE) {
    case PLANE_FWD:
    case PLANE_INV_STORE:
      static_cast<C *>(a.dst)[v * a.ld_dst + r] = val;
      break;
    case PLANE_INV_HPSI: {
      const C x = static_cast<const C *>(a.e.x)[v * a.ld_x + r];
      const R V = static_cast<const R *>(a.e.vloc)[r];
      val.x += V * x.x;
      val.y += V * x.y;
      static_cast<C *>(a.dst)[v * a.ld_dst + r] = val;
    } break;
    case PLANE_INV_CHEB: {
      // x = v_n:  w = (H x - c x)/R ; v_{n+1} = s2 w - v_{n-1} (no v_{n-1}
      // on the first step).  The projector part of H x is added to v_{n+1}
      // afterwards, so v_{n-1} and v_n are complete here; on odd n the pair
      // b_{n-1} v_{n-1} + b_n v_n goes into acc.
      const int64_t o = v * a.ld_x + r;
      const C x = static_cast<const C *>(a.e.x)[o];
      const R V = static_cast<const R *>(a.e.vloc)[r];
      const R c = (R)a.e.c, iR = (R)a.e.invR, s2 = (R)a.e.scale2;
      C *vold = static_cast<C *>(a.e.vold);
      C *vout = a.e.vout ? static_cast<C *>(a.e.vout) : vold;
      C *acc = static_cast<C *>(a.e.acc);
      C p;
      p.x = p.y = 0;
      if (!a.e.first) p = vold[o];
      C nv;
      nv.x = s2 * ((val.x + (V - c) * x.x) * iR) - p.x;
      nv.y = s2 * ((val.y + (V - c) * x.y) * iR) - p.y;
      vout[o] = nv;
      if (a.e.acc_mode) {
        R b0r = (R)a.e.cprev_re, b0i = (R)a.e.cprev_im, b1r = (R)a.e.coef_re, b1i = (R)a.e.coef_im;
        if (a.e.coef_dev) {
          const int k = a.e.term_dev[0];
          b0r = (R)a.e.coef_dev[2 * k - 2];
          b0i = (R)a.e.coef_dev[2 * k - 1];
          b1r = (R)a.e.coef_dev[2 * k];
          b1i = (R)a.e.coef_dev[2 * k + 1];
        }
        C sm;
        sm.x = sm.y = 0;
        if (a.e.acc_mode == 2) sm = acc[o];
        sm.x += b0r * p.x - b0i * p.y;
        sm.y += b0r * p.y + b0i * p.x;
        sm.x += b1r * x.x - b1i * x.y;
        sm.y += b1r * x.y + b1i * x.x;
        acc[o] = sm;
      }
    } break;
    case PLANE_INV_POISSON: {
      const int64_t o = v * a.N + r;
      const R V = static_cast<const R *>(a.e.vloc)[r];
      static_cast<R *>(a.e.r0)[o] = V + val.x - static_cast<const R *>(a.e.vh0)[o];
      static_cast<R *>(a.e.r1)[o] = val.y;
    } break;
    case PLANE_INV_SPLIT: {
      const int64_t o = v * a.N + r;
      if (a.e.r0) static_cast<R *>(a.e.r0)[o] = val.x;
      if (a.e.r1) static_cast<R *>(a.e.r1)[o] = val.y;
    } break;
  }
}

// ----------------------------------------------------------------- plane
template <typename R, int NX, int NY, int MODE>
__global__ __launch_bounds__(NT_FFT) void k_plane(PassArgs a) {
  constexpr bool INV = MODE != PLANE_FWD;
  using C = cplx<R>;
  constexpr int P = NX + 1;
  constexpr int E = NX * NY;
  __shared__ C s[NY * P];
  __shared__ C twx[NX], twy[NY];
  const int tid = threadIdx.x;
  const int z = blockIdx.x;
  const int64_t v = a.rev ? gridDim.y - 1 - blockIdx.y : blockIdx.y;
  for (int i = tid; i < NX; i += NT_FFT) twx[i] = static_cast<const C *>(a.tw0)[i];
  for (int i = tid; i < NY; i += NT_FFT) twy[i] = static_cast<const C *>(a.tw1)[i];
  const int64_t plane = (int64_t)z * E;
  const C *src = static_cast<const C *>(a.src) + v * a.ld_src + plane;
#pragma unroll
  for (int q = 0; q < (E + NT_FFT - 1) / NT_FFT; ++q) {
    const int e = tid + q * NT_FFT;
    if (E % NT_FFT == 0 || e < E) {
      C val = src[e];
      if (INV) val = cconj(val);
      s[(e / NX) * P + (e % NX)] = val;
    }
  }
  __syncthreads();
  lds_fft<C, NX, NY, P, 1, true, NT_FFT>(s, twx, tid);
  lds_fft<C, NY, NX, 1, P, true, NT_FFT>(s, twy, tid);
  constexpr int Q = (E + NT_FFT - 1) / NT_FFT;
  if constexpr (MODE == PLANE_INV_CHEB && E % NT_FFT == 0) {
    // all operand loads of this thread in flight at once, then the updates
    // (the stores to vold / acc would otherwise order every later load)
    const C *xp = static_cast<const C *>(a.e.x) + v * a.ld_x + plane;
    C *vp = static_cast<C *>(a.e.vold) + v * a.ld_x + plane;
    C *wp = (a.e.vout ? static_cast<C *>(a.e.vout) : static_cast<C *>(a.e.vold)) + v * a.ld_x + plane;
    C *ap = static_cast<C *>(a.e.acc) + v * a.ld_x + plane;
    const R *Vp = static_cast<const R *>(a.e.vloc) + plane;
    const bool first = a.e.first != 0;
    const int am = a.e.acc_mode;
    const R c = (R)a.e.c, iR = (R)a.e.invR, s2 = (R)a.e.scale2;
    R b0r = (R)a.e.cprev_re, b0i = (R)a.e.cprev_im, b1r = (R)a.e.coef_re, b1i = (R)a.e.coef_im;
    if (am && a.e.coef_dev) {
      const int k = a.e.term_dev[0];
      b0r = (R)a.e.coef_dev[2 * k - 2];
      b0i = (R)a.e.coef_dev[2 * k - 1];
      b1r = (R)a.e.coef_dev[2 * k];
      b1i = (R)a.e.coef_dev[2 * k + 1];
    }
    // two halves keep the operands within the 4-waves-per-SIMD register budget
    constexpr int QH = Q % 2 == 0 ? Q / 2 : Q;
#pragma unroll
    for (int h = 0; h < Q / QH; ++h) {
      C xs[QH], ps[QH], ss[QH];
      R Vs[QH];
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        const int e = tid + (h * QH + q) * NT_FFT;
        xs[q] = xp[e];
        Vs[q] = Vp[e];
        ps[q].x = ps[q].y = 0;
        ss[q].x = ss[q].y = 0;
        if (!first) ps[q] = vp[e];
        if (am == 2) ss[q] = ap[e];
      }
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        const int e = tid + (h * QH + q) * NT_FFT;
        const C val = cconj(s[(e / NX) * P + (e % NX)]);
        const C x = xs[q], pv = ps[q];
        // w = (H x - c x)/R; v_{n+1} = s2 w - v_{n-1}; on odd n
        // acc (+)= b_{n-1} v_{n-1} + b_n v_n
        C nv;
        nv.x = s2 * ((val.x + (Vs[q] - c) * x.x) * iR) - pv.x;
        nv.y = s2 * ((val.y + (Vs[q] - c) * x.y) * iR) - pv.y;
        wp[e] = nv;
        if (am) {
          C sm = ss[q];
          sm.x += b0r * pv.x - b0i * pv.y;
          sm.y += b0r * pv.y + b0i * pv.x;
          sm.x += b1r * x.x - b1i * x.y;
          sm.y += b1r * x.y + b1i * x.x;
          ap[e] = sm;
        }
      }
    }
  } else if constexpr (MODE == PLANE_INV_HPSI && E % NT_FFT == 0) {
    // H psi = (T psi) + V psi: loads first, then the stores
    const C *xp = static_cast<const C *>(a.e.x) + v * a.ld_x + plane;
    const R *Vp = static_cast<const R *>(a.e.vloc) + plane;
    C *dp = static_cast<C *>(a.dst) + v * a.ld_dst + plane;
    C xs[Q];
    R Vs[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      xs[q] = xp[tid + q * NT_FFT];
      Vs[q] = Vp[tid + q * NT_FFT];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + q * NT_FFT;
      C val = cconj(s[(e / NX) * P + (e % NX)]);
      val.x += Vs[q] * xs[q].x;
      val.y += Vs[q] * xs[q].y;
      dp[e] = val;
    }
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + q * NT_FFT;
      if (E % NT_FFT == 0 || e < E) {
        C val = s[(e / NX) * P + (e % NX)];
        if (INV) val = cconj(val);
        epilogue<R, MODE>(a, v, plane + e, val);
      }
    }
  }
}

// ----------------------------------------------------------------- xlines
template <typename R, int NX, int NL, int MODE>
__global__ __launch_bounds__(NT_FFT) void k_xlines(PassArgs a) {
  constexpr bool INV = MODE != PLANE_FWD;
  using C = cplx<R>;
  constexpr int P = NX + 1;
  constexpr int E = NX * NL;
  __shared__ C s[NL * P];
  __shared__ C twx[NX];
  const int tid = threadIdx.x;
  const int64_t v = a.rev ? gridDim.y - 1 - blockIdx.y : blockIdx.y;
  const int64_t nlines = (int64_t)a.ny * a.nz;
  const int64_t l0 = (int64_t)blockIdx.x * NL;
  for (int i = tid; i < NX; i += NT_FFT) twx[i] = static_cast<const C *>(a.tw0)[i];
  const C *src = static_cast<const C *>(a.src) + v * a.ld_src;
#pragma unroll
  for (int q = 0; q < (E + NT_FFT - 1) / NT_FFT; ++q) {
    const int e = tid + q * NT_FFT;
    if ((E % NT_FFT == 0 || e < E) && l0 + e / NX < nlines) {
      C val = src[l0 * NX + e];
      if (INV) val = cconj(val);
      s[(e / NX) * P + (e % NX)] = val;
    }
  }
  __syncthreads();
  lds_fft<C, NX, NL, P, 1, true, NT_FFT>(s, twx, tid);
#pragma unroll
  for (int q = 0; q < (E + NT_FFT - 1) / NT_FFT; ++q) {
    const int e = tid + q * NT_FFT;
    if ((E % NT_FFT == 0 || e < E) && l0 + e / NX < nlines) {
      C val = s[(e / NX) * P + (e % NX)];
      if (INV) val = cconj(val);
      epilogue<R, MODE>(a, v, l0 * NX + e, val);
    }
  }
}

// ----------------------------------------------------------------- pencil
template <typename R>
__device__ __forceinline__ cplx<R> kmul(const PassArgs &a, int ix, int iy, int iz) {
  using C = cplx<R>;
  const R k2 = static_cast<const R *>(a.k2x)[ix] + static_cast<const R *>(a.k2y)[iy] +
               static_cast<const R *>(a.k2z)[iz];
  C m;
  m.y = 0;
  if (a.mul == MUL_COUL) {
    m.x = k2 > (R)0 ? (R)(4.0 * M_PI) / k2 * (R)a.invN : (R)0;
  } else {
    R T = (R)0.5 * k2;
    if (a.ecut > 0 && T > (R)a.ecut) T = (R)a.ecut;
    if (a.mul == MUL_KIN) {
      m.x = T * (R)a.invN;
    } else {  // MUL_PROP: exp(-i T tau) / N
      R sn, cs;
      if constexpr (sizeof(R) == 4) sincosf(T * (R)a.tau, &sn, &cs);
      else sincos(T * (R)a.tau, &sn, &cs);
      m.x = cs * (R)a.invN;
      m.y = -sn * (R)a.invN;
    }
  }
  return m;
}

// Columns x0..x0+TX-1 of one (y or z) line family; NLEN = length of the axis.
template <typename R, int NLEN, int TX>
__global__ __launch_bounds__(NT_FFT) void k_pencil(PassArgs a) {
  using C = cplx<R>;
  constexpr int P = TX + 1;
  constexpr int E = NLEN * TX;
  __shared__ C s[NLEN * P];
  __shared__ C tw[NLEN];
  const int tid = threadIdx.x;
  const int nxb = a.nx / TX;
  const int xb = blockIdx.x % nxb;
  const int w = blockIdx.x / nxb;       // z (axis y) or y (axis z)
  const int64_t v = a.rev ? gridDim.y - 1 - blockIdx.y : blockIdx.y;
  const int x0 = xb * TX;
  const int64_t stride = a.axis == 2 ? (int64_t)a.nx * a.ny : (int64_t)a.nx;
  const int64_t base = a.axis == 2 ? x0 + (int64_t)w * a.nx : x0 + (int64_t)w * a.nx * a.ny;
  for (int i = tid; i < NLEN; i += NT_FFT) tw[i] = static_cast<const C *>(a.tw0)[i];
  // in place on dst, or from src (ld_src) into dst when src is given
  C *data = static_cast<C *>(a.dst) + v * a.ld_dst + base;
  const C *in = a.src ? static_cast<const C *>(a.src) + v * a.ld_src + base : data;
#pragma unroll
  for (int q = 0; q < (E + NT_FFT - 1) / NT_FFT; ++q) {
    const int e = tid + q * NT_FFT;
    if (E % NT_FFT == 0 || e < E) {
      C val = in[(e / TX) * stride + (e % TX)];
      if (a.inverse) val = cconj(val);
      s[(e / TX) * P + (e % TX)] = val;
    }
  }
  __syncthreads();
  lds_fft<C, NLEN, TX, 1, P, true, NT_FFT>(s, tw, tid);
  bool conj_out = a.inverse;
  if (a.mul != MUL_NONE) {
    // multiply in k space, then inverse transform as conj(FFT(conj))
#pragma unroll
    for (int q = 0; q < (E + NT_FFT - 1) / NT_FFT; ++q) {
      const int e = tid + q * NT_FFT;
      if (E % NT_FFT == 0 || e < E) {
        const int j = e / TX, c = e % TX;
        C m = kmul<R>(a, x0 + c, w, j);
        C val = cmul(s[j * P + c], m);
        s[j * P + c] = cconj(val);
      }
    }
    __syncthreads();
    lds_fft<C, NLEN, TX, 1, P, true, NT_FFT>(s, tw, tid);
    conj_out = true;
  }
#pragma unroll
  for (int q = 0; q < (E + NT_FFT - 1) / NT_FFT; ++q) {
    const int e = tid + q * NT_FFT;
    if (E % NT_FFT == 0 || e < E) {
      C val = s[(e / TX) * P + (e % TX)];
      if (conj_out) val = cconj(val);
      data[(e / TX) * stride + (e % TX)] = val;
    }
  }
}

// ----------------------------------------------------------------- dispatch
template <typename R> constexpr int plane_max_bytes() { return 64 * 1024 - 4096; }

template <typename R, int N> constexpr bool plane_fits() {
  return (int64_t)N * (N + 1) * sizeof(cplx<R>) + 2 * N * sizeof(cplx<R>) <= plane_max_bytes<R>();
}

template <int N> constexpr int pencil_tx() { return N % 16 == 0 ? 16 : N % 8 == 0 ? 8 : 4; }
// wider pencils (rows of 32 complex) where the length allows them
template <int N> constexpr int pencil_tx_wide() { return N % 32 == 0 ? 32 : pencil_tx<N>(); }
template <int N> constexpr int xlines_nl() { return N >= 2048 ? 1 : 2048 / N; }

template <typename R, int N, int MODE> static void launch_plane(dim3 g, hipStream_t st,
                                                              const PassArgs &a) {
  if constexpr (plane_fits<R, N>())
    hipLaunchKernelGGL((k_plane<R, N, N, MODE>), g, dim3(NT_FFT), 0, st, a);
}
template <typename R, int N, int MODE> static void launch_xlines(dim3 g, hipStream_t st,
                                                               const PassArgs &a) {
  hipLaunchKernelGGL((k_xlines<R, N, xlines_nl<N>(), MODE>), g, dim3(NT_FFT), 0, st, a);
}

template <typename R, int N> struct Kernels {
  static void plane(dim3 g, hipStream_t st, const PassArgs &a) {
    switch (a.mode) {
      case PLANE_FWD: launch_plane<R, N, PLANE_FWD>(g, st, a); break;
      case PLANE_INV_STORE: launch_plane<R, N, PLANE_INV_STORE>(g, st, a); break;
      case PLANE_INV_HPSI: launch_plane<R, N, PLANE_INV_HPSI>(g, st, a); break;
      case PLANE_INV_CHEB: launch_plane<R, N, PLANE_INV_CHEB>(g, st, a); break;
      case PLANE_INV_POISSON: launch_plane<R, N, PLANE_INV_POISSON>(g, st, a); break;
      case PLANE_INV_SPLIT: launch_plane<R, N, PLANE_INV_SPLIT>(g, st, a); break;
    }
  }
  static void pencil(dim3 g, hipStream_t st, const PassArgs &a) {
    hipLaunchKernelGGL((k_pencil<R, N, pencil_tx<N>()>), g, dim3(NT_FFT), 0, st, a);
  }
  static void pencil_wide(dim3 g, hipStream_t st, const PassArgs &a) {
    hipLaunchKernelGGL((k_pencil<R, N, pencil_tx_wide<N>()>), g, dim3(NT_FFT), 0, st, a);
  }
  static void xlines(dim3 g, hipStream_t st, const PassArgs &a) {
    switch (a.mode) {
      case PLANE_FWD: launch_xlines<R, N, PLANE_FWD>(g, st, a); break;
      case PLANE_INV_STORE: launch_xlines<R, N, PLANE_INV_STORE>(g, st, a); break;
      case PLANE_INV_HPSI: launch_xlines<R, N, PLANE_INV_HPSI>(g, st, a); break;
      case PLANE_INV_CHEB: launch_xlines<R, N, PLANE_INV_CHEB>(g, st, a); break;
      case PLANE_INV_POISSON: launch_xlines<R, N, PLANE_INV_POISSON>(g, st, a); break;
      case PLANE_INV_SPLIT: launch_xlines<R, N, PLANE_INV_SPLIT>(g, st, a); break;
    }
  }
  static constexpr bool has_plane = plane_fits<R, N>();
  static constexpr int tx = pencil_tx<N>();
  static constexpr int tx_wide = pencil_tx_wide<N>();
  static constexpr int nl = xlines_nl<N>();
};

struct SizeOps {
  void (*plane)(dim3, hipStream_t, const PassArgs &);
  void (*pencil)(dim3, hipStream_t, const PassArgs &);
  void (*xlines)(dim3, hipStream_t, const PassArgs &);
  void (*pencil_wide)(dim3, hipStream_t, const PassArgs &);
  bool has_plane;
  int tx, nl, tx_wide;
};

template <typename R, int N> SizeOps make_ops() {
  return SizeOps{&Kernels<R, N>::plane, &Kernels<R, N>::pencil, &Kernels<R, N>::xlines,
                 &Kernels<R, N>::pencil_wide, Kernels<R, N>::has_plane, Kernels<R, N>::tx,
                 Kernels<R, N>::nl, Kernels<R, N>::tx_wide};
}

template <typename R> bool get_ops(int n, SizeOps &o) {
  switch (n) {
#define SGW_SIZE(N) case N: o = make_ops<R, N>(); return true;
    SGW_SIZE(8) SGW_SIZE(12) SGW_SIZE(16) SGW_SIZE(24) SGW_SIZE(32) SGW_SIZE(40)
    SGW_SIZE(48) SGW_SIZE(56) SGW_SIZE(64) SGW_SIZE(80) SGW_SIZE(96) SGW_SIZE(112)
    SGW_SIZE(128) SGW_SIZE(160)
#undef SGW_SIZE
    default: return false;
  }
}

bool fft_size_supported(int n, bool dbl) {
  SizeOps o;
  return dbl ? get_ops<double>(n, o) : get_ops<float>(n, o);
}

// The pencil passes launch (nx / width) workgroups per row of columns, the
// width being that of the pencil length: every column is covered only when
// nx is a multiple of the z pencils' width (and of the y pencils', which
// holds whenever nx == ny).
bool fft_pencils_cover(int nx, int ny, int nz, bool dbl) {
  SizeOps oy, oz;
  const bool ok = dbl ? (get_ops<double>(ny, oy) && get_ops<double>(nz, oz))
                      : (get_ops<float>(ny, oy) && get_ops<float>(nz, oz));
  return ok && nx % oz.tx == 0 && nx % oy.tx == 0;
}

template <typename R>
void fft3d_apply_t(sgw_ctx *ctx, const void *src, void *tmp, void *dst, int64_t nvec,
                   int64_t ld, MulMode mul, double tau, PlaneMode inv_mode,
                   const EpiArgs &epi, int64_t ldt, void *tmp2, bool rev) {
  using C = cplx<R>;
  SizeOps ox, oy, oz;
  SGW_REQUIRE(get_ops<R>(ctx->nx, ox) && get_ops<R>(ctx->ny, oy) && get_ops<R>(ctx->nz, oz),
              SGW_EUNSUPPORTED, "grid size not built");
  const int64_t N = ctx->N;
  const C *tw = ctx->d_tw.as<C>();
  const R *k2 = ctx->d_k2.as<R>();
  PassArgs base;
  base.nx = ctx->nx; base.ny = ctx->ny; base.nz = ctx->nz;
  base.N = N;
  base.invN = 1.0 / (double)N;
  base.tau = tau;
  base.ecut = ctx->ecut;
  base.k2x = k2; base.k2y = k2 + ctx->nx; base.k2z = k2 + ctx->nx + ctx->ny;
  base.e = epi;
  const C *twx = tw, *twy = tw + ctx->nx, *twz = tw + ctx->nx + ctx->ny;
  hipStream_t st = ctx->stream;
  const bool use_plane = ctx->nx == ctx->ny && ox.has_plane;
  for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
    const int64_t nv = std::min<int64_t>(65535, nvec - v0);
    const C *srcv = static_cast<const C *>(src) + v0 * ld;
    C *tmpv = static_cast<C *>(tmp) + v0 * ldt;
    C *tmp2v = tmp2 ? static_cast<C *>(tmp2) + v0 * ldt : tmpv;   // z pencils' output
    C *dstv = dst ? static_cast<C *>(dst) + v0 * ld : nullptr;
    PassArgs a = base;
    // shift epilogue vector pointers to this chunk
    if (a.e.x) a.e.x = static_cast<const C *>(a.e.x) + v0 * ld;
    if (a.e.vold) a.e.vold = static_cast<C *>(a.e.vold) + v0 * ld;
    if (a.e.vout) a.e.vout = static_cast<C *>(a.e.vout) + v0 * ld;
    if (a.e.acc) a.e.acc = static_cast<C *>(a.e.acc) + v0 * ld;
    if (a.e.vh0) a.e.vh0 = static_cast<const R *>(a.e.vh0) + v0 * N;
    if (a.e.r0) a.e.r0 = static_cast<R *>(a.e.r0) + v0 * N;
    if (a.e.r1) a.e.r1 = static_cast<R *>(a.e.r1) + v0 * N;
    a.ld_x = ld;
    // forward xy
    PassArgs f = a;
    // successive passes run the vectors in alternate directions, each starting
    // on those the pass before wrote last
    int dir = rev ? 1 : 0;
    f.src = srcv; f.dst = tmpv; f.ld_src = ld; f.ld_dst = ldt; f.mode = PLANE_FWD; f.inverse = 0;
    f.rev = dir;
    if (use_plane) {
      f.tw0 = twx; f.tw1 = twy;
      ox.plane(dim3(ctx->nz, nv), st, f);
    } else {
      f.tw0 = twx;
      ox.xlines(dim3((ctx->ny * ctx->nz + ox.nl - 1) / ox.nl, nv), st, f);
      PassArgs py = a;
      py.dst = tmpv; py.ld_dst = ldt; py.axis = 1; py.tw0 = twy; py.inverse = 0; py.mul = MUL_NONE;
      dir ^= 1;
      py.rev = dir;
      oy.pencil(dim3((ctx->nx / oy.tx) * ctx->nz, nv), st, py);
    }
    SGW_HIP(hipGetLastError());
    // z: forward, multiply, inverse
    PassArgs pz = a;
    pz.dst = tmp2v; pz.ld_dst = ldt; pz.axis = 2; pz.tw0 = twz; pz.inverse = 0; pz.mul = mul;
    if (tmp2) { pz.src = tmpv; pz.ld_src = ldt; }
    dir ^= 1;
    pz.rev = dir;
    // z pencils: rows of 32 complex when the lengths allow it (SGW_FORCE_VARIANT
    // pencil=0 keeps rows of 16); every column is the same 1D transform either way
    const auto fp = ctx->forced.find("pencil");
    const bool wide = oz.tx_wide != oz.tx && ctx->nx % oz.tx_wide == 0 &&
                      (fp == ctx->forced.end() || fp->second != 0);
    if (wide)
      oz.pencil_wide(dim3((ctx->nx / oz.tx_wide) * ctx->ny, nv), st, pz);
    else
      oz.pencil(dim3((ctx->nx / oz.tx) * ctx->ny, nv), st, pz);
    SGW_HIP(hipGetLastError());
    // inverse xy with the epilogue
    PassArgs b = a;
    b.src = tmp2v; b.ld_src = ldt; b.dst = dstv; b.ld_dst = ld; b.mode = inv_mode; b.inverse = 1;
    const bool timed = (ctx->ktimer & 1) && inv_mode == PLANE_INV_CHEB && ctx->ns.empty();
    if (!use_plane) {
      PassArgs py = a;
      py.dst = tmp2v; py.ld_dst = ldt; py.axis = 1; py.tw0 = twy; py.inverse = 1; py.mul = MUL_NONE;
      dir ^= 1;
      py.rev = dir;
      oy.pencil(dim3((ctx->nx / oy.tx) * ctx->nz, nv), st, py);
    }
    dir ^= 1;
    b.rev = dir;
    if (timed) SGW_HIP(hipEventRecord(ctx->kt[0].event(0), st));
    if (use_plane) {
      b.tw0 = twx; b.tw1 = twy;
      ox.plane(dim3(ctx->nz, nv), st, b);
    } else {
      b.tw0 = twx;
      ox.xlines(dim3((ctx->ny * ctx->nz + ox.nl - 1) / ox.nl, nv), st, b);
    }
    if (timed) {
      SGW_HIP(hipEventRecord(ctx->kt[0].event(1), st));
      ctx->kt[0].used++;
      ctx->kt[0].points += nv * N;
    }
    SGW_HIP(hipGetLastError());
  }
}

void fft3d_apply(sgw_ctx *ctx, const void *src, void *tmp, void *dst, int64_t nvec,
                 int64_t ld, MulMode mul, double tau, PlaneMode inv_mode,
                 const EpiArgs &epi, int64_t ld_tmp, void *tmp2, bool rev) {
  if (nvec <= 0) return;
  const int64_t ldt = ld_tmp > 0 ? ld_tmp : ctx->N;
  if (ctx->dbl)
    fft3d_apply_t<double>(ctx, src, tmp, dst, nvec, ld, mul, tau, inv_mode, epi, ldt, tmp2, rev);
  else
    fft3d_apply_t<float>(ctx, src, tmp, dst, nvec, ld, mul, tau, inv_mode, epi, ldt, tmp2, rev);
}

}  // namespace sgw
