// In-LDS mixed-radix FFT building blocks (forward sign, exp(-2 pi i jk/N)).
//
// Self-sorting Stockham stages: a stage of radix R on lines of length N whose
// sub-transforms already have length NS reads x[j + i N/R], twiddles by
// exp(-2 pi i i (j mod NS)/(NS R)), applies an R-point DFT and writes
// y[(j div NS) NS R + (j mod NS) + i NS].  Each thread keeps its butterflies
// in registers between the read and the write so one LDS buffer serves as
// both (barrier in between).  Radices 8, 7, 5, 4, 3, 2 are chosen greedily
// at compile time; inverse transforms are taken as conj(FFT(conj(x))).
#pragma once

#include "common.h"

namespace sgw {

__host__ __device__ constexpr int pick_radix(int m) {
  return m % 8 == 0 ? 8 : m % 7 == 0 ? 7 : m % 5 == 0 ? 5 : m % 4 == 0 ? 4 : m % 3 == 0 ? 3 : 2;
}

__host__ __device__ constexpr bool fft_len_ok(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  while (n % 7 == 0) n /= 7;
  return n == 1;
}

// cos(2 pi m / R) and sin(2 pi m / R) for the odd radices
__device__ __forceinline__ constexpr double rcos(int R, int m) {
  return R == 3 ? (m == 0 ? 1.0 : -0.5)
       : R == 5 ? (m == 0 ? 1.0 : (m == 1 || m == 4) ? 0.30901699437494745 : -0.8090169943749475)
       : (m == 0 ? 1.0 : (m == 1 || m == 6) ? 0.6234898018587336
          : (m == 2 || m == 5) ? -0.22252093395631434 : -0.9009688679024191);
}
__device__ __forceinline__ constexpr double rsin(int R, int m) {
  return R == 3 ? (m == 0 ? 0.0 : m == 1 ? 0.8660254037844386 : -0.8660254037844386)
       : R == 5 ? (m == 0 ? 0.0 : m == 1 ? 0.9510565162951535 : m == 2 ? 0.5877852522924731
                   : m == 3 ? -0.5877852522924731 : -0.9510565162951535)
       : (m == 0 ? 0.0 : m == 1 ? 0.7818314824680298 : m == 2 ? 0.9749279121818236
          : m == 3 ? 0.4338837391175582 : m == 4 ? -0.4338837391175582
          : m == 5 ? -0.9749279121818236 : -0.7818314824680298);
}

template <typename C> __device__ __forceinline__ C mul_mi(C z) {  // (-i) z
  C r; r.x = z.y; r.y = -z.x; return r;
}

template <typename C, int R> struct DFT;

template <typename C> struct DFT<C, 2> {
  static __device__ __forceinline__ void run(C *a) {
    C t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <typename C> struct DFT<C, 4> {
  static __device__ __forceinline__ void run(C *a) {
    C s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    C s13 = cadd(a[1], a[3]), d13 = mul_mi(csub(a[1], a[3]));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, d13);
    a[3] = csub(d02, d13);
  }
};

template <typename C> struct DFT<C, 8> {
  static __device__ __forceinline__ void run(C *a) {
    using R = decltype(a[0].x);
    C e[4] = {a[0], a[2], a[4], a[6]};
    C o[4] = {a[1], a[3], a[5], a[7]};
    DFT<C, 4>::run(e);
    DFT<C, 4>::run(o);
    const R h = (R)0.70710678118654752440;
    C w1; w1.x = h * (o[1].x + o[1].y); w1.y = h * (o[1].y - o[1].x);   // e^{-i pi/4}
    C w2 = mul_mi(o[2]);                                                 // e^{-i pi/2}
    C w3; w3.x = h * (o[3].y - o[3].x); w3.y = -h * (o[3].x + o[3].y);   // e^{-3i pi/4}
    a[0] = cadd(e[0], o[0]); a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], w1);   a[5] = csub(e[1], w1);
    a[2] = cadd(e[2], w2);   a[6] = csub(e[2], w2);
    a[3] = cadd(e[3], w3);   a[7] = csub(e[3], w3);
  }
};

// odd radix by symmetric pairs: X_k = A_k - i B_k, X_{R-k} = A_k + i B_k,
// A_k = a_0 + sum_j (a_j + a_{R-j}) cos(2 pi jk/R),
// B_k = sum_j (a_j - a_{R-j}) sin(2 pi jk/R)
template <typename C, int R> struct DFTodd {
  static __device__ __forceinline__ void run(C *a) {
    using T = decltype(a[0].x);
    constexpr int H = (R - 1) / 2;
    C s[H], d[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      s[j - 1] = cadd(a[j], a[R - j]);
      d[j - 1] = csub(a[j], a[R - j]);
    }
    C x0 = a[0];
    C X0 = x0;
#pragma unroll
    for (int j = 0; j < H; ++j) X0 = cadd(X0, s[j]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      C A = x0, B;
      B.x = 0; B.y = 0;
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const T cc = (T)rcos(R, (j * k) % R), ss = (T)rsin(R, (j * k) % R);
        A.x += cc * s[j - 1].x; A.y += cc * s[j - 1].y;
        B.x += ss * d[j - 1].x; B.y += ss * d[j - 1].y;
      }
      C mB = mul_mi(B);
      a[k] = cadd(A, mB);
      a[R - k] = csub(A, mB);
    }
    a[0] = X0;
  }
};
template <typename C> struct DFT<C, 3> : DFTodd<C, 3> {};
template <typename C> struct DFT<C, 5> : DFTodd<C, 5> {};
template <typename C> struct DFT<C, 7> : DFTodd<C, 7> {};

// One Stockham stage and the stages after it, over NL lines of length N
// stored at buf[line * LS + index * ES].  LINE_FAST: consecutive threads take
// consecutive lines (lines interleaved in memory), else consecutive indices.
template <typename C, int N, int NS, int NL, int LS, int ES, bool LINE_FAST, int NT>
__device__ __forceinline__ void fft_stages(C *__restrict__ buf, const C *__restrict__ tw,
                                           int tid) {
  constexpr int R = pick_radix(N / NS);
  constexpr int M = N / R;
  constexpr int NB = NL * M;
  constexpr int Q = (NB + NT - 1) / NT;
  constexpr int TWS = N / (NS * R);
  C reg[Q][R];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = tid + q * NT;
    if (NB % NT == 0 || b < NB) {
      const int line = LINE_FAST ? b % NL : b / M;
      const int j = LINE_FAST ? b / NL : b % M;
      const int k = j % NS;
      const C *base = buf + line * LS;
#pragma unroll
      for (int i = 0; i < R; ++i) reg[q][i] = base[(j + i * M) * ES];
      if (NS > 1) {
#pragma unroll
        for (int i = 1; i < R; ++i) reg[q][i] = cmul(reg[q][i], tw[i * k * TWS]);
      }
      DFT<C, R>::run(reg[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = tid + q * NT;
    if (NB % NT == 0 || b < NB) {
      const int line = LINE_FAST ? b % NL : b / M;
      const int j = LINE_FAST ? b / NL : b % M;
      const int k = j % NS;
      const int o = (j / NS) * NS * R + k;
      C *base = buf + line * LS;
#pragma unroll
      for (int i = 0; i < R; ++i) base[(o + i * NS) * ES] = reg[q][i];
    }
  }
  __syncthreads();
  if constexpr (NS * R < N) fft_stages<C, N, NS * R, NL, LS, ES, LINE_FAST, NT>(buf, tw, tid);
}

template <typename C, int N, int NL, int LS, int ES, bool LINE_FAST, int NT>
__device__ __forceinline__ void lds_fft(C *buf, const C *tw, int tid) {
  if constexpr (N > 1) fft_stages<C, N, 1, NL, LS, ES, LINE_FAST, NT>(buf, tw, tid);
}

}  // namespace sgw
