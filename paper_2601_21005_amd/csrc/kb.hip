// Kleinman-Bylander projector contraction (the separable pseudopotential
// part, applied in the paper with atomic adds where neighbouring projector
// spheres overlap, Sec. 3).  Here the work is owned by 512-point grid tiles
// (16 x 8 x 4 where the grid allows it, else 8 x 8 x 8):
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

// the same with the x extent 2^LX known at compile time (y extent 8), in
// 32-bit arithmetic (grids below 2^31 points)
template <int LX>
__device__ __forceinline__ int tile_point_c(int base, int p, int nx, int ny) {
  const int x = p & ((1 << LX) - 1), y = (p >> LX) & 7, z = p >> (LX + 3);
  return base + x + nx * (y + ny * z);
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
  // unrolled so that several loads are in flight; the sum keeps its order
#pragma unroll 8
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
  auto add = [&](cplx<R> a, cplx<R> b) {
    sr += (double)a.x * b.x - (double)a.y * b.y;
    si += (double)a.x * b.y + (double)a.y * b.x;
  };
  // the inputs of eight q are requested before they are summed (in order of q)
  int q = 0;
  for (; q + 8 <= np; q += 8) {
    cplx<R> b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = in[(int64_t)(q + j) * nvec + v];
#pragma unroll
    for (int j = 0; j < 8; ++j) add(k[q + j], b[j]);
  }
  for (; q < np; ++q) add(k[q], in[(int64_t)q * nvec + v]);
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

// ---------------------------------------------------------------- MFMA
// Per tile the gather is the GEMM  D[e][c] = sum_p beta[e][p] Psi[p][c]
// (M = projector entries, K = 512 points, N = 2 NVB real columns = NVB
// complex vectors) and the scatter  D[p][c] = sum_e beta[e][p] C'[e][c]
// (M = 512 points, K = entries padded to the K group).  The operands are stored in
// FP32 (SGW_C64) or in BF16 rounded to nearest even (SGW_C64_BF16KB; with
// SGW_C64_BF16X2KB the psi / coefficient operand as two BF16 terms); the
// accumulation is FP32 either way.  A lane feeds 16 contiguous bytes of A and
// of B per group of K values:
//   FP32: four v_mfma_f32_16x16x4f32, K group 16, lane l holds the K slots
//         4 (l / 16) + s, s = 0..3, one per instruction;
//   BF16: one v_mfma_f32_16x16x32_bf16, K group 32, lane l holds the K slots
//         8 (l / 16) + s, s = 0..7;
// lane l supplies row l % 16 of A and column l % 16 of B and receives
// D[4 (l / 16) + r][l % 16] in accumulator register r.  Every variant below
// (vectors per workgroup NVB, entry tiles per pass MT) computes each output
// with the same instructions in the same order, so the choice changes the
// speed, not a bit of the result.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__host__ __device__ __forceinline__ uint32_t bf16_bits(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

struct OpF32 {
  using T = float;
  static constexpr int GK = 16;
  static constexpr bool SPLIT = false;
  __device__ static void mma(f32x4 &acc, const u32x4 &a, const u32x4 &b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[0]), __uint_as_float(b[0]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[1]), __uint_as_float(b[1]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[2]), __uint_as_float(b[2]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[3]), __uint_as_float(b[3]), acc, 0, 0, 0);
  }
  __device__ static void put2(T *d, float x, float y) {
    *reinterpret_cast<float2 *>(d) = make_float2(x, y);
  }
  __device__ static u32x4 pack(const float *e) {      // 4 values -> one operand
    return u32x4{__float_as_uint(e[0]), __float_as_uint(e[1]), __float_as_uint(e[2]),
                 __float_as_uint(e[3])};
  }
  __device__ static void put1(T *d, float x) { *d = x; }
};

struct OpBF16 {
  using T = uint16_t;
  static constexpr int GK = 32;
  static constexpr bool SPLIT = false;
  __device__ static void mma(f32x4 &acc, const u32x4 &a, const u32x4 &b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
  }
  __device__ static void put2(T *d, float x, float y) {
    *reinterpret_cast<uint32_t *>(d) = bf16_bits(x) | (bf16_bits(y) << 16);
  }
  __device__ static void put1(T *d, float x) { *d = (uint16_t)bf16_bits(x); }
  __device__ static u32x4 pack(const float *e) {      // 8 values -> one operand (RNE)
    return u32x4{bf16_bits(e[0]) | (bf16_bits(e[1]) << 16), bf16_bits(e[2]) | (bf16_bits(e[3]) << 16),
                 bf16_bits(e[4]) | (bf16_bits(e[5]) << 16), bf16_bits(e[6]) | (bf16_bits(e[7]) << 16)};
  }
};

__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// BF16 products with the state-vector operand (psi in the gather, the mixed
// coefficients in the scatter) carried as two BF16 terms hi + lo, hi = RNE(x),
// lo = RNE(x - hi): two MFMAs per operand pair, the split operand exact to
// about 2^-17; beta stays one BF16 term.
struct OpBF16x2 : OpBF16 {
  static constexpr bool SPLIT = true;
  __device__ static void pack2(const float *e, u32x4 &hi, u32x4 &lo) {
    uint32_t h[8], l[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      h[i] = bf16_bits(e[i]);
      l[i] = bf16_bits(e[i] - bf16_value(h[i]));
    }
    hi = u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
    lo = u32x4{l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16)};
  }
  __device__ static void put1x2(T *dhi, T *dlo, float x) {
    const uint32_t h = bf16_bits(x);
    *dhi = (uint16_t)h;
    *dlo = (uint16_t)bf16_bits(x - bf16_value(h));
  }
};

// Workgroup -> (tile, vector block).  Consecutive workgroups go to the 8
// XCDs in turn, so tile t is given to workgroups on XCD t % 8 only, and one
// XCD walks all vector blocks of a tile in a row: the tile's beta rows are
// read from memory once per XCD L2 instead of once per workgroup.
__device__ __forceinline__ bool tile_block(int ntile, int nvb, int &t, int64_t &vb) {
  const int b = blockIdx.x, xcd = b & 7, i = b >> 3;
  t = xcd + 8 * (i / nvb);
  vb = i % nvb;
  return t < ntile;
}

inline dim3 tile_grid(int ntile, int64_t nvb) {
  return dim3((unsigned)(8 * ((ntile + 7) / 8) * nvb));
}

template <class T> __device__ __forceinline__ u32x4 ld16(const T *p) {
  return *reinterpret_cast<const u32x4 *>(p);
}

// partial[off + e][v] = dV sum_p beta_e(p) psi_v(p) for the entries e of tile t.
// The B operand of lane (q, col) in K group g is EL consecutive tile points
// (consecutive x, so EL consecutive complex values in memory) of the real
// (col even) or imaginary (col odd) part of vector v0 + 8 n + col / 2: the
// lane reads them straight from memory (lanes col and col ^ 1 read the same
// bytes in the same instruction) -- no staging in LDS.  The tile's x extent
// is 2^LX (y 8).  Lanes of vectors past nvec read the last vector and entry
// rows past ne the last row: both only feed outputs that are never written,
// so the loads need no branch.
template <class Op, int NVB, int MT, int LX>
__global__ __launch_bounds__(NTK) void k_kb_gather_mma(
    const float2 *psi, int64_t ld, int64_t nvec, const int *tile_base, const int *tile_off,
    const typename Op::T *beta, float2 *partial, int nx, int ny, float dV, int ntile,
    int nvb, const uint32_t *__restrict__ tile_mask) {
  using T = typename Op::T;
  constexpr int NC = 2 * NVB, NTL = NC / 16;
  constexpr int EL = 16 / (int)sizeof(T);           // operand elements per lane per group
  constexpr int NG = 128 / Op::GK;                  // K groups of one wave (128 points)
  static_assert(Op::GK == 16 || Op::GK == 32, "K group of 16 or 32 points");
  constexpr int NS = Op::SPLIT ? NG : 1, NSN = Op::SPLIT ? NTL : 1;
  __shared__ __align__(16) float red[4 * MT * NTL * 256];   // cross-wave sums
  int t;
  int64_t vb;
  if (!tile_block(ntile, nvb, t, vb)) return;
  const int64_t v0 = vb * NVB;
  const int base = tile_base[t];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, col = lane & 15;
  const int off = tile_off[t], ne = tile_off[t + 1] - off;
  // bit g of glive: some point of this wave's K group g (GK consecutive tile
  // points) lies in a projector's support.  A group without one holds only
  // zero beta values: its psi values are not loaded and its products (exact
  // zeros) are not taken.  The condition is uniform over the wave.
  uint32_t glive = 0;
  const int wu = __builtin_amdgcn_readfirstlane(w);   // scalar loads of the four words
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t word = tile_mask[(int64_t)t * (KB_TP / 32) + 4 * wu + i];
    if constexpr (Op::GK == 16)
      glive |= ((word & 0xffffu) ? 1u : 0u) << (2 * i) | ((word >> 16) ? 1u : 0u) << (2 * i + 1);
    else
      glive |= (word ? 1u : 0u) << i;
  }
  glive = __builtin_amdgcn_readfirstlane(glive);
  auto live = [&](int g) { return (glive >> g) & 1u; };
  // B operands of this wave's quarter of K, kept in registers for all entries:
  // every load of a live group is issued first, the lane exchanges follow
  auto load_b = [&](int64_t v0, u32x4 (*b)[NTL], u32x4 (*blo)[NSN]) {
    constexpr int NZ = EL / 4;
    float4 z[NG][NTL][NZ];
    // the lane pair (col, col ^ 1) reads each group of 4 complex values once:
    // the even lane points 0, 1 and the odd lane points 2, 3
    const int od = col & 1;
#pragma unroll
    for (int n = 0; n < NTL; ++n) {
      const int64_t v = min(v0 + 8 * n + (col >> 1), nvec - 1);
      const float2 *src = psi + v * ld;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const int p = 128 * w + g * Op::GK + EL * q;  // EL consecutive points along x
        const float4 *s4 = reinterpret_cast<const float4 *>(src + tile_point_c<LX>(base, p, nx, ny));
#pragma unroll
        for (int i = 0; i < NZ; ++i) z[g][n][i] = live(g) ? s4[2 * i + od] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    // then they swap the parts the other needs (real parts to the even lane,
    // imaginary parts to the odd lane)
#pragma unroll
    for (int n = 0; n < NTL; ++n)
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        float e[EL];
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
          const float4 zz = z[g][n][i];
          const float g0 = __shfl_xor(od ? zz.x : zz.y, 1, 64);
          const float g1 = __shfl_xor(od ? zz.z : zz.w, 1, 64);
          e[4 * i] = od ? g0 : zz.x;
          e[4 * i + 1] = od ? g1 : zz.z;
          e[4 * i + 2] = od ? zz.y : g0;
          e[4 * i + 3] = od ? zz.w : g1;
        }
        if constexpr (Op::SPLIT) Op::pack2(e, b[g][n], blo[g][n]);
        else b[g][n] = Op::pack(e);
      }
  };
  // A operands (beta rows of MT entry tiles, one K group) alternate between
  // two register sets: group g + 1 is requested before the products of group
  // g (after the last group, the next pass's first one), so one group's loads
  // are in flight behind the products (three in flight, with a ring of four,
  // cost a wave per SIMD in registers and ran 5 % slower).  Entry rows past
  // ne read row ne - 1: in bounds, and their products are never stored.
  constexpr int D = 1, RA = 2;
  static_assert(NG % RA == 0, "the A operands alternate with the K groups");
  auto load_a = [&](int mg, int g, u32x4 *a) {
#pragma unroll
    for (int j = 0; j < MT; ++j) {
      const int e = min(mg + 16 * j + col, ne - 1);   // A row = lane % 16
      a[j] = ld16(beta + (int64_t)(off + e) * KB_TP + 128 * w + g * Op::GK + EL * q);
    }
  };
  u32x4 a[RA][MT];
#pragma unroll
  for (int g = 0; g < D; ++g)
    if (live(g)) load_a(0, g, a[g]);
  u32x4 b[NG][NTL], blo[NS][NSN];
  load_b(v0, b, blo);
  for (int mg = 0; mg < ne; mg += 16 * MT) {
    f32x4 acc[MT][NTL];
#pragma unroll
    for (int j = 0; j < MT; ++j)
#pragma unroll
      for (int n = 0; n < NTL; ++n) acc[j][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      if (live((g + D) % NG)) load_a(g + D < NG ? mg : mg + 16 * MT, (g + D) % NG, a[(g + D) % RA]);
      if (!live(g)) continue;
#pragma unroll
      for (int j = 0; j < MT; ++j)
        if (mg + 16 * j < ne)
#pragma unroll
          for (int n = 0; n < NTL; ++n) {
            Op::mma(acc[j][n], a[g % RA][j], b[g][n]);
            if constexpr (Op::SPLIT) Op::mma(acc[j][n], a[g % RA][j], blo[g][n]);
          }
    }
    // a barrier between the last products and the LDS writes of their
    // accumulators (without it the <8, 2> instantiation read some
    // accumulators before their last product had landed)
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MT; ++j)
#pragma unroll
      for (int n = 0; n < NTL; ++n)
        *reinterpret_cast<f32x4 *>(red + (((w * MT + j) * NTL + n) * 64 + lane) * 4) = acc[j][n];
    __syncthreads();
    // the four K quarters summed in wave order; one complex (entry, vector) per item
    for (int o = tid; o < MT * 16 * NVB; o += NTK) {
      const int j = o / (16 * NVB), er = (o / NVB) % 16, vl = o % NVB;
      const int e = mg + 16 * j + er;
      const int n = vl >> 3, lre = 16 * (er >> 2) + 2 * (vl & 7), r = er & 3;
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        const float *s = red + (((ww * MT + j) * NTL + n) * 64) * 4;
        re += s[lre * 4 + r];
        im += s[(lre + 1) * 4 + r];
      }
      if (e < ne && v0 + vl < nvec)
        partial[(int64_t)(off + e) * nvec + v0 + vl] = make_float2(dV * re, dV * im);
    }
    __syncthreads();
  }
}

// dst_v(r) += s1 sum_e beta_e(r) C'[p(e)][v] on the points r of tile t (s1 real).
// betaT holds each tile's block transposed, [512 points][nek entries], with the
// entry count nek padded to the K group (16 FP32, 32 BF16; zeros).  The
// coefficient columns sit in dynamic LDS with pitch pe = (largest nek of the
// context) + one 16-byte group, so the LDS a workgroup holds follows the
// projector density of the system, not the 256-entry limit.  A wave
// owns MJ M tiles of 16 points, so a workgroup covers 64 MJ points and a tile
// takes 512 / (64 MJ) workgroups per vector block (fewer registers per wave
// for MJ = 4, more waves per SIMD).  PF (always with one N tile): the old
// destination values are loaded first, so their latency overlaps the
// staging and the products (more registers, fewer waves per SIMD).
template <class Op, int NVB, int MJ, int LX, bool PF>
__device__ __forceinline__ void scatter_mma(
    const float2 *coef, int64_t nvec, const int *tile_base, const int *tile_off,
    const int *tile_offT, const int *entry_proj, const typename Op::T *betaT, float2 *dst,
    int64_t ld, float s1, int nx, int ny, int ntile, int nvb, int pe,
    const uint32_t *tile_mask) {
  using T = typename Op::T;
  constexpr int NC = 2 * NVB, NTL = NC / 16;
  constexpr int EL = 16 / (int)sizeof(T);
  constexpr int NH = KB_TP / (64 * MJ);             // workgroups per tile and vector block
  extern __shared__ __align__(16) unsigned char kb_lds[];
  T *sc = reinterpret_cast<T *>(kb_lds);            // C' [column][entry] (hi, lo), pitch pe
  int t;
  int64_t vbh;
  if (!tile_block(ntile, nvb * NH, t, vbh)) return;
  const int64_t vb = vbh / NH;
  const int p0 = (int)(vbh % NH) * 64 * MJ;       // first point of this workgroup
  const int64_t v0 = vb * NVB;
  const int off = tile_off[t], ne = tile_off[t + 1] - off;
  const int offT = tile_offT[t], nek = tile_offT[t + 1] - offT;
  const int base = tile_base[t];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, col = lane & 15;
  // The products are taken transposed, D'[column][point] = sum_e C'[e][column]
  // beta_e(point) (C' from LDS as the A operand, betaT as B): lane l then
  // holds D'[4 (l / 16) + r][l % 16], i.e. the real and imaginary parts of
  // vectors 8 n + 2 (l / 16) (r = 0, 1) and + 1 (r = 2, 3) at point l % 16 of
  // the M tile: two complete complex values, stored without a lane exchange.
  // Lanes of vectors past nvec read the last vector and store nothing.
  const int cg = q;                                 // column group: vectors 2 cg, 2 cg + 1
  int rp[MJ];
#pragma unroll
  for (int j = 0; j < MJ; ++j)
    rp[j] = tile_point_c<LX>(base, p0 + 16 * (MJ * w + j) + col, nx, ny);
  // support bits: M tile j (16 points) with none is skipped by the whole wave
  // (no products, no read or write of psi there: the update is an exact
  // zero).  A live M tile is read and written whole: with 16 x 8 x 4 tiles it
  // is one 128-byte row of each vector, and storing only its supported
  // points would leave partly written cache lines that the next pass over
  // psi pays for.
  uint32_t rowbits[MJ];
  bool live[MJ];
#pragma unroll
  for (int j = 0; j < MJ; ++j) {
    const int pj = p0 + 16 * (MJ * w + j);
    const uint32_t word = __builtin_amdgcn_readfirstlane(
        tile_mask[(int64_t)t * (KB_TP / 32) + (pj >> 5)]);
    rowbits[j] = (word >> (pj & 31)) & 0xffffu;
    live[j] = rowbits[j] != 0u;
  }
  float2 *vrow[NTL][2];
  bool vok[NTL][2];
#pragma unroll
  for (int n = 0; n < NTL; ++n)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t v = v0 + 8 * n + 2 * cg + u;
      vok[n][u] = v < nvec;
      vrow[n][u] = dst + min(v, nvec - 1) * ld;
    }
  // with one N tile, or PF, the old destination values are loaded here, before
  // the staging, so their memory latency overlaps it and the products
  constexpr bool PREFETCH = NTL == 1 || PF;
  float2 o[MJ][NTL][2];
  if constexpr (PREFETCH) {
#pragma unroll
    for (int j = 0; j < MJ; ++j)
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        o[j][n][0] = live[j] ? vrow[n][0][rp[j]] : make_float2(0.f, 0.f);
        o[j][n][1] = live[j] ? vrow[n][1][rp[j]] : make_float2(0.f, 0.f);
      }
  }
  // betaT rows of this wave's points: the first K group is loaded before the
  // coefficient staging, so its latency overlaps that of the staging loads
  const T *bt =
      betaT + (int64_t)offT * KB_TP + (int64_t)(p0 + 16 * MJ * w + col) * nek + EL * q;
  constexpr int NS = Op::SPLIT ? 2 : 1;            // C' terms (hi, lo)
  u32x4 a_cur[MJ], a_nxt[MJ], b_cur[NS][NTL], b_nxt[NS][NTL];
  if (nek > 0) {
#pragma unroll
    for (int j = 0; j < MJ; ++j) a_cur[j] = ld16(bt + (int64_t)(16 * j) * nek);
  }
  // C' rows of this tile's entries (zero from ne up to nek), four loads in flight
  for (int i0 = 0; i0 < nek * NVB; i0 += 4 * NTK) {
    float2 val[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * NTK + tid, el = idx / NVB, vl = idx % NVB;
      val[u] = make_float2(0.f, 0.f);
      if (el < ne && v0 + vl < nvec) val[u] = coef[(int64_t)entry_proj[off + el] * nvec + v0 + vl];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * NTK + tid, el = idx / NVB, vl = idx % NVB;
      if (el < nek) {
        if constexpr (Op::SPLIT) {
          Op::put1x2(sc + (2 * vl) * pe + el, sc + NC * pe + (2 * vl) * pe + el, val[u].x);
          Op::put1x2(sc + (2 * vl + 1) * pe + el, sc + NC * pe + (2 * vl + 1) * pe + el, val[u].y);
        } else {
          Op::put1(sc + (2 * vl) * pe + el, val[u].x);
          Op::put1(sc + (2 * vl + 1) * pe + el, val[u].y);
        }
      }
    }
  }
  __syncthreads();
  // wave w owns the M tiles (16 points each) MJ w .. MJ w + MJ - 1 from p0
  f32x4 acc[MJ][NTL];
#pragma unroll
  for (int j = 0; j < MJ; ++j)
#pragma unroll
    for (int n = 0; n < NTL; ++n) acc[j][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto load_b = [&](int k0, u32x4 (*b)[NTL]) {
#pragma unroll
    for (int h = 0; h < NS; ++h)
#pragma unroll
      for (int n = 0; n < NTL; ++n)
        b[h][n] = ld16(sc + h * NC * pe + (16 * n + col) * pe + k0 + EL * q);
  };
  auto load_group = [&](int k0, u32x4 *a, u32x4 (*b)[NTL]) {
#pragma unroll
    for (int j = 0; j < MJ; ++j) a[j] = ld16(bt + (int64_t)(16 * j) * nek + k0);
    load_b(k0, b);
  };
  if (nek > 0) load_b(0, b_cur);                  // a_cur holds group 0 already
  for (int k0 = 0; k0 < nek; k0 += Op::GK) {
    if (k0 + Op::GK < nek) load_group(k0 + Op::GK, a_nxt, b_nxt);
#pragma unroll
    for (int j = 0; j < MJ; ++j)
      if (rowbits[j])
#pragma unroll
        for (int n = 0; n < NTL; ++n)
#pragma unroll
          for (int h = 0; h < NS; ++h) Op::mma(acc[j][n], b_cur[h][n], a_cur[j]);
#pragma unroll
    for (int j = 0; j < MJ; ++j) a_cur[j] = a_nxt[j];
#pragma unroll
    for (int h = 0; h < NS; ++h)
#pragma unroll
      for (int n = 0; n < NTL; ++n) b_cur[h][n] = b_nxt[h][n];
  }
  if constexpr (!PREFETCH) {
#pragma unroll
    for (int j = 0; j < MJ; ++j)
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        o[j][n][0] = live[j] ? vrow[n][0][rp[j]] : make_float2(0.f, 0.f);
        o[j][n][1] = live[j] ? vrow[n][1][rp[j]] : make_float2(0.f, 0.f);
      }
  }
#pragma unroll
  for (int j = 0; j < MJ; ++j)
#pragma unroll
    for (int n = 0; n < NTL; ++n) {
      const f32x4 d = acc[j][n];
      if (live[j] && vok[n][0])
        vrow[n][0][rp[j]] = make_float2(o[j][n][0].x + s1 * d[0], o[j][n][0].y + s1 * d[1]);
      if (live[j] && vok[n][1])
        vrow[n][1][rp[j]] = make_float2(o[j][n][1].x + s1 * d[2], o[j][n][1].y + s1 * d[3]);
    }
}

template <class Op, int NVB, int MJ, int LX, bool PF>
__global__ __launch_bounds__(NTK) void k_kb_scatter_mma(
    const float2 *coef, int64_t nvec, const int *tile_base, const int *tile_off,
    const int *tile_offT, const int *entry_proj, const typename Op::T *betaT, float2 *dst,
    int64_t ld, float s1, int nx, int ny, int ntile, int nvb, int pe,
    const uint32_t *tile_mask) {
  scatter_mma<Op, NVB, MJ, LX, PF>(coef, nvec, tile_base, tile_off, tile_offT, entry_proj, betaT, dst, ld, s1, nx, ny, ntile, nvb, pe, tile_mask);
}

// the same code held to 64 registers per lane, i.e. eight waves per SIMD (the
// accumulators then sit in ordinary vector registers): instantiated for the
// variants of two M tiles per wave, which fit without spilling in FP32 and
// BF16 (the split-BF16 instances spill a few registers; the tuner weighs that)
template <class Op, int NVB, int MJ, int LX, bool PF>
__global__ __launch_bounds__(NTK) __attribute__((amdgpu_waves_per_eu(8, 8))) void
k_kb_scatter_mma_w8(
    const float2 *coef, int64_t nvec, const int *tile_base, const int *tile_off,
    const int *tile_offT, const int *entry_proj, const typename Op::T *betaT, float2 *dst,
    int64_t ld, float s1, int nx, int ny, int ntile, int nvb, int pe,
    const uint32_t *tile_mask) {
  scatter_mma<Op, NVB, MJ, LX, PF>(coef, nvec, tile_base, tile_off, tile_offT, entry_proj, betaT, dst, ld, s1, nx, ny, ntile, nvb, pe, tile_mask);
}

// variants (autotuned per context, operand type and batch width)
// (w: the instance held to that many waves per SIMD, 0: the compiler's
// choice; the tuner keeps the first variant within 3 % of the fastest, so a
// held instance comes before its twin)
struct GatherVariant { int nvb, mt; };
static const GatherVariant kGather[] = {{8, 2}, {8, 4}, {16, 2}, {16, 4}};
struct ScatterVariant { int nvb, mj, pf, w; };
static const ScatterVariant kScatter[] = {{8, 8, 0, 0}, {16, 8, 0, 0}, {8, 4, 0, 0},
                                          {16, 4, 0, 0}, {8, 2, 0, 8}, {8, 2, 0, 0},
                                          {16, 2, 0, 8}, {16, 2, 0, 0}, {16, 2, 1, 0}};
constexpr int NGATHER = 4, NSCATTER = 9;

template <class Op>
static void launch_gather_variant(int vi, dim3 g, hipStream_t st, const float2 *psi, int64_t ld,
                                  int64_t nvec, const int *tb, const int *to,
                                  const typename Op::T *beta, float2 *partial, int nx, int ny,
                                  int lx, float dV, int ntile, int nvb, const uint32_t *mask) {
  const GatherVariant v = kGather[vi];
#define SGW_G(A, B, X)                                                                           \
  if (v.nvb == A && v.mt == B && lx == X)                                                        \
    hipLaunchKernelGGL((k_kb_gather_mma<Op, A, B, X>), g, dim3(NTK), 0, st, psi, ld, nvec, tb,  \
                       to, beta, partial, nx, ny, dV, ntile, nvb, mask);
  SGW_G(8, 2, 4) SGW_G(8, 4, 4) SGW_G(16, 2, 4) SGW_G(16, 4, 4)
  SGW_G(8, 2, 3) SGW_G(8, 4, 3) SGW_G(16, 2, 3) SGW_G(16, 4, 3)
#undef SGW_G
}

template <class Op>
static void launch_scatter_variant(int vi, dim3 g, hipStream_t st, const float2 *coef,
                                   int64_t nvec, const int *tb, const int *to, const int *toT,
                                   const int *ep, const typename Op::T *betaT, float2 *dst,
                                   int64_t ld, float s1, int nx, int ny, int lx, int ntile,
                                   int nvb, int nek_max, const uint32_t *mask) {
  const ScatterVariant v = kScatter[vi];
  constexpr int EL = 16 / (int)sizeof(typename Op::T);
  const int pe = nek_max + EL;
  const size_t lds = (Op::SPLIT ? 2 : 1) * 2 * (size_t)v.nvb * pe * sizeof(typename Op::T);
#define SGW_S(A, B, X, F, W, K)                                                                  \
  if (v.nvb == A && v.mj == B && v.pf == F && v.w == W && lx == X)                               \
    hipLaunchKernelGGL((K<Op, A, B, X, F>), g, dim3(NTK), lds, st, coef, nvec, tb, to, toT, ep, \
                       betaT, dst, ld, s1, nx, ny, ntile, nvb, pe, mask);
  SGW_S(8, 8, 4, 0, 0, k_kb_scatter_mma) SGW_S(16, 8, 4, 0, 0, k_kb_scatter_mma)
  SGW_S(8, 4, 4, 0, 0, k_kb_scatter_mma) SGW_S(16, 4, 4, 0, 0, k_kb_scatter_mma)
  SGW_S(8, 2, 4, 0, 0, k_kb_scatter_mma) SGW_S(16, 2, 4, 0, 0, k_kb_scatter_mma)
  SGW_S(16, 2, 4, 1, 0, k_kb_scatter_mma)
  SGW_S(8, 2, 4, 0, 8, k_kb_scatter_mma_w8) SGW_S(16, 2, 4, 0, 8, k_kb_scatter_mma_w8)
  SGW_S(8, 8, 3, 0, 0, k_kb_scatter_mma) SGW_S(16, 8, 3, 0, 0, k_kb_scatter_mma)
  SGW_S(8, 4, 3, 0, 0, k_kb_scatter_mma) SGW_S(16, 4, 3, 0, 0, k_kb_scatter_mma)
  SGW_S(8, 2, 3, 0, 0, k_kb_scatter_mma) SGW_S(16, 2, 3, 0, 0, k_kb_scatter_mma)
  SGW_S(16, 2, 3, 1, 0, k_kb_scatter_mma)
  SGW_S(8, 2, 3, 0, 8, k_kb_scatter_mma_w8) SGW_S(16, 2, 3, 0, 8, k_kb_scatter_mma_w8)
#undef SGW_S
}

// Operand arrays of the MFMA kernels: beta per entry [entry][512] in the
// operand type (BF16 only; FP32 uses the working-precision copy) and the
// transposed per-tile blocks [512][nek], nek = entries rounded up to the
// scatter's K group.
void kb_upload_operands(sgw_ctx *ctx) {
  const KBHost &kb = ctx->kb;
  auto upload = [](DevBuf &b, const auto *src, size_t n) {
    b.ensure(n * sizeof(*src));
    SGW_HIP(hipMemcpy(b.p, src, n * sizeof(*src), hipMemcpyHostToDevice));
  };
  const int nt = (int)kb.tile_base.size();
  const bool bf = ctx->prec == SGW_C64_BF16KB || ctx->prec == SGW_C64_BF16X2KB;
  const int kg = bf ? OpBF16::GK : OpF32::GK;      // the scatter's K group
  std::vector<int> offT(nt + 1, 0);
  ctx->kb_nek_max = 0;
  for (int t = 0; t < nt; ++t) {
    const int ne = kb.tile_off[t + 1] - kb.tile_off[t];
    offT[t + 1] = offT[t] + (ne + kg - 1) / kg * kg;
    ctx->kb_nek_max = std::max(ctx->kb_nek_max, offT[t + 1] - offT[t]);
  }
  upload(ctx->d_kb_tile_offT, offT.data(), offT.size());
  const size_t nT = (size_t)offT[nt] * KB_TP;
  auto fill_T = [&](auto *out, auto conv) {
    for (int t = 0; t < nt; ++t) {
      const int e0 = kb.tile_off[t], ne = kb.tile_off[t + 1] - e0, nek = offT[t + 1] - offT[t];
      auto *blk = out + (size_t)offT[t] * KB_TP;
      for (int p = 0; p < KB_TP; ++p)
        for (int e = 0; e < ne; ++e) blk[(size_t)p * nek + e] = conv(kb.beta[(size_t)(e0 + e) * KB_TP + p]);
    }
  };
  if (bf) {
    auto conv = [](double v) { return (uint16_t)bf16_bits((float)v); };
    std::vector<uint16_t> t16(nT, 0);
    fill_T(t16.data(), conv);
    upload(ctx->d_kb_betaT, t16.data(), t16.size());
    std::vector<uint16_t> b16(kb.beta.size());
    for (size_t i = 0; i < b16.size(); ++i) b16[i] = conv(kb.beta[i]);
    upload(ctx->d_kb_beta16, b16.data(), b16.size());
  } else {
    std::vector<float> tf(nT, 0.f);
    fill_T(tf.data(), [](double v) { return (float)v; });
    upload(ctx->d_kb_betaT, tf.data(), tf.size());
  }
}

// ---------------------------------------------------------------- launchers
template <typename R>
static void gather_t(sgw_ctx *ctx, const void *psi, int64_t nvec, int64_t ld, void *out,
                     bool use_e, void *partial_ext) {
  constexpr int NV = KBV<R>::NV;
  using C = cplx<R>;
  C *partial = partial_ext ? static_cast<C *>(partial_ext)
                           : ctx->buf("kb_partial", sizeof(C) * (size_t)ctx->kb_nentry * nvec).as<C>();
  SGW_REQUIRE(ctx->kb_ntile <= 65535, SGW_EUNSUPPORTED, "KB gather: too many tiles");
  if constexpr (sizeof(R) == 4) {
    SGW_REQUIRE(ld % 2 == 0, SGW_EUNSUPPORTED,
                "projectors in complex FP32 need an even leading dimension");
    SGW_REQUIRE(ctx->kb_ly == 3 && (ctx->kb_lx == 3 || ctx->kb_lx == 4), SGW_EUNSUPPORTED,
                "KB tile shape not built");
    auto go = [&](auto op, const char *name, const auto *beta) {
      using Op = decltype(op);
      auto run = [&](int vi) {
        const int64_t nvb = (nvec + kGather[vi].nvb - 1) / kGather[vi].nvb;
        launch_gather_variant<Op>(vi, tile_grid(ctx->kb_ntile, nvb), ctx->stream,
                                  static_cast<const float2 *>(psi), ld, nvec,
                                  ctx->d_kb_tile_base.as<int>(), ctx->d_kb_tile_off.as<int>(),
                                  beta, reinterpret_cast<float2 *>(partial), ctx->nx, ctx->ny,
                                  ctx->kb_lx, (float)ctx->dV, ctx->kb_ntile,
                                  (int)nvb, ctx->d_kb_mask.as<uint32_t>());
      };
      const int vi = ctx->tune(name, nvec, NGATHER, run);   // the gather overwrites: trials are harmless
      const bool timed = (ctx->ktimer & 4) && ctx->ns.empty();
      if (timed) SGW_HIP(hipEventRecord(ctx->kt[2].event(0), ctx->stream));
      run(vi);
      if (timed) {
        SGW_HIP(hipEventRecord(ctx->kt[2].event(1), ctx->stream));
        ctx->kt[2].used++;
        ctx->kt[2].points += (int64_t)ctx->kb_ntile * KB_TP * nvec;
      }
    };
    if (ctx->prec == SGW_C64_BF16KB)
      go(OpBF16{}, "kb_gather_bf16", ctx->d_kb_beta16.as<uint16_t>());
    else if (ctx->prec == SGW_C64_BF16X2KB)
      go(OpBF16x2{}, "kb_gather_bf16x2", ctx->d_kb_beta16.as<uint16_t>());
    else
      go(OpF32{}, "kb_gather", ctx->d_kb_beta.as<float>());
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
  if (ctx->dbl) gather_t<double>(ctx, psi, nvec, ld, coef_out, false, nullptr);
  else gather_t<float>(ctx, psi, nvec, ld, coef_out, false, nullptr);
}

void kb_gather_e(sgw_ctx *ctx, const void *psi, int64_t nvec, int64_t ld, void *coef_out,
                 void *partial) {
  if (ctx->dbl) gather_t<double>(ctx, psi, nvec, ld, coef_out, true, partial);
  else gather_t<float>(ctx, psi, nvec, ld, coef_out, true, partial);
}

size_t kb_partial_bytes_per_vec(const sgw_ctx *ctx) {
  return ctx->csize() * (size_t)ctx->kb_nentry;
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
    SGW_REQUIRE(dst2 == nullptr && s1im == 0.0, SGW_EUNSUPPORTED,
                "KB scatter (FP32): complex scale or second output not built");
    SGW_REQUIRE(ctx->kb_ly == 3 && (ctx->kb_lx == 3 || ctx->kb_lx == 4), SGW_EUNSUPPORTED,
                "KB tile shape not built");
    auto go = [&](auto op, const char *name, const auto *betaT) {
      using Op = decltype(op);
      auto launch = [&](int vi, float s) {
        const ScatterVariant &sv = kScatter[vi];
        const int64_t nvb = (nvec + sv.nvb - 1) / sv.nvb;
        const int64_t nh = KB_TP / (64 * sv.mj);
        launch_scatter_variant<Op>(vi, tile_grid(ctx->kb_ntile, nvb * nh), ctx->stream,
                                   static_cast<const float2 *>(coef), nvec,
                                   ctx->d_kb_tile_base.as<int>(), ctx->d_kb_tile_off.as<int>(),
                                   ctx->d_kb_tile_offT.as<int>(), ctx->d_kb_entry_proj.as<int>(),
                                   betaT, static_cast<float2 *>(dst), ld, s, ctx->nx, ctx->ny,
                                   ctx->kb_lx, ctx->kb_ntile, (int)nvb, ctx->kb_nek_max,
                                   ctx->d_kb_mask.as<uint32_t>());
      };
      // trials add 0 * (B C) to dst, which leaves it unchanged
      const int vi = ctx->tune(name, nvec, NSCATTER, [&](int i) { launch(i, 0.0f); });
      const bool timed = (ctx->ktimer & 2) && ctx->ns.empty();
      if (timed) SGW_HIP(hipEventRecord(ctx->kt[1].event(0), ctx->stream));
      launch(vi, (float)s1re);
      if (timed) {
        SGW_HIP(hipEventRecord(ctx->kt[1].event(1), ctx->stream));
        ctx->kt[1].used++;
        ctx->kt[1].points += (int64_t)ctx->kb_ntile * KB_TP * nvec;
      }
    };
    if (ctx->prec == SGW_C64_BF16KB)
      go(OpBF16{}, "kb_scatter_bf16", ctx->d_kb_betaT.as<uint16_t>());
    else if (ctx->prec == SGW_C64_BF16X2KB)
      go(OpBF16x2{}, "kb_scatter_bf16x2", ctx->d_kb_betaT.as<uint16_t>());
    else
      go(OpF32{}, "kb_scatter", ctx->d_kb_betaT.as<float>());
    SGW_HIP(hipGetLastError());
    return;
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
