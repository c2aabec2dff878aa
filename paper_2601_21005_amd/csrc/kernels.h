// Launchers of the elementwise, reduction, TDH and sROI kernels.
#pragma once

#include "common.h"

namespace sgw {

bool fft_size_supported(int n, bool dbl);
bool fft_pencils_cover(int nx, int ny, int nz, bool dbl);

// ---- vectors
// acc[v] = (cre + i cim) x[v]
void launch_scale_copy(sgw_ctx *ctx, const void *x, int64_t ldx, void *acc, int64_t lda,
                       int64_t nvec, double cre, double cim);
// acc[v] += (cre + i cim) x[v]
void launch_axpy(sgw_ctx *ctx, const void *x, int64_t ldx, void *acc, int64_t lda,
                 int64_t nvec, double cre, double cim);
// acc[v] (= when assign, else +=) c0 a[v] + c1 b[v]  (common leading dimension ld)
void launch_axpy2(sgw_ctx *ctx, const void *a, const void *b, int64_t ld, void *acc,
                  int64_t nvec, double c0r, double c0i, double c1r, double c1i, bool assign);
// Several sums over one Chebyshev recurrence (the zeta sweep): for g < G,
// acc_g[v] (= when assign, else +=) c0_g a[v] + c1_g b[v] (b nullable); all
// vectors N apart, the accumulators G-major (acc + (g nvec + v) N).
constexpr int kMaxSweep = 8;
constexpr int kSweepGroup = 8;   // terms per accumulation of a sweep
// a group of up to kSweepGroup terms x_j and their coefficients for the G
// sums (c[g][2 j], c[g][2 j + 1]: re, im)
struct ChebAccTerms {
  const void *x[kSweepGroup];
  double c[kMaxSweep][2 * kSweepGroup];
};
void launch_cheb_accs(sgw_ctx *ctx, const ChebAccTerms &t, int nterm, void *acc, int64_t nvec,
                      int G, bool assign);
// dst[v] = src[v]
void launch_copy(sgw_ctx *ctx, const void *src, int64_t lds, void *dst, int64_t ldd,
                 int64_t nvec);
// out[v] = sum_r |x_v(r)|^2 (FP64, deterministic two-stage)
void launch_norm2(sgw_ctx *ctx, const void *x, int64_t ld, int64_t nvec, double *d_out);
// out[f] = sum_r Re(conj(a_f(r)) b_f(r))  (FP64)
void launch_redot(sgw_ctx *ctx, const void *a, const void *b, int64_t ld, int64_t nf,
                  double *d_out);

// ---- white noise and unpacking (sgw_sigma_estimate)
// Filter input: complex vector k carries real noise vectors 2k and 2k+1 of the
// flat list keys[0..nr-1] (+-1/sqrt(dV)).
void launch_fill_noise(sgw_ctx *ctx, const uint64_t *d_keys, int64_t nr, void *out);
struct UnpackArgs {
  const void *filt;        // [nc][N] complex, filtered
  const uint64_t *keys;    // [nr] noise keys (zeta-bar of sample s at s (1+neta))
  const void *phi;         // [N] real
  void *psi;               // [S][ncopy][neta] vectors ldp apart: copy 0 <- eta (nullable)
  void *zeta;              // [S][2][N] complex: zeta^+ = zb - F zb, zeta~ = F zb
                           // (nullable)
  void *kick;              // [S][N] complex: phi zb
  void *xsrc;              // [S][neta/2][N] complex: phi eta_2k + i phi eta_2k+1
  int S = 0, neta = 0, ncopy = 2;
  int64_t ldp = 0;         // psi leading dimension (0: N)
};
void launch_unpack(sgw_ctx *ctx, const UnpackArgs &a);

// ---- TDH
// psi [S][1 + nk][neta] vectors ld apart; dv, u [nk][S][N]; v [S][N];
// rho [1 + nk/2][S][N]
void launch_tdh_tangent(sgw_ctx *ctx, void *psi, int64_t ld, const void *dv, int S, int neta,
                        int nk);
void launch_tdh_local(sgw_ctx *ctx, void *psi, int64_t ld, const void *v, const void *u, int S,
                      int neta, int nk, double a);
void launch_tdh_density(sgw_ctx *ctx, const void *psi, int64_t ld, void *rho, int S, int neta,
                        int nk, double w);
void launch_bcast_real(sgw_ctx *ctx, const void *src, void *dst, int S);

// ---- sROI
void launch_xi_supports(sgw_ctx *ctx, const uint64_t *d_keys, int S, int n_xi, int nseg,
                        int *blocks);
// cR[(s (n_t) + j) n_xi + m] = amp dV <xi_m|u_s>; the offset is out_off, plus
// step_dev[0] * step_stride when step_dev is given (a graph's step counter)
void launch_xi_real(sgw_ctx *ctx, const void *u, const int *blocks, const uint64_t *d_sign_keys,
                    int S, int n_xi, int nseg, double amp_dv, void *out, int64_t out_stride_s,
                    int64_t out_off, const int *step_dev = nullptr, int64_t step_stride = 0);
// d_counter[idx] = value (add: += value), one lane
void launch_counter(sgw_ctx *ctx, int idx, int value, bool add);
// dp[s][m] = amp dV <xi_m|phi zeta_s0>, dt[s][m] = amp dV <xi_m|phi zeta_s1>
void launch_xi_zeta(sgw_ctx *ctx, const void *zeta, const void *phi, const int *blocks,
                    const uint64_t *d_sign_keys, int S, int n_xi, int nseg, double amp_dv,
                    void *dp, void *dt);
// time ordering of rows: in real, out complex, element (row, j) at
// base(row) + j * stride with base(row) = (row / n_inner) * nt1 * n_inner + row % n_inner
bool launch_time_order(sgw_ctx *ctx, const void *in, void *out, int64_t nrows,
                       int64_t n_inner, int nt1, int nft, const void *d_tw);
// sig_p[s][j] += sum_m c[s][j][m] dp[s][m];  sig_m[s][j] += sum_m c (-conj dt)
// steps j .. j + nsteps - 1 in one launch, their overlaps dstride elements apart
void launch_contract_xi(sgw_ctx *ctx, const void *cto, const void *dp, const void *dt,
                        int S, int n_xi, int nt1, int j, double *d_sig, int nsteps = 1,
                        int64_t dstride = 0);
// exact mode: sig[s][j] (+: dV sum phi z+ u ; -: -dV sum phi conj(z~) u)
void launch_contract_exact(sgw_ctx *ctx, const void *uto, const void *zeta, const void *phi,
                           int S, int nt1, int j, double *d_partial, double *d_sig);

}  // namespace sgw
