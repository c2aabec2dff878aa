/*
 * sgw.h -- C ABI of the MI355X stochastic-GW hot-path library (libsgw).
 *
 * The library applies the Kohn-Sham Hamiltonian of Eq. (1) on a periodic
 * real-space grid to large batches of stochastic orbitals and runs the three
 * loops built on it in arXiv 2601.21005 (StochasticGW-GPU): the Chebyshev
 * occupied-space filter of Eq. (3), the time-dependent-Hartree linear
 * response that builds W (Sec. 2.1, first phase), and the propagation of the
 * stochastic Green's-function orbitals of Eq. (4) with the sROI contraction
 * of Eq. (5); Eq. (6) and Eq. (7) give the QP energy.
 *
 * Conventions shared by every call
 *  - Units are Hartree atomic units.
 *  - Grid: points r = h (ix, iy, iz), flat index ix + nx (iy + ny iz),
 *    periodic box of nx h x ny h x nz h bohr.  <f|g> = h^3 sum conj(f) g.
 *  - Precision SGW_C128: device vectors are interleaved complex double
 *    (16 B per point); SGW_C64 and SGW_C64_BF16KB: interleaved complex float
 *    (8 B per point).  Real fields (densities, potentials) are double resp.
 *    float.
 *  - A batch of nvec device vectors is nvec consecutive blocks of ld >= N_g
 *    complex elements (N_g = nx ny nz); pointers are caller-owned HIP device
 *    pointers, 16-byte aligned.  Host pointers are marked "host".
 *  - Every call enqueues its work on the context's stream; calls that return
 *    host results synchronise that stream before returning.
 *  - Errors are returned as sgw_status; nothing aborts or throws across the
 *    ABI.  sgw_last_error() gives the message of the last failing call made
 *    on that context (or of the last failing sgw_create in this thread).
 *  - One context per stream; calls on one context must not overlap.
 */
#ifndef SGW_H
#define SGW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgw_ctx sgw_ctx;

typedef enum {
  SGW_OK = 0,
  SGW_EINVAL = -1,        /* invalid argument (size, pointer, non-finite input) */
  SGW_ENOMEM = -2,        /* device or host allocation failed */
  SGW_EHIP = -3,          /* a HIP runtime call failed */
  SGW_EDIVERGED = -4,     /* a Chebyshev recurrence grew: bounds too narrow */
  SGW_ENOROOT = -5,       /* the QP equation has no root in the search window */
  SGW_EUNSUPPORTED = -6   /* grid size or option not built into this library */
} sgw_status;

typedef enum {
  SGW_C128 = 0,           /* complex double throughout */
  SGW_C64 = 1,            /* complex float; FP64 coefficients and sums */
  SGW_C64_BF16KB = 2,     /* as SGW_C64, but the projector GEMMs take their operands
                           * (beta, psi, the mixed coefficients) rounded to BF16
                           * (nearest even) with FP32 accumulation on MFMA */
  SGW_C64_BF16X2KB = 3    /* as SGW_C64_BF16KB, but psi and the mixed coefficients
                           * enter as two BF16 terms (hi + lo, two MFMAs); beta is
                           * one BF16 term */
} sgw_precision;

/* Grid (Eq. 1 on a Fourier grid, Sec. 2.2).  ecut > 0 clips the kinetic
 * energy T(k) = |k|^2/2 at ecut (Sec. 3 applies such a cutoff to the kinetic
 * operator); ecut <= 0 leaves it unclipped.  Each of nx, ny, nz must be one
 * of the built FFT lengths (8, 12, 16, 24, 32, 40, 48, 56, 64, 80, 96, 112,
 * 128, 160), with nx == ny and nx a multiple of the z pencils' width (16 when
 * nz % 16 == 0, else 8 when nz % 8 == 0, else 4); otherwise SGW_EUNSUPPORTED.
 * The x and y transforms run on whole xy planes in LDS when a plane fits
 * (n <= 80 in complex FP32, n <= 56 in complex FP64), else on x lines and y
 * pencils (one more pass over the batch, same results). */
typedef struct {
  int32_t nx, ny, nz;
  double h;               /* grid spacing, bohr */
  double ecut;            /* kinetic cutoff, Ha (<= 0: none) */
} sgw_grid;

/* Kleinman-Bylander projectors (the separable non-local pseudopotential part
 * whose neighbouring spheres overlap, Sec. 3).  Projector p sits on atom
 * a(p) (CSR: projectors proj_begin[a] .. proj_begin[a+1]-1 belong to atom a)
 * with angular channel l in {0, 1} and component m (l = 1: 0 = x, 1 = y,
 * 2 = z):
 *     beta_p(r) = N_p Y_lm(d) exp(-|d|^2 / (2 rc^2)),  |d| <= rcut_over_rc rc,
 *     Y_00 = 1, Y_1m = d_m,  d = minimum-image r - R_a,
 * N_p normalising <beta_p|beta_p> = 1 on the grid, and
 *     V_NL = sum_p |beta_p> ekb_p <beta_p|.
 * All arrays are host arrays, copied by sgw_create. */
typedef struct {
  int32_t natom;
  const double *pos;          /* host [natom][3], bohr */
  const int32_t *proj_begin;  /* host [natom + 1] */
  const int32_t *l;           /* host [nproj] */
  const int32_t *m;           /* host [nproj] */
  const double *rc;           /* host [nproj], bohr */
  const double *ekb;          /* host [nproj], Ha */
  double rcut_over_rc;        /* support radius in units of rc (> 0) */
} sgw_projectors;

/* Create a context: H = T + V_loc + V_NL on the grid (Eq. 1).  v_loc is a
 * host [N_g] array (Ha, x fastest) holding the whole local potential;
 * projectors may be NULL (local-only H).  hip_stream is a hipStream_t (NULL
 * = the null stream).  max_nvec bounds the batch of the vector-level calls
 * (sgw_apply_H, sgw_fermi_filter, sgw_cheb_propagate process larger batches
 * in chunks of max_nvec); the context's scratch is sized from it.  All host
 * inputs are copied.  On failure *out is NULL and the message is available
 * from sgw_last_error(NULL).
 * Switches read from the environment here (tuning and testing):
 *   SGW_ZETA_OVERLAP=0  the zeta propagation of sgw_sigma_estimate runs after
 *                       the TDH steps on the context's stream (bitwise the
 *                       same results);
 *   SGW_KB_OVERLAP=0    the Chebyshev terms' projector gathers stay on the
 *                       context's stream (bitwise the same results);
 *   SGW_ZETA_SWEEP=G    zeta output steps per Chebyshev sweep (1 .. 8);
 *   SGW_KB_MASK=0       the projector kernels process every row of a touched
 *                       tile (bitwise the same results);
 *   SGW_FILTER_CHUNK=n  sgw_sigma_estimate filters n vectors at a time;
 *   SGW_FORCE_VARIANT="name=i,..."  pins autotuned kernel variants (every
 *                       variant of a kernel gives the same bits);
 *   SGW_TUNE_CACHE=path keeps the autotuner's choices in a JSON file, read
 *                       at the first tuning and rewritten after each new one. */
sgw_status sgw_create(const sgw_grid *grid, const double *v_loc,
                      const sgw_projectors *projectors, sgw_precision prec,
                      void *hip_stream, int64_t max_nvec, sgw_ctx **out);

/* Release every resource of the context (NULL is ignored). */
void sgw_destroy(sgw_ctx *ctx);

/* Message of the last failing call on ctx (ctx = NULL: last failing
 * sgw_create of the calling thread).  Valid until the next call. */
const char *sgw_last_error(const sgw_ctx *ctx);

/* Rigorous spectral interval of H (Weyl): [min V + lo, T_max + max V + hi]
 * where [lo, hi] encloses spec(V_NL) by the Gershgorin bound of the
 * projector Gram matrix, widened by pad times its width on each side.  The
 * paper finds the interval by shifted power iteration (Sec. 2.1); any
 * enclosing interval serves the Chebyshev maps that follow. */
sgw_status sgw_bounds(sgw_ctx *ctx, double pad, double *emin, double *emax);

/* Spectral interval from k Lanczos steps on the device (the paper finds the
 * interval by shifted power iteration, Sec. 2.1; Lanczos gives both ends from
 * one Krylov sequence).  Start: the +-1 white noise of RNG stream (kind 5,
 * sample 0, l 0) for `seed`, unit Euclidean norm; no reorthogonalisation;
 * FP64 dot products.  With theta the Ritz values of the k x k tridiagonal
 * and r = beta_k |y_last| their residual norms,
 *   emin = theta_min - r_min - pad (theta_max - theta_min),
 *   emax = theta_max + r_max + pad (theta_max - theta_min),
 * each clipped to the rigorous interval of sgw_bounds(pad = 0), which it can
 * only narrow.  The ends are estimates: a Chebyshev recurrence that grows
 * on such an interval reports SGW_EDIVERGED.  2 <= k <= 1000.  Synchronous. */
sgw_status sgw_lanczos_bounds(sgw_ctx *ctx, int32_t k, uint64_t seed, double pad, double *emin,
                              double *emax);

/* hpsi[v] = H psi[v] for v < nvec (Eq. 1; Sec. 2.2: FFT pair for the
 * kinetic term, potential diagonal in r).  psi and hpsi are device batches
 * with leading dimension ld; they must not overlap.  With projectors in a
 * complex-FP32 precision, ld must be even (the projector kernels read
 * 16-byte operands); otherwise SGW_EUNSUPPORTED. */
sgw_status sgw_apply_H(sgw_ctx *ctx, const void *psi, void *hpsi,
                       int64_t nvec, int64_t ld);

/* sgw_apply_H for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operation and result, with no hipMalloc, hipFree or other
 * allocating call.  The projector partial sums and coefficients live in one
 * static 64 MiB device array per GPU, reserved when the library is loaded
 * (its address is looked up by the first sgw_create on each device); the
 * FFT intermediate lives in hpsi.  Vectors are processed in chunks of as
 * many as that array holds (per vector: 8 or 16 bytes times the projector
 * entries of all grid tiles plus the projectors); SGW_EUNSUPPORTED when not
 * even one vector fits.  Kernel variants are not timed: the choice already
 * made for this batch width, the tuning cache's, or the first (all variants
 * give identical results).  The context's device must be current
 * (SGW_EINVAL otherwise), psi and hpsi must not overlap, and the launch
 * timers are off during the call.  Every call on one GPU shares its array:
 * calls that overlap in time on one GPU (other streams, other contexts,
 * other threads) race and must be serialised by the caller.  Nothing in the
 * array has to start at zero (each call overwrites what it reads). */
sgw_status sgw_apply_H_noalloc(sgw_ctx *ctx, const void *psi, void *hpsi,
                               int64_t nvec, int64_t ld);

/* Chebyshev coefficients of the Fermi filter F(E) = 1/(1 + e^{beta(E-mu)})
 * on [emin, emax] (Eq. 3 with the step smoothed), by Chebyshev-Gauss
 * quadrature on M = 4 ncoef nodes:
 *   a_n = (2 - delta_n0)/M sum_j F(c + R cos t_j) cos(n t_j),
 *   t_j = pi (j + 1/2)/M, c = (emax+emin)/2, R = (emax-emin)/2.
 * coef: host [ncoef] output.  Pure host computation. */
sgw_status sgw_fermi_coefficients(double mu, double beta, double emin,
                                  double emax, int32_t ncoef, double *coef);

/* Chebyshev coefficients of the gapped filter (Sec. 2.1: the cutoff is
 * spread over the band gap E_HOMO <= mu <= E_LUMO): the step
 * G(E) = erfc((E - mu)/sigma)/2, mu = (e_homo + e_lumo)/2,
 * sigma = (e_lumo - e_homo)/(2 erfcinv(2 eps)), so G = 1 - eps at e_homo
 * and eps at e_lumo; same quadrature as sgw_fermi_coefficients.  Needs
 * e_homo < e_lumo and 0 < eps < 0.5.  Pure host computation. */
sgw_status sgw_gapped_coefficients(double e_homo, double e_lumo, double eps, double emin,
                                   double emax, int32_t ncoef, double *coef);

/* In place: v[k] <- sum_{n<ncoef} coef[n] T_n((H - c)/R) v[k] (Eq. 3) for
 * k < nvec, by the three-term recurrence.  The filter is real, so complex
 * vectors may carry two real orbitals each (real and imaginary parts).
 * coef: host [ncoef].  [emin, emax] must enclose spec(H); a recurrence that
 * grows anyway returns SGW_EDIVERGED (v is then undefined).  With projectors
 * and batches of 16 vectors or more, each term's projections of v_n are
 * computed on a second stream of the context beside the term's FFT passes
 * (they only read v_n), and the stream
 * of the context waits for them before the projector update; the call thus
 * orders itself on the context's stream as before, and its results are
 * bitwise those of one stream, which SGW_KB_OVERLAP=0 at sgw_create selects
 * (the same holds for sgw_cheb_propagate and the filter of
 * sgw_sigma_estimate). */
sgw_status sgw_fermi_filter(sgw_ctx *ctx, void *v, int64_t nvec, int64_t ld,
                            const double *coef, int32_t ncoef, double emin,
                            double emax);

/* Coefficients b_n of exp(-i H tau) = sum_n b_n T_n((H - c)/R) (Jacobi-Anger
 * expansion, b_n = e^{-i c tau} (2 - delta_n0) (-i)^n J_n(R tau)), truncated
 * at the first n > R|tau| with |J_n(R|tau|)| < tol.  J_n by Miller's backward
 * recurrence.  coef: host [max_terms][2] (re, im); *nterms receives the count
 * (SGW_EINVAL if it exceeds max_terms).  Pure host computation. */
sgw_status sgw_propagator_coefficients(double emin, double emax, double tau,
                                       double tol, int32_t max_terms,
                                       double *coef, int32_t *nterms);

/* In place: psi[k] <- exp(-i H dt)^nsteps psi[k] (the propagator of the
 * zeta orbitals, Sec. 2.1 second phase), one Chebyshev series per step with
 * the coefficients of sgw_propagator_coefficients(emin, emax, dt, tol). */
sgw_status sgw_cheb_propagate(sgw_ctx *ctx, void *psi, int64_t nvec,
                              int64_t ld, double dt, int32_t nsteps,
                              double emin, double emax, double tol);

/* Linear-response TDH state for nsample Monte Carlo samples (Sec. 2.1 first
 * phase; Sec. 2.3 packs the unperturbed and perturbed copies together).
 * Device arrays, caller-owned:
 *   psi  [nsample][2][neta][N_g] complex: copy 0 = eta_l(t), copy 1 = the
 *        tangent delta-eta_l(t) of the perturbed copy (lambda -> 0 limit of
 *        (eta^lambda - eta)/lambda);
 *   v    [nsample][N_g] real: V(t) = V_loc + v_H[n(t)] - v_H[n(0)];
 *   u    [nsample][N_g] real: u^R(t) = v_H[delta n(t)];
 *   vh0  [nsample][N_g] real: v_H[n(0)];
 * with n = weight sum_l |eta_l|^2, delta n = weight sum_l 2 Re(conj(eta_l)
 * delta-eta_l) and v_H[rho] = F^{-1}[4 pi/|k|^2 F[rho]] (k = 0 dropped). */
typedef struct {
  int32_t nsample;
  int32_t neta;
  double weight;
  void *psi;
  void *v;
  void *u;
  void *vh0;
} sgw_tdh_state;

/* Start the response: given eta(0) in copy 0 of psi and the kick potential
 * dv (device [nsample][N_g] real, dv_i = v_H[phi zeta-bar_i]), set
 * delta-eta(0) = -i dv eta(0), vh0 = v_H[n(0)], v = V_loc, u = v_H[delta
 * n(0)] (= 0). */
sgw_status sgw_tdh_init(sgw_ctx *ctx, sgw_tdh_state *st, const void *dv);

/* Advance the state by nsub Strang substeps of length dt_sub:
 *   exp(-i V(t) tau/2), exp(-i V_NL tau/2), F^-1 exp(-i T tau) F,
 *   exp(-i V_NL tau/2), densities -> V(t+tau), u^R(t+tau),
 *   exp(-i V(t+tau) tau/2),
 * where the local half steps act on the tangent copy as
 *   delta-eta <- exp(-i V a)(delta-eta - i a u^R eta)   (a = tau/2)
 * (the exact tangent of the finite-lambda step). */
sgw_status sgw_tdh_step(sgw_ctx *ctx, sgw_tdh_state *st, int32_t nsub,
                        double dt_sub);

/* Parameters of one stochastic Sigma_c(t) estimate (Sec. 2.1, Table 2). */
typedef struct {
  uint64_t seed;          /* counter-based RNG seed (SplitMix64 streams) */
  int32_t first_sample;   /* global index of the first Monte Carlo sample */
  int32_t n_zeta;         /* number of samples in this call */
  int32_t n_eta;          /* stochastic occupied orbitals per sample (even) */
  int32_t n_tau;          /* output time steps on each side of t = 0 */
  double dt;              /* output time step, a.u. */
  int32_t m_sub;          /* TDH Strang substeps per output step */
  double mu, beta;        /* Fermi filter (filter = 0) */
  int32_t ncoef;          /* filter length */
  double emin, emax;      /* spectral interval for every Chebyshev map */
  int32_t n_xi;           /* sparse stochastic functions per sample */
  double f_g;             /* grid fraction of each xi (segments of 32) */
  int32_t mode;           /* 0: sparse xi basis; 1: exact (full-grid u) */
  double prop_tol;        /* Jacobi-Anger truncation of the zeta propagator */
  int32_t n_ft;           /* time-ordering FFT length (0: smallest power of
                             two >= 4 (n_tau + 1)) */
  int32_t batch;          /* samples resident on the device at once (0: all) */
  int32_t filter;         /* 0: Fermi (mu, beta); 1: gapped (e_homo, e_lumo,
                             filter_eps), see sgw_gapped_coefficients */
  double e_homo, e_lumo;  /* gapped filter: the band gap */
  double filter_eps;      /* gapped filter: its value at the gap edges */
} sgw_sigma_params;

/* Per-sample Sigma_c,i(t_j), j = -n_tau..n_tau, and exchange X_i for the
 * orbital phi (host [N_g] real, <phi|phi> = 1), following Sec. 2.1:
 * white noise -> filter (Eq. 3) -> TDH response u^R in the xi basis ->
 * time ordering -> zeta^+ forward / occupied part backward (Eq. 4) ->
 * contraction (Eq. 5).  sigma_t: host [n_zeta][2 n_tau + 1][2] (re, im);
 * x: host [n_zeta]; phase_ms: nullable host [6] receiving the device time
 * of the phases (filter, TDH, time ordering, zeta propagation and
 * contraction, the rest, total).  In xi mode the zeta propagation runs on a
 * second stream of the context beside the TDH steps (its time then falls in
 * the TDH phase; the results are bitwise those of running it afterwards,
 * which the environment variable SGW_ZETA_OVERLAP=0 at sgw_create selects).
 * The zeta states of G consecutive output steps come from one Chebyshev
 * sweep with the Jacobi-Anger coefficients of the times dt, 2 dt, ..., G dt
 * (each truncated at prop_tol), so the propagation is exact to prop_tol at
 * every step; G is 8, or SGW_ZETA_SWEEP at sgw_create (clamped to 1 .. 8).
 * Requires N_g to be a multiple of 32 in xi mode. */
sgw_status sgw_sigma_estimate(sgw_ctx *ctx, const sgw_sigma_params *params,
                              const double *phi, double *sigma_t, double *x,
                              double *phase_ms);

/* Several quasiparticle states in one pass (Sec. 3 computes the HOMO and the
 * LUMO of each system, Table 3).  The white noise, the filtered zeta and
 * eta sets (Eq. 3), the xi sets and the zeta propagation (Eq. 4) do not
 * depend on phi and are computed once; each state k gets its own kick
 * v_H[phi_k zeta-bar], TDH response (one tangent copy of every eta per
 * state, beside one shared unperturbed copy), time ordering and contraction
 * (Eq. 5), and its exchange from the shared eta.  State k's results are those
 * of sgw_sigma_estimate with phi_k and the same params: bitwise for k = 0 and
 * up to rounding for k > 0 (its response field shares a complex Poisson FFT
 * with another state's).  phi: host [nstate][N_g]; sigma_t: host
 * [nstate][n_zeta][2 n_tau + 1][2]; x: host [nstate][n_zeta]; 1 <= nstate
 * <= SGW_MAX_STATES (SGW_EINVAL otherwise). */
#define SGW_MAX_STATES 8
sgw_status sgw_sigma_estimate_states(sgw_ctx *ctx, const sgw_sigma_params *params,
                                     int32_t nstate, const double *phi, double *sigma_t,
                                     double *x, double *phase_ms);

/* QP energy from the sample-mean Sigma_c(t_j) (host [2 n_tau + 1][2]):
 *   Sigma(w) = dt sum_j w_j e^{-gamma^2 t_j^2/2} e^{i w t_j} Sigma(t_j)
 * (Eq. 7, trapezoid weights), Z = 1/(1 - d Re Sigma/dw (eps_ks)),
 * eps_lin = eps_ks + Z (x + Re Sigma(eps_ks) - vxc), and the graphical root
 * of eps_ks + x + Re Sigma(w) - vxc - w (Eq. 6) nearest eps_lin (1 mHa scan
 * outwards to +-2 Ha, bisection to 1e-10 Ha).  SGW_ENOROOT if none. */
sgw_status sgw_qp_solve(const double *sigma_t, int32_t n_tau, double dt,
                        double gamma, double eps_ks, double x, double vxc,
                        double *eqp_graphical, double *eqp_linear, double *z);

/* Damped Fourier transform of Eq. (7) on the trapezoid rule:
 *   Sigma(w_k) = dt sum_j w_j e^{-gamma^2 t_j^2/2} e^{i w_k t_j} Sigma(t_j),
 * t_j = j dt, j = -n_tau..n_tau, w_j = 1/2 at the ends.  sigma_t: host
 * [2 n_tau + 1][2]; omega: host [n_omega]; out: host [n_omega][2]. */
sgw_status sgw_sigma_omega(const double *sigma_t, int32_t n_tau, double dt, double gamma,
                           const double *omega, int32_t n_omega, double *out);

/* Launch timers of the largest kernels (bits of `which`):
 *   SGW_TIMER_CHEB_PLANE  the inverse xy-plane FFT pass that carries the
 *                         Chebyshev-recurrence epilogue (Eq. 3 filter and the
 *                         zeta propagator); points = grid points x vectors;
 *   SGW_TIMER_KB_SCATTER  the projector scatter GEMM psi += s B C' (complex
 *                         FP32 precisions; filter terms, H applications and
 *                         the KB exponential of the TDH steps); points =
 *                         points of the tiles that projectors touch x vectors;
 *   SGW_TIMER_KB_GATHER   the projector gather GEMM C = B^T psi (complex FP32
 *                         precisions, the same calls); points as the scatter.
 * From sgw_kernel_timer(ctx, bits) on, every launch of the selected kernels
 * on the context's stream is bracketed by a pair of HIP events (launches on
 * the context's second stream -- the zeta propagation of sgw_sigma_estimate
 * beside the TDH steps, the Chebyshev terms' projector gathers beside their
 * FFT passes -- are not timed: they share the device with other kernels;
 * with SGW_KB_OVERLAP=0 the gathers run on the context's stream and are
 * timed); bits = 0 stops timing, other bits are
 * SGW_EINVAL.  sgw_kernel_timer_read(ctx, which, ...) takes one timer,
 * synchronises the stream and returns its summed event time (ms), the number
 * of timed launches and the points they processed, then resets that timer. */
#define SGW_TIMER_CHEB_PLANE 1
#define SGW_TIMER_KB_SCATTER 2
#define SGW_TIMER_KB_GATHER 4
sgw_status sgw_kernel_timer(sgw_ctx *ctx, int32_t which);
sgw_status sgw_kernel_timer_read(sgw_ctx *ctx, int32_t which, double *total_ms,
                                 int64_t *launches, int64_t *points);

/* Sizes of the projector layout (the separable non-local part applied with
 * overlapping spheres, Sec. 3), for byte and flop accounting: out[0] the
 * 512-point grid tiles that some projector touches, out[1] their points,
 * out[2] the grid points inside at least one projector's support, out[3]
 * the (tile, projector) entries, out[4] the nonzero projector values
 * (point, projector pairs).  All zero without projectors.  out: host [5]. */
sgw_status sgw_kb_stats(const sgw_ctx *ctx, int64_t *out);

/* HIP graphs for repeated launch sequences.  enable != 0: a Chebyshev series
 * of at most 64 terms (the zeta propagator, Eq. 4) runs as one captured graph
 * per set of buffers, a longer one (the filter, Eq. 3) as a captured pair of
 * terms that reads its coefficient from device memory, and the TDH output
 * steps 2 .. n_tau of sgw_sigma_estimate (xi mode) as one captured step
 * whose output row comes from a device counter.  Each sequence runs eagerly
 * the first time (autotuning and allocation happen there) and is replayed
 * afterwards; results are bitwise the same as without graphs.  Needs a
 * context created on a non-default stream (SGW_EINVAL otherwise); graphs are
 * not used while the kernel timer is on.  Synchronises the stream. */
sgw_status sgw_use_graphs(sgw_ctx *ctx, int32_t enable);


/* Many clusters of uneven size in one call.  Each item is one
 * sgw_sigma_estimate on its own context; the items are ordered by an
 * estimate of their work (grid points x log, filter, TDH and propagation
 * vectors) and dealt, longest first, to `nworkers` host threads (each item
 * to the least-loaded thread).  Each thread issues its items in turn, so
 * items on contexts with different streams run concurrently on the GPU.
 * Every item needs its own context (SGW_EINVAL otherwise).  Contexts with
 * graphs on replay the graphs they already hold and capture no new ones
 * inside the batch (a sequence without a graph runs eagerly, with the same
 * result): run each such context once before the batch.  Per item:
 * status and wall time (ms) are written back; the call returns SGW_OK or
 * the status of the first failed item (in item order).  phase timings are
 * not recorded. */
typedef struct {
  sgw_ctx *ctx;
  const sgw_sigma_params *params;
  const double *phi;        /* host [N] */
  double *sigma_t;          /* host [n_zeta][2 n_tau + 1][2] */
  double *x;                /* host [n_zeta] */
  sgw_status status;        /* out */
  double ms;                /* out */
} sgw_batch_item;
sgw_status sgw_batch_sigma_estimate(sgw_batch_item *items, int32_t n, int32_t nworkers);

/* ---------------------------------------------------------------------------
 * Learned control variate (an addition to the paper's Monte Carlo average,
 * Sec. 3: samples are averaged until the QP error bar is below 0.03 eV).
 * Per sample i, y_i = X_i + Re Sigma_c,i(omega) enters the QP equation
 * (Eq. 6) linearly.  A network g(x_i) of cheap features x_i of the same white
 * noise (zeta-bar_i and the eta-bar set of the sample), fitted to y on a set
 * A, gives the estimate
 *   mean_B(y - c g) + c mean_M(g),  c = Cov_A(y, g) / Var_A(g),
 * over an evaluation set B and M cheap samples (features only).  All
 * products run on MFMA with BF16 operands and FP32 accumulation.
 * ------------------------------------------------------------------------- */

/* Features x[i][k] = |<phi_k|zeta_i>|^2 for samples i = first_sample ..
 * first_sample + nsamp - 1, zeta_i the white noise of Monte Carlo sample i
 * (the zeta-bar stream that sgw_sigma_estimate draws for that sample).
 * phi: device float [K][ld_phi] real orbitals (1 <= K <= 64, ld_phi >= N),
 * rounded to BF16 on the device; x: device float [nsamp][K].  The sample
 * indices must lie in [0, 2^20); N must be divisible by 64 (else
 * SGW_EUNSUPPORTED).  Asynchronous on the context's stream. */
sgw_status sgw_cv_features(sgw_ctx *ctx, const float *phi, int32_t K, int64_t ld_phi,
                           uint64_t seed, int64_t first_sample, int64_t nsamp, float *x);

/* Features of a sample's occupied-orbital white noise (the eta-bar set that
 * Sec. 2.1 filters into the stochastic occupied orbitals; their density and
 * the exchange X_i follow from it):
 *   x[i][k] = (1/n_eta) sum_l |<phi_k|eta-bar_{i,l}>|^2,  l = 0 .. n_eta - 1,
 * eta-bar_{i,l} the white noise that sgw_sigma_estimate draws for sample i.
 * Arguments as sgw_cv_features; rows of x are ldx >= K floats apart (so the
 * zeta-bar and eta-bar features of one sample can share a row).  Needs
 * 4 nsamp n_eta K bytes of context scratch. */
sgw_status sgw_cv_features_eta(sgw_ctx *ctx, const float *phi, int32_t K, int64_t ld_phi,
                               uint64_t seed, int64_t first_sample, int64_t nsamp,
                               int32_t n_eta, float *x, int64_t ldx);

/* The network g(x) = w3 . tanh(W2 tanh(W1 xh + b1) + b2) + b3 with
 * xh = (x - mean) / std.  Parameters are packed W1 [h1][din], b1 [h1],
 * W2 [h2][h1], b2 [h2], w3 [h2], b3 [1]; the library keeps FP32 master
 * copies, Adam moments and a gradient on the device.  theta0: host FP64
 * initial parameters (copied).  Work is enqueued on hip_stream (NULL: the
 * default stream).  The standardization starts as mean 0, std 1. */
typedef struct sgw_mlp sgw_mlp;
sgw_status sgw_mlp_create(int32_t din, int32_t h1, int32_t h2, const double *theta0,
                          void *hip_stream, sgw_mlp **out);
void sgw_mlp_destroy(sgw_mlp *mlp);
const char *sgw_mlp_last_error(const sgw_mlp *mlp);   /* NULL: last create failure */
/* mean, std: host FP64 [din], std > 0 (synchronous) */
sgw_status sgw_mlp_set_standardization(sgw_mlp *mlp, const double *mean, const double *std);
/* theta: host FP64 [nparam] <- the FP32 master parameters (synchronous) */
sgw_status sgw_mlp_get_params(sgw_mlp *mlp, double *theta);
/* g: device float [n] <- network(x), x: device float [n][din] (asynchronous) */
sgw_status sgw_mlp_forward(sgw_mlp *mlp, const float *x, int64_t n, float *g);
/* Mean squared error L = (1/n) sum (g(x_i) - y_i)^2 (host *loss) and its
 * gradient (host FP64 [nparam], also kept on the device for sgw_mlp_adam);
 * x: device [n][din], y: device [n] (synchronous). */
sgw_status sgw_mlp_gradient(sgw_mlp *mlp, const float *x, const float *y, int64_t n,
                            double *loss, double *grad);
/* One Adam step (bias-corrected moments) with the device gradient of the
 * last sgw_mlp_gradient / training step, or with the host FP64 gradient
 * `grad` when it is not NULL. */
sgw_status sgw_mlp_adam(sgw_mlp *mlp, const double *grad, double lr, double b1, double b2,
                        double eps);
/* `steps` full-batch steps (forward, gradient, Adam with b1 = 0.9,
 * b2 = 0.999, eps = 1e-8) on device data x [n][din], y [n], all on the
 * device; loss_hist (host [steps] or NULL) receives the loss before each
 * step (synchronous when loss_hist is given). */
sgw_status sgw_mlp_train(sgw_mlp *mlp, const float *x, const float *y, int64_t n,
                         int32_t steps, double lr, double *loss_hist);
/* Mean and sample variance (FP64) of g over the cheap samples first_sample
 * .. first_sample + count - 1: features and network in chunks of `chunk`
 * samples on the context's stream, which must be the network's stream.
 * K must equal the network's din. Synchronous. */
sgw_status sgw_cv_cheap_moments(sgw_ctx *ctx, sgw_mlp *mlp, const float *phi, int32_t K,
                                int64_t ld_phi, uint64_t seed, int64_t first_sample,
                                int64_t count, int64_t chunk, double *mean, double *var);
/* The same for a network whose input row is [the Kz zeta-bar features over
 * phi_z, the Ke eta-bar features over phi_e (n_eta vectors per sample)],
 * Kz + Ke = din; either part may be empty (K = 0, its phi NULL). */
sgw_status sgw_cv_cheap_moments_mixed(sgw_ctx *ctx, sgw_mlp *mlp, const float *phi_z,
                                      int32_t Kz, const float *phi_e, int32_t Ke,
                                      int64_t ld_phi, uint64_t seed, int32_t n_eta,
                                      int64_t first_sample, int64_t count, int64_t chunk,
                                      double *mean, double *var);

typedef struct {
  double estimate;        /* the control-variate estimate, or the plain one on fallback */
  double sigma;           /* its standard error */
  double c;               /* Cov_A(y, g) / Var_A(g) */
  double rho2;            /* squared correlation of y and g on A */
  double plain;           /* mean of y over A and B */
  double sigma_plain;     /* its standard error */
  double sigma_cv;        /* standard error of the control-variate form */
  int32_t fallback;       /* 1: |cv - plain| > 3 sqrt(sigma_cv^2 + sigma_plain^2) */
} sgw_cv_result;

/* Host FP64: the estimator above from per-sample y, g on A (nA >= 2) and B
 * (nB >= 2) and the mean and variance of g over M >= 2 cheap samples.
 * Sample variances use n - 1. */
sgw_status sgw_cv_estimate(const double *yA, const double *gA, int64_t nA, const double *yB,
                           const double *gB, int64_t nB, double gM_mean, double gM_var,
                           int64_t M, sgw_cv_result *out);

#ifdef __cplusplus
}
#endif

#endif /* SGW_H */
