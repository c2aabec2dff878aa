"""Thin Python binding of libsgw (include/sgw.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device arrays are torch tensors on the ROCm device (torch supplies
memory and the stream); host arrays are numpy.  If the library is missing
the import fails -- there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgw.so")

SGW_OK, SGW_EINVAL, SGW_ENOMEM, SGW_EHIP, SGW_EDIVERGED, SGW_ENOROOT, SGW_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
SGW_C128, SGW_C64, SGW_C64_BF16KB, SGW_C64_BF16X2KB = 0, 1, 2, 3
SGW_MAX_STATES = 8
SGW_TIMER_CHEB_PLANE, SGW_TIMER_KB_SCATTER, SGW_TIMER_KB_GATHER = 1, 2, 4

STATUS_NAMES = {0: "SGW_OK", -1: "SGW_EINVAL", -2: "SGW_ENOMEM", -3: "SGW_EHIP",
                -4: "SGW_EDIVERGED", -5: "SGW_ENOROOT", -6: "SGW_EUNSUPPORTED"}

# every entry point declared in include/sgw.h
EXPORTS = ["sgw_create", "sgw_destroy", "sgw_last_error", "sgw_bounds", "sgw_lanczos_bounds",
           "sgw_apply_H", "sgw_apply_H_noalloc",
           "sgw_fermi_coefficients", "sgw_gapped_coefficients", "sgw_fermi_filter", "sgw_propagator_coefficients",
           "sgw_cheb_propagate", "sgw_tdh_init", "sgw_tdh_step", "sgw_sigma_estimate",
           "sgw_sigma_estimate_states",
           "sgw_qp_solve", "sgw_sigma_omega", "sgw_kernel_timer", "sgw_kernel_timer_read", "sgw_kb_stats",
           "sgw_use_graphs", "sgw_batch_sigma_estimate", "sgw_cv_features", "sgw_cv_features_eta", "sgw_cv_cheap_moments_mixed", "sgw_mlp_create", "sgw_mlp_destroy", "sgw_mlp_last_error",
           "sgw_mlp_set_standardization", "sgw_mlp_get_params", "sgw_mlp_forward",
           "sgw_mlp_gradient", "sgw_mlp_adam", "sgw_mlp_train", "sgw_cv_cheap_moments",
           "sgw_cv_estimate"]


class SgwGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double), ("ecut", C.c_double)]


class SgwProjectors(C.Structure):
    _fields_ = [("natom", C.c_int32),
                ("pos", C.POINTER(C.c_double)),
                ("proj_begin", C.POINTER(C.c_int32)),
                ("l", C.POINTER(C.c_int32)),
                ("m", C.POINTER(C.c_int32)),
                ("rc", C.POINTER(C.c_double)),
                ("ekb", C.POINTER(C.c_double)),
                ("rcut_over_rc", C.c_double)]


class SgwTdhState(C.Structure):
    _fields_ = [("nsample", C.c_int32), ("neta", C.c_int32), ("weight", C.c_double),
                ("psi", C.c_void_p), ("v", C.c_void_p), ("u", C.c_void_p),
                ("vh0", C.c_void_p)]


class SgwSigmaParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("first_sample", C.c_int32), ("n_zeta", C.c_int32),
                ("n_eta", C.c_int32), ("n_tau", C.c_int32), ("dt", C.c_double),
                ("m_sub", C.c_int32), ("mu", C.c_double), ("beta", C.c_double),
                ("ncoef", C.c_int32), ("emin", C.c_double), ("emax", C.c_double),
                ("n_xi", C.c_int32), ("f_g", C.c_double), ("mode", C.c_int32),
                ("prop_tol", C.c_double), ("n_ft", C.c_int32), ("batch", C.c_int32),
                ("filter", C.c_int32), ("e_homo", C.c_double), ("e_lumo", C.c_double),
                ("filter_eps", C.c_double)]


class SgwBatchItem(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("params", C.POINTER(SgwSigmaParams)),
                ("phi", C.POINTER(C.c_double)), ("sigma_t", C.POINTER(C.c_double)),
                ("x", C.POINTER(C.c_double)), ("status", C.c_int), ("ms", C.c_double)]


class SgwCvResult(C.Structure):
    _fields_ = [("estimate", C.c_double), ("sigma", C.c_double), ("c", C.c_double),
                ("rho2", C.c_double), ("plain", C.c_double), ("sigma_plain", C.c_double),
                ("sigma_cv", C.c_double), ("fallback", C.c_int32)]


class SgwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libsgw.so (build it first with paper_2601_21005_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2601_21005_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, d, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.POINTER(C.c_double)
    lib.sgw_create.argtypes = [C.POINTER(SgwGrid), dp, C.POINTER(SgwProjectors), C.c_int,
                               vp, i64, C.POINTER(vp)]
    lib.sgw_destroy.argtypes = [vp]
    lib.sgw_destroy.restype = None
    lib.sgw_last_error.argtypes = [vp]
    lib.sgw_last_error.restype = C.c_char_p
    lib.sgw_bounds.argtypes = [vp, d, dp, dp]
    lib.sgw_lanczos_bounds.argtypes = [vp, i32, C.c_uint64, d, dp, dp]
    lib.sgw_apply_H.argtypes = [vp, vp, vp, i64, i64]
    lib.sgw_apply_H_noalloc.argtypes = [vp, vp, vp, i64, i64]
    lib.sgw_fermi_coefficients.argtypes = [d, d, d, d, i32, dp]
    lib.sgw_gapped_coefficients.argtypes = [d, d, d, d, d, i32, dp]
    lib.sgw_fermi_filter.argtypes = [vp, vp, i64, i64, dp, i32, d, d]
    lib.sgw_propagator_coefficients.argtypes = [d, d, d, d, i32, dp, C.POINTER(i32)]
    lib.sgw_cheb_propagate.argtypes = [vp, vp, i64, i64, d, i32, d, d, d]
    lib.sgw_tdh_init.argtypes = [vp, C.POINTER(SgwTdhState), vp]
    lib.sgw_tdh_step.argtypes = [vp, C.POINTER(SgwTdhState), i32, d]
    lib.sgw_sigma_estimate.argtypes = [vp, C.POINTER(SgwSigmaParams), dp, dp, dp, dp]
    lib.sgw_qp_solve.argtypes = [dp, i32, d, d, d, d, d, dp, dp, dp]
    lib.sgw_sigma_omega.argtypes = [dp, i32, d, d, dp, i32, dp]
    lib.sgw_kernel_timer.argtypes = [vp, i32]
    lib.sgw_use_graphs.argtypes = [vp, i32]
    lib.sgw_batch_sigma_estimate.argtypes = [C.POINTER(SgwBatchItem), i32, i32]
    lib.sgw_kernel_timer_read.argtypes = [vp, i32, dp, C.POINTER(i64), C.POINTER(i64)]
    lib.sgw_kb_stats.argtypes = [vp, C.POINTER(i64)]
    u64, fp = C.c_uint64, C.c_void_p
    lib.sgw_cv_features.argtypes = [vp, fp, i32, i64, u64, i64, i64, fp]
    lib.sgw_mlp_create.argtypes = [i32, i32, i32, dp, vp, C.POINTER(vp)]
    lib.sgw_mlp_destroy.argtypes = [vp]
    lib.sgw_mlp_destroy.restype = None
    lib.sgw_mlp_last_error.argtypes = [vp]
    lib.sgw_mlp_last_error.restype = C.c_char_p
    lib.sgw_mlp_set_standardization.argtypes = [vp, dp, dp]
    lib.sgw_mlp_get_params.argtypes = [vp, dp]
    lib.sgw_mlp_forward.argtypes = [vp, fp, i64, fp]
    lib.sgw_mlp_gradient.argtypes = [vp, fp, fp, i64, dp, dp]
    lib.sgw_mlp_adam.argtypes = [vp, dp, d, d, d, d]
    lib.sgw_mlp_train.argtypes = [vp, fp, fp, i64, i32, d, dp]
    lib.sgw_cv_cheap_moments.argtypes = [vp, vp, fp, i32, i64, u64, i64, i64, i64, dp, dp]
    lib.sgw_cv_features_eta.argtypes = [vp, fp, i32, i64, u64, i64, i64, i32, fp, i64]
    lib.sgw_cv_cheap_moments_mixed.argtypes = [vp, vp, fp, i32, fp, i32, i64, u64, i32, i64,
                                               i64, i64, dp, dp]
    lib.sgw_cv_estimate.argtypes = [dp, dp, i64, dp, dp, i64, d, d, i64,
                                    C.POINTER(SgwCvResult)]
    for name in EXPORTS:
        if name not in ("sgw_destroy", "sgw_last_error", "sgw_mlp_destroy",
                        "sgw_mlp_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _check(code, ctx=None):
    if code != SGW_OK:
        msg = load().sgw_last_error(ctx)
        raise SgwError(code, msg.decode() if msg else "")


def _check_mlp(code, mlp=None):
    if code != SGW_OK:
        msg = load().sgw_mlp_last_error(mlp)
        raise SgwError(code, msg.decode() if msg else "")


def _dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ host calls
def sgw_fermi_coefficients(mu, beta, emin, emax, ncoef):
    out = np.zeros(int(ncoef))
    _check(load().sgw_fermi_coefficients(mu, beta, emin, emax, int(ncoef), _dptr(out)))
    return out


def sgw_gapped_coefficients(e_homo, e_lumo, eps, emin, emax, ncoef):
    out = np.zeros(int(ncoef))
    _check(load().sgw_gapped_coefficients(e_homo, e_lumo, eps, emin, emax, int(ncoef),
                                          _dptr(out)))
    return out


def sgw_propagator_coefficients(emin, emax, tau, tol=1e-14, max_terms=4096):
    out = np.zeros(2 * max_terms)
    nt = C.c_int32(0)
    _check(load().sgw_propagator_coefficients(emin, emax, tau, tol, max_terms, _dptr(out),
                                             C.byref(nt)))
    b = out[:2 * nt.value]
    return b[0::2] + 1j * b[1::2]


def sgw_qp_solve(sigma_t, dt, gamma, eps_ks, x, vxc=0.0):
    s = np.ascontiguousarray(np.asarray(sigma_t, dtype=np.complex128))
    n_tau = (s.size - 1) // 2
    buf = np.ascontiguousarray(np.stack([s.real, s.imag], axis=-1).ravel())
    eg, el, z = C.c_double(), C.c_double(), C.c_double()
    _check(load().sgw_qp_solve(_dptr(buf), n_tau, dt, gamma, eps_ks, x, vxc, C.byref(eg),
                               C.byref(el), C.byref(z)))
    return eg.value, el.value, z.value


def sgw_sigma_omega(sigma_t, dt, gamma, omega):
    s = np.asarray(sigma_t, dtype=np.complex128)
    n_tau = (s.size - 1) // 2
    buf = np.ascontiguousarray(np.stack([s.real, s.imag], axis=-1).ravel())
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, dtype=np.float64)))
    out = np.zeros(2 * om.size)
    _check(load().sgw_sigma_omega(_dptr(buf), n_tau, dt, gamma, _dptr(om), om.size, _dptr(out)))
    return out[0::2] + 1j * out[1::2]


# ------------------------------------------------------------------ context
class Context:
    """A libsgw context: H on a grid, in one precision, on one stream."""

    def __init__(self, n, h, v_loc, projectors=None, precision=SGW_C64, ecut=0.0,
                 max_nvec=256, stream=None):
        import torch
        lib = load()
        nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
        self.n = (int(nx), int(ny), int(nz))
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.precision = precision
        self.cdtype = torch.complex128 if precision == SGW_C128 else torch.complex64
        self.rdtype = torch.float64 if precision == SGW_C128 else torch.float32
        g = SgwGrid(self.n[0], self.n[1], self.n[2], float(h), float(ecut))
        v = np.ascontiguousarray(np.asarray(v_loc, dtype=np.float64).ravel())
        if v.size != self.N:
            raise ValueError("v_loc has the wrong size")
        self._keep = [v]
        pp = None
        if projectors is not None:
            p = projectors
            arrs = dict(pos=np.ascontiguousarray(np.asarray(p.pos, dtype=np.float64)),
                        pb=np.ascontiguousarray(np.asarray(p.proj_begin, dtype=np.int32)),
                        l=np.ascontiguousarray(np.asarray(p.l, dtype=np.int32)),
                        m=np.ascontiguousarray(np.asarray(p.m, dtype=np.int32)),
                        rc=np.ascontiguousarray(np.asarray(p.rc, dtype=np.float64)),
                        ekb=np.ascontiguousarray(np.asarray(p.ekb, dtype=np.float64)))
            self._keep.append(arrs)
            pp = SgwProjectors(len(arrs["pb"]) - 1, _dptr(arrs["pos"]), _iptr(arrs["pb"]),
                               _iptr(arrs["l"]), _iptr(arrs["m"]), _dptr(arrs["rc"]),
                               _dptr(arrs["ekb"]), float(p.rcut_over_rc))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        ctx = C.c_void_p()
        code = lib.sgw_create(C.byref(g), _dptr(v), C.byref(pp) if pp is not None else None,
                              int(precision), C.c_void_p(stream), int(max_nvec), C.byref(ctx))
        _check(code, None)
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            load().sgw_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # device arrays of this context's precision
    def vectors(self, nvec):
        import torch
        return torch.zeros((nvec, self.N), dtype=self.cdtype, device="cuda")

    def fields(self, n):
        import torch
        return torch.zeros((n, self.N), dtype=self.rdtype, device="cuda")

    def bounds(self, pad=0.01):
        a, b = C.c_double(), C.c_double()
        _check(load().sgw_bounds(self.ctx, pad, C.byref(a), C.byref(b)), self.ctx)
        return a.value, b.value

    def lanczos_bounds(self, k=40, seed=0, pad=0.01):
        a, b = C.c_double(), C.c_double()
        _check(load().sgw_lanczos_bounds(self.ctx, int(k), int(seed), pad, C.byref(a),
                                         C.byref(b)), self.ctx)
        return a.value, b.value

    def apply_H(self, psi, hpsi):
        _check(load().sgw_apply_H(self.ctx, _dev(psi, "psi"), _dev(hpsi, "hpsi"),
                                  psi.shape[0], psi.shape[-1]), self.ctx)

    def apply_H_noalloc(self, psi, hpsi):
        _check(load().sgw_apply_H_noalloc(self.ctx, _dev(psi, "psi"), _dev(hpsi, "hpsi"),
                                          psi.shape[0], psi.shape[-1]), self.ctx)

    def fermi_filter(self, v, coef, emin, emax):
        c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
        _check(load().sgw_fermi_filter(self.ctx, _dev(v, "v"), v.shape[0], v.shape[-1],
                                       _dptr(c), c.size, emin, emax), self.ctx)

    def cheb_propagate(self, psi, dt, nsteps, emin, emax, tol=1e-14):
        _check(load().sgw_cheb_propagate(self.ctx, _dev(psi, "psi"), psi.shape[0],
                                         psi.shape[-1], dt, int(nsteps), emin, emax, tol),
               self.ctx)

    def tdh_state(self, psi, v, u, vh0, nsample, neta, weight):
        st = SgwTdhState(int(nsample), int(neta), float(weight), _dev(psi, "psi"),
                         _dev(v, "v"), _dev(u, "u"), _dev(vh0, "vh0"))
        st._keep = (psi, v, u, vh0)
        return st

    def tdh_init(self, st, dv):
        _check(load().sgw_tdh_init(self.ctx, C.byref(st), _dev(dv, "dv")), self.ctx)

    def tdh_step(self, st, nsub, dt_sub):
        _check(load().sgw_tdh_step(self.ctx, C.byref(st), int(nsub), float(dt_sub)), self.ctx)

    def use_graphs(self, enable=True):
        _check(load().sgw_use_graphs(self.ctx, 1 if enable else 0), self.ctx)

    def kernel_timer(self, which):
        """which: SGW_TIMER_CHEB_PLANE | SGW_TIMER_KB_SCATTER bits (True: the
        Chebyshev plane pass), 0 / False stops timing."""
        which = SGW_TIMER_CHEB_PLANE if which is True else int(which)
        _check(load().sgw_kernel_timer(self.ctx, which), self.ctx)

    def kernel_timer_read(self, which=None):
        """(summed ms, launches, points) of one timer, which resets."""
        which = SGW_TIMER_CHEB_PLANE if which is None else which
        ms, n, pts = C.c_double(), C.c_int64(), C.c_int64()
        _check(load().sgw_kernel_timer_read(self.ctx, which, C.byref(ms), C.byref(n),
                                            C.byref(pts)), self.ctx)
        return ms.value, n.value, pts.value

    def kb_stats(self):
        """Projector layout sizes: dict of touched tiles, their points, the
        support points, (tile, projector) entries and nonzero values."""
        out = (C.c_int64 * 5)()
        _check(load().sgw_kb_stats(self.ctx, out), self.ctx)
        return dict(zip(("tiles", "tile_points", "support_points", "entries", "nnz"),
                        list(out)))

    def sigma_estimate(self, phi, seed, n_zeta, n_eta, n_tau, dt, m_sub, ncoef, emin, emax,
                       mu=0.0, beta=0.0, n_xi=10000, f_g=0.003, mode=0, prop_tol=1e-14, n_ft=0,
                       first_sample=0, batch=0, filter=0, e_homo=0.0, e_lumo=0.0,
                       filter_eps=1e-7):
        p = sigma_params(seed, n_zeta, n_eta, n_tau, dt, m_sub, ncoef, emin, emax, mu, beta,
                         n_xi, f_g, mode, prop_tol, n_ft, first_sample, batch, filter, e_homo,
                         e_lumo, filter_eps)
        ph = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).ravel())
        sig = np.zeros((n_zeta, 2 * n_tau + 1, 2))
        x = np.zeros(n_zeta)
        ms = np.zeros(6)
        _check(load().sgw_sigma_estimate(self.ctx, C.byref(p), _dptr(ph), _dptr(sig), _dptr(x),
                                         _dptr(ms)), self.ctx)
        return sig[..., 0] + 1j * sig[..., 1], x, ms

    def sigma_estimate_states(self, phis, seed, n_zeta, n_eta, n_tau, dt, m_sub, ncoef, emin,
                              emax, mu=0.0, beta=0.0, n_xi=10000, f_g=0.003, mode=0,
                              prop_tol=1e-14, n_ft=0, first_sample=0, batch=0, filter=0,
                              e_homo=0.0, e_lumo=0.0, filter_eps=1e-7):
        """sigma_estimate for several orbitals phis [K][N] that share the
        filtered sets, xi sets and zeta propagation; returns Sigma [K][n_zeta]
        [2 n_tau + 1], X [K][n_zeta] and the phase times."""
        p = sigma_params(seed, n_zeta, n_eta, n_tau, dt, m_sub, ncoef, emin, emax, mu, beta,
                         n_xi, f_g, mode, prop_tol, n_ft, first_sample, batch, filter, e_homo,
                         e_lumo, filter_eps)
        ph = np.ascontiguousarray(np.asarray(phis, dtype=np.float64))
        K = ph.shape[0]
        if ph.ndim != 2 or ph.shape[1] != self.N:
            raise ValueError("phis must have shape [K][N_g]")
        sig = np.zeros((K, n_zeta, 2 * n_tau + 1, 2))
        x = np.zeros((K, n_zeta))
        ms = np.zeros(6)
        _check(load().sgw_sigma_estimate_states(self.ctx, C.byref(p), K, _dptr(ph), _dptr(sig),
                                                _dptr(x), _dptr(ms)), self.ctx)
        return sig[..., 0] + 1j * sig[..., 1], x, ms


# ------------------------------------------------------------------ control variate
def sgw_cv_estimate(yA, gA, yB, gB, gM_mean, gM_var, M):
    """Control-variate estimate (host FP64); returns a dict of sgw_cv_result."""
    arr = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (yA, gA, yB, gB)]
    if arr[0].size != arr[1].size or arr[2].size != arr[3].size:
        raise ValueError("y and g must have the same length on each set")
    r = SgwCvResult()
    _check(load().sgw_cv_estimate(_dptr(arr[0]), _dptr(arr[1]), arr[0].size, _dptr(arr[2]),
                                  _dptr(arr[3]), arr[2].size, float(gM_mean), float(gM_var),
                                  int(M), C.byref(r)))
    return {f: getattr(r, f) for f, _ in SgwCvResult._fields_} | {"fallback": bool(r.fallback)}


def _fdev(t, name, n=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} is too small")
    return C.c_void_p(t.data_ptr())


def cv_features(ctx, phi, seed, first_sample, nsamp, out=None):
    """x[i][k] = |<phi_k|zeta_i>|^2 for samples first_sample .. + nsamp - 1
    (phi: float32 [K][N] on the GPU); returns a float32 [nsamp][K] tensor."""
    import torch
    K = phi.shape[0]
    if out is None:
        out = torch.empty((nsamp, K), dtype=torch.float32, device="cuda")
    _check(load().sgw_cv_features(ctx.ctx, _fdev(phi, "phi"), K, phi.shape[-1], int(seed),
                                  int(first_sample), int(nsamp), _fdev(out, "x", nsamp * K)),
           ctx.ctx)
    return out


def cv_features_eta(ctx, phi, seed, first_sample, nsamp, n_eta, out=None, col0=0):
    """x[i][k] = mean over l < n_eta of |<phi_k|eta-bar_{i,l}>|^2 (phi: float32
    [K][N] on the GPU); returns a float32 [nsamp][K] tensor, or writes
    columns col0 .. col0 + K - 1 of the given [nsamp][ldx] tensor."""
    import torch
    K = phi.shape[0]
    if out is None:
        out = torch.empty((nsamp, K), dtype=torch.float32, device="cuda")
    ldx = out.shape[-1]
    if out.dim() != 2 or out.shape[0] < nsamp or col0 + K > ldx:
        raise ValueError("out must be [nsamp][ldx] with room for K columns at col0")
    _fdev(out, "x", nsamp * ldx)
    ptr = C.c_void_p(out.data_ptr() + 4 * col0)
    _check(load().sgw_cv_features_eta(ctx.ctx, _fdev(phi, "phi"), K, phi.shape[-1], int(seed),
                                      int(first_sample), int(nsamp), int(n_eta), ptr, ldx),
           ctx.ctx)
    return out


def cv_cheap_moments_mixed(ctx, mlp, phi_z, phi_e, seed, n_eta, first_sample, count,
                           chunk=65536):
    """Cheap-sample mean and variance of g for the input row [zeta-bar
    features over phi_z, eta-bar features over phi_e] (either may be None)."""
    m, v = C.c_double(), C.c_double()
    kz = 0 if phi_z is None else phi_z.shape[0]
    ke = 0 if phi_e is None else phi_e.shape[0]
    ld = (phi_z if phi_z is not None else phi_e).shape[-1]
    pz = _fdev(phi_z, "phi_z") if phi_z is not None else None
    pe = _fdev(phi_e, "phi_e") if phi_e is not None else None
    _check(load().sgw_cv_cheap_moments_mixed(ctx.ctx, mlp.mlp, pz, kz, pe, ke, ld, int(seed),
                                             int(n_eta), int(first_sample), int(count),
                                             int(chunk), C.byref(m), C.byref(v)), ctx.ctx)
    return m.value, v.value


def cv_cheap_moments(ctx, mlp, phi, seed, first_sample, count, chunk=65536):
    m, v = C.c_double(), C.c_double()
    _check(load().sgw_cv_cheap_moments(ctx.ctx, mlp.mlp, _fdev(phi, "phi"), phi.shape[0],
                                       phi.shape[-1], int(seed), int(first_sample), int(count),
                                       int(chunk), C.byref(m), C.byref(v)), ctx.ctx)
    return m.value, v.value


class Mlp:
    """The control-variate network (FP32 masters on the device, BF16 MFMA)."""

    def __init__(self, theta0, din=64, h1=256, h2=256, stream=None):
        import torch
        th = np.ascontiguousarray(np.asarray(theta0, dtype=np.float64))
        self.din, self.h1, self.h2 = din, h1, h2
        self.nparam = h1 * din + h1 + h2 * h1 + h2 + h2 + 1
        if th.size != self.nparam:
            raise ValueError("theta0 has the wrong size")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        m = C.c_void_p()
        _check_mlp(load().sgw_mlp_create(din, h1, h2, _dptr(th), C.c_void_p(stream),
                                         C.byref(m)), None)
        self.mlp = m

    def close(self):
        if getattr(self, "mlp", None):
            load().sgw_mlp_destroy(self.mlp)
            self.mlp = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_standardization(self, mean, std):
        m = np.ascontiguousarray(np.asarray(mean, dtype=np.float64))
        s = np.ascontiguousarray(np.asarray(std, dtype=np.float64))
        _check_mlp(load().sgw_mlp_set_standardization(self.mlp, _dptr(m), _dptr(s)), self.mlp)

    def params(self):
        out = np.zeros(self.nparam)
        _check_mlp(load().sgw_mlp_get_params(self.mlp, _dptr(out)), self.mlp)
        return out

    def forward(self, x, out=None):
        import torch
        n = x.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device="cuda")
        _check_mlp(load().sgw_mlp_forward(self.mlp, _fdev(x, "x", n * self.din), n,
                                          _fdev(out, "g", n)), self.mlp)
        return out

    def gradient(self, x, y):
        n = x.shape[0]
        loss = C.c_double()
        g = np.zeros(self.nparam)
        _check_mlp(load().sgw_mlp_gradient(self.mlp, _fdev(x, "x", n * self.din),
                                           _fdev(y, "y", n), n, C.byref(loss), _dptr(g)),
                   self.mlp)
        return loss.value, g

    def adam(self, grad=None, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        gp = None
        if grad is not None:
            grad = np.ascontiguousarray(np.asarray(grad, dtype=np.float64))
            gp = _dptr(grad)
        _check_mlp(load().sgw_mlp_adam(self.mlp, gp, lr, b1, b2, eps), self.mlp)

    def train(self, x, y, steps, lr=1e-3):
        n = x.shape[0]
        hist = np.zeros(max(1, steps))
        _check_mlp(load().sgw_mlp_train(self.mlp, _fdev(x, "x", n * self.din), _fdev(y, "y", n),
                                        n, int(steps), lr, _dptr(hist)), self.mlp)
        return hist[:steps]


# ------------------------------------------------------------------ batches
def sigma_params(seed, n_zeta, n_eta, n_tau, dt, m_sub, ncoef, emin, emax, mu=0.0, beta=0.0,
                 n_xi=10000, f_g=0.003, mode=0, prop_tol=1e-14, n_ft=0, first_sample=0,
                 batch=0, filter=0, e_homo=0.0, e_lumo=0.0, filter_eps=1e-7):
    return SgwSigmaParams(int(seed), int(first_sample), int(n_zeta), int(n_eta), int(n_tau),
                          float(dt), int(m_sub), float(mu), float(beta), int(ncoef),
                          float(emin), float(emax), int(n_xi), float(f_g), int(mode),
                          float(prop_tol), int(n_ft), int(batch), int(filter), float(e_homo),
                          float(e_lumo), float(filter_eps))


def batch_sigma_estimate(jobs, nworkers=4):
    """jobs: list of (Context, phi, dict of sigma_estimate keywords).  Returns
    a list of (sigma_t, x, wall ms) in job order; raises on the first failed
    item after all have run."""
    items = (SgwBatchItem * len(jobs))()
    keep = []
    outs = []
    for i, (ctx, phi, kw) in enumerate(jobs):
        p = sigma_params(**kw)
        ph = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).ravel())
        sig = np.zeros((kw["n_zeta"], 2 * kw["n_tau"] + 1, 2))
        x = np.zeros(kw["n_zeta"])
        keep += [p, ph]
        outs.append((sig, x))
        items[i].ctx = ctx.ctx
        items[i].params = C.pointer(p)
        items[i].phi = _dptr(ph)
        items[i].sigma_t = _dptr(sig)
        items[i].x = _dptr(x)
    for i in range(len(jobs)):
        items[i].status = SGW_EINVAL           # overwritten by every item that runs
    code = load().sgw_batch_sigma_estimate(items, len(jobs), int(nworkers))
    if code != SGW_OK:
        ran = [i for i in range(len(jobs)) if items[i].ms > 0]
        bad = [i for i in ran if items[i].status != SGW_OK]
        if bad:
            _check(items[bad[0]].status, jobs[bad[0]][0].ctx)
        raise SgwError(code, "batch rejected: every item needs its own context")
    return [(o[0][..., 0] + 1j * o[0][..., 1], o[1], items[i].ms) for i, o in enumerate(outs)]
