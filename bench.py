#!/usr/bin/env python3
"""Benchmark of the sGW/sROI hot path on one MI355X.

Workload: the Si35H36-shaped cluster on a 64^3 grid (h = 0.5 bohr, kinetic
cutoff 28 Ha), local Gaussian pseudopotentials plus s/p Kleinman-Bylander
projectors (176 projectors, 88 occupied states), N_eta = 64 stochastic
occupied orbitals per Monte Carlo sample, TDH linear response over 400 steps
of dt = 0.05 a.u., N_xi = 10000 sparse functions at f_g = 0.003, the gapped
filter (cutoff spread over the HOMO-LUMO gap, 1e-7 at the gap edges),
complex FP32 bulk arithmetic.

One step = the whole hot path (white noise, filter, TDH with xi overlaps,
time ordering, zeta propagation, contraction) for a batch of samples, through
sgw_sigma_estimate.  The QP energy of the HOMO and its per-sample spread give
GPU-seconds per QP energy at +-0.03 eV.  Printed as one JSON line.

Forms: "plain" (complex FP32, the value; --steps timed steps), and, over
--form-steps steps each: "c64_graphs" (the same with launch sequences
replayed from HIP graphs), "bf16x2kb_graphs" (projector GEMMs on BF16 MFMA
with the state operand split into two BF16 terms, graphs), "homo_lumo_shared"
(both states from one pass); "cfg1_32_c128_plain" (the 32^3 Gaussian-well
system in complex FP64); "cfg3_128_bf16" (the 128^3 cluster shape with 512
TDH orbitals per launch, complex FP64 against split and plain BF16 projector
GEMMs on the same samples, shortened time axis); with --cv N,
"control_variate": N more samples are split into a fit set and an evaluation
set, a network on |<phi_k|zeta>|^2 over the 64 near-gap states is trained on
the fit set and its mean taken over --cv-cheap cheap samples.  --counters
runs only the workload of the rocprofv3 counter profiles.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HA_EV = 27.211386245988
METRIC = ("GPU-s per QP energy at +/-0.03 eV (plain vs chosen); "
          "Hpsi Gpt*vec/s vs HBM roofline")
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0      # dense BF16 MFMA of one MI355X
# algorithmic bytes per (grid point x complex vector) of the dominant kernel,
# the inverse xy-plane pass carrying the Chebyshev update: the real FP32
# filter term reads v_n, v_{n-1}, acc and writes v_{n+1}, acc (20 B per real
# vector), two real vectors per complex vector -> 40 B.
CHEB_ALGO_BYTES = 40.0
# H psi in complex FP32: read psi, write H psi
HPSI_ALGO_BYTES = 16.0
# HBM bytes per (grid point x complex vector) that the same kernel moves, from
# FETCH_SIZE + WRITE_SIZE hardware counters on the 260-vector filter launch,
# scaled by the counters' reading for a plain 256 MiB device copy.  Valid only
# for the kernel source it was measured on; None once that kernel changes.
CHEB_MEASURED_BYTES = 36.68
# The dominant kernel by time, the projector scatter psi += s B C' (the TDH's
# KB exponential twice per substep at 1024 vectors, every filter term at 260):
# algorithmic bytes per (grid point inside some projector's support x complex
# vector) = read and write of psi there, 16 B (the reads of B and C', under
# 2 % of that at these batch widths, are left out).  The kernel works on
# whole 512-point tiles; the support points (sgw_kb_stats) are the method's.
KB_SCATTER_ALGO_BYTES = 16.0
# the gather C = B^T psi reads psi on the support: 8 B per support pt x vector
KB_GATHER_ALGO_BYTES = 8.0
# counter bytes per touched-tile point x vector (FETCH_SIZE + WRITE_SIZE,
# scaled as above), the scatter and the gather at 1024 vectors; None once the
# kernel changes
KB_SCATTER_MEASURED_BYTES = 14.0
KB_GATHER_MEASURED_BYTES = 7.34


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=8, help="samples per step")
    ap.add_argument("--n-tau", type=int, default=400)
    ap.add_argument("--n-eta", type=int, default=64)
    ap.add_argument("--quick", action="store_true", help="short functional run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-terms", type=int, default=6,
                    help="filter terms timed for the CPU baseline sample")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the graph-replay forms (FP32, BF16 and split BF16 KB)")
    ap.add_argument("--no-states", action="store_true",
                    help="skip the HOMO + LUMO shared-pass form")
    ap.add_argument("--cv", type=int, default=0,
                    help="samples for the control-variate form (0: skip it)")
    ap.add_argument("--cv-cheap", type=int, default=200000)
    ap.add_argument("--form-steps", type=int, default=2,
                    help="timed steps of each secondary form (graph replay, BF16, states)")
    ap.add_argument("--form-warmup", type=int, default=1)
    ap.add_argument("--no-cfg1", action="store_true", help="skip the 32^3 complex FP64 form")
    ap.add_argument("--no-cfg3", action="store_true", help="skip the 128^3 BF16-MFMA form")
    ap.add_argument("--cfg3-ntau", type=int, default=40)
    ap.add_argument("--cfg4", action="store_true",
                    help="uneven-batch mode only (32 clusters 40^3..112^3, then 32 small ones)")
    ap.add_argument("--cfg4-ntau", type=int, default=400)
    ap.add_argument("--cfg4-workers", type=int, default=8)
    ap.add_argument("--cfg4-small-only", action="store_true")
    ap.add_argument("--ecut-study", action="store_true",
                    help="kinetic-cutoff tuning on the 64^3 cluster")
    ap.add_argument("--ecut-list", type=float, nargs="+", default=[16.0, 20.0, 28.0, 40.0, 0.0])
    ap.add_argument("--cfg5", action="store_true",
                    help="control-variate mode on the 160^3 Si705H300-shaped cluster")
    ap.add_argument("--cfg5-first", type=int, default=0)
    ap.add_argument("--cfg5-count", type=int, default=0)
    ap.add_argument("--cfg5-load", default="")
    ap.add_argument("--cfg5-out", default="")
    ap.add_argument("--cfg5-cheap", type=int, default=0)
    ap.add_argument("--counters", action="store_true",
                    help="counter-profile driver only: a 256 MiB device copy, filter terms "
                         "at the bench launch shape and H applications on --hpsi-nvec "
                         "vectors; meant to run under rocprofv3 --pmc")
    ap.add_argument("--terms", type=int, default=8, help="--counters: filter terms")
    ap.add_argument("--hpsi-nvec", type=int, default=1024, help="--counters: H batch")
    return ap.parse_args()


T_START = time.perf_counter()


def progress(msg):
    print(f"[{time.perf_counter() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def suggested_ncoef(sgw, e_homo, e_lumo, eps, emin, emax, tol):
    """Length of the gapped filter whose discarded tail is below tol."""
    import numpy as np
    for nmax in (2048, 4096, 8192, 16384, 32768):
        a = sgw.sgw_gapped_coefficients(e_homo, e_lumo, eps, emin, emax, nmax)
        tail = np.cumsum(np.abs(a[::-1]))[::-1]
        ok = np.nonzero(tail < tol)[0]
        if ok.size and ok[0] < nmax // 2:
            return int(ok[0])
    raise RuntimeError("filter too long")


def cpu_baseline(system, phi, p, n_terms, ncoef):
    """Time the FP64 oracle on a bounded sample of one Monte Carlo sample:
    n_terms filter terms on its 65 real vectors, 2 TDH substeps on its
    2 x 64 orbitals and 2 zeta propagation steps; scale each to the full
    counts (ncoef terms, n_tau steps)."""
    import numpy as np
    from oracle import chebyshev as cheb
    from oracle.grid import Grid
    from oracle.hamiltonian import Hamiltonian, Projectors
    from oracle.tdh import TDH, hartree
    from oracle import rng
    workers = os.cpu_count()
    g = Grid(system.grid.n, h=system.grid.h, workers=workers)
    pr = system.projectors
    P = Projectors(g, pr.pos, pr.atom_of, pr.l, pr.m, pr.rc, pr.ekb, pr.rcut_over_rc)
    H = Hamiltonian(g, system.v_loc, P, system.ecut)
    zb = rng.white_noise(p["seed"], rng.ZETA, 0, 0, g.N, g.dV)
    eb = np.stack([rng.white_noise(p["seed"], rng.ETA, 0, l, g.N, g.dV)
                   for l in range(p["n_eta"])])
    x = np.vstack([zb[None], eb])
    a = cheb.gapped_coefficients(p["e_homo"], p["e_lumo"], p["filter_eps"], p["emin"],
                                 p["emax"], n_terms)
    t0 = time.perf_counter()
    cheb.apply_series(H, a, p["emin"], p["emax"], x)
    t_filter = (time.perf_counter() - t0) / max(1, n_terms - 1) * (ncoef - 1)
    tdh = TDH(H, p["dt"] / p["m_sub"], 2.0 / p["n_eta"])
    st = tdh.start(eb[:p["n_eta"]], hartree(g, phi * zb))
    t0 = time.perf_counter()
    for _ in range(2):
        st = tdh.substep(*st)
    t_tdh = (time.perf_counter() - t0) / 2 * p["n_tau"] * p["m_sub"]
    b = cheb.propagator_coefficients(p["emin"], p["emax"], p["dt"])
    z = np.vstack([zb, zb]).astype(np.complex128)
    t0 = time.perf_counter()
    for _ in range(2):
        z = cheb.apply_series(H, b, p["emin"], p["emax"], z)
    t_zeta = (time.perf_counter() - t0) / 2 * p["n_tau"]
    total = t_filter + t_tdh + t_zeta
    sample = (f"one Monte Carlo sample extrapolated from {n_terms} filter terms "
              f"(x {ncoef}), 2 TDH substeps (x {p['n_tau'] * p['m_sub']}) and 2 zeta "
              f"steps (x {p['n_tau']}); FP64 numpy/scipy oracle, scipy.fft workers = "
              f"{workers}")
    return total, dict(filter=t_filter, tdh=t_tdh, zeta=t_zeta), workers, sample


def graph_form(args, s, phi, p, sigma1, sig_plain, homo, gam, precision):
    """The same samples with HIP-graph replay on a stream of its own, in the
    given precision (FP32, BF16 or split BF16 projector GEMMs): time per
    sample and the largest Sigma_c(t) difference from the plain form."""
    import numpy as np
    import torch
    from paper_2601_21005_amd import sgw
    st = torch.cuda.Stream()
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=precision,
                      ecut=s.ecut, max_nvec=256, stream=st.cuda_stream)
    ctx.use_graphs(True)
    B = args.batch
    W, K = args.form_warmup, min(args.form_steps, args.steps)
    for w in range(W):
        ctx.sigma_estimate(phi, n_zeta=B, first_sample=w * B, **p)
    torch.cuda.synchronize()
    sigs = []
    t0 = time.perf_counter()
    for k in range(K):
        # the same samples as the plain form's first K steps
        sigs.append(ctx.sigma_estimate(phi, n_zeta=B, first_sample=(args.warmup + k) * B, **p)[0])
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / (K * B)
    ctx.close()
    sig = np.concatenate(sigs)
    ref = sig_plain[:sig.shape[0]]
    d_sigma = float(np.max(np.abs(sig - ref)) / np.max(np.abs(ref)))
    return {"gpu_s_per_qp": t * (sigma1 / 0.03) ** 2, "gpu_s_per_sample": t, "steps": K,
            "sigma_t_max_rel_diff_vs_plain": d_sigma}


def states_form(args, ctx, phi2, p, homo, lumo, gam, t_sample):
    """HOMO and LUMO from one shared pass over the same samples: time per
    sample against two single-state runs, both QP energies, and the gap with
    its error bar from the per-sample differences (both states see every
    random set of a sample, so their noise is correlated)."""
    import numpy as np
    import torch
    from paper_2601_21005_amd import sgw
    B = args.batch
    W, K = args.form_warmup, min(args.form_steps, args.steps)
    for w in range(W):
        ctx.sigma_estimate_states(phi2, n_zeta=B, first_sample=w * B, **p)
    torch.cuda.synchronize()
    sigs, xs = [], []
    t0 = time.perf_counter()
    for k in range(K):
        sig, x, _ = ctx.sigma_estimate_states(phi2, n_zeta=B, first_sample=(args.warmup + k) * B,
                                              **p)
        sigs.append(sig)
        xs.append(x)
    torch.cuda.synchronize()
    sig, x = np.concatenate(sigs, axis=1), np.concatenate(xs, axis=1)
    n = sig.shape[1]
    t = (time.perf_counter() - t0) / n
    out, y = {}, []
    for k, (name, eks) in enumerate((("homo", homo), ("lumo", lumo))):
        eq, _, Z = sgw.sgw_qp_solve(sig[k].mean(0), p["dt"], gam, eks, x[k].mean())
        re_i = np.array([sgw.sgw_sigma_omega(si, p["dt"], gam, eq)[0].real for si in sig[k]])
        y.append(Z * (x[k] + re_i))
        out[f"eqp_{name}_eV"] = eq * HA_EV
    out["qp_gap_eV"] = out["eqp_lumo_eV"] - out["eqp_homo_eV"]
    out["gap_err_eV"] = float(np.std(y[1] - y[0], ddof=1) / np.sqrt(n) * HA_EV)
    out["gap_err_if_independent_eV"] = float(
        np.sqrt(np.var(y[0], ddof=1) + np.var(y[1], ddof=1)) / np.sqrt(n) * HA_EV)
    return {"gpu_s_per_sample_two_states": t, "speedup_vs_two_runs": 2 * t_sample / t,
            "samples": n, **out}


def features_roofline(ctx, phis, s, nsamp=262144, reps=3):
    """The control variate's feature GEMM on MFMA (BF16 operands, FP32
    accumulation): 64 states x N_g points x nsamp white-noise vectors whose
    signs the kernel draws in registers; 2 flop per multiply-add, HIP events on
    the context's stream (the default stream, torch's current one here)."""
    import torch
    from paper_2601_21005_amd import sgw
    k = 64
    i0 = max(0, s.n_occ - k // 2)
    phi = phis[i0:i0 + k].real.float().contiguous()
    out = torch.empty((nsamp, k), dtype=torch.float32, device="cuda")
    sgw.cv_features(ctx, phi, 7, 0, nsamp, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        sgw.cv_features(ctx, phi, 7, (r + 1) * nsamp, nsamp, out)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    tflops = 2.0 * k * s.grid.N * nsamp / t / 1e12
    return {"bound": "mfma", "kernel": "k_features (BF16 16x16x32)", "achieved": tflops,
            "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / BF16_PEAK_TFLOPS,
            "traffic": None, "samples": nsamp, "states": k, "avg_launch_us": t * 1e6}


def cv_form(args, ctx, s, phis, ev, phi, p, homo, eg, gam, t_sample, sigma1, Z):
    """Control variate: args.cv new samples split 3/8 train, 1/8 validation
    (early stopping), 1/4 fit of c (A), 1/4 evaluation (B); E[g] over
    args.cv_cheap cheap samples.  GPU-s per QP = sample time x samples needed
    at the reduced spread + feature and training time."""
    import numpy as np
    import torch
    from paper_2601_21005_amd import sgw, systems
    n = args.cv - args.cv % 8
    first = 4096
    t0 = time.perf_counter()
    sig, xs = [], []
    for b0 in range(0, n, args.batch):
        nb = min(args.batch, n - b0)
        a, x, _ = ctx.sigma_estimate(phi, n_zeta=nb, first_sample=first + b0, **p)
        sig.append(a)
        xs.append(x)
        if (b0 + nb) % 64 == 0 or b0 + nb == n:
            progress(f"control variate: {b0 + nb} / {n} samples")
    torch.cuda.synchronize()
    t_samples = time.perf_counter() - t0
    sig, xs = np.concatenate(sig), np.concatenate(xs)
    y = xs + np.array([sgw.sgw_sigma_omega(si, p["dt"], gam, eg)[0].real for si in sig])
    # input row: |<phi_k|zeta-bar>|^2 and the mean over l of |<phi_k|eta-bar_l>|^2
    # for the 32 states around the gap (HOMO - 15 ... LUMO + 15)
    k0 = max(0, s.n_occ - 16)
    sel = phis[k0:k0 + 32].float().contiguous()
    t1 = time.perf_counter()
    feats = torch.empty((n, 64), dtype=torch.float32, device="cuda")
    feats[:, :32] = sgw.cv_features(ctx, sel, p["seed"], first, n)
    sgw.cv_features_eta(ctx, sel, p["seed"], first, n, p["n_eta"], out=feats, col0=32)
    xn = feats.cpu().numpy().astype(np.float64)
    tr, va = slice(0, 3 * n // 8), slice(3 * n // 8, n // 2)
    A, B = slice(n // 2, 3 * n // 4), slice(3 * n // 4, n)
    mean, std = xn[tr].mean(axis=0), xn[tr].std(axis=0)
    std[std == 0] = 1.0
    ym, ysd = y[tr].mean(), y[tr].std()
    yt = torch.from_numpy(((y - ym) / ysd).astype(np.float32)).cuda()
    net = sgw.Mlp(systems.mlp_init(3))
    net.set_standardization(mean, std)
    best, best_loss = None, np.inf
    for _ in range(30):
        net.train(feats[tr].contiguous(), yt[tr].contiguous(), 10, lr=1e-3)
        gv = net.forward(feats[va].contiguous()).cpu().numpy().astype(np.float64)
        loss = float(np.mean((gv - (y[va] - ym) / ysd) ** 2))
        if loss < best_loss:
            best, best_loss = net.params(), loss
    net.close()
    net = sgw.Mlp(best)
    net.set_standardization(mean, std)
    g = net.forward(feats).cpu().numpy().astype(np.float64)
    gm, gv = sgw.cv_cheap_moments_mixed(ctx, net, sel, sel, p["seed"], p["n_eta"], first + n,
                                        args.cv_cheap, chunk=16384)
    torch.cuda.synchronize()
    t_cv = time.perf_counter() - t1
    net.close()
    r = sgw.sgw_cv_estimate(y[A], g[A], y[B], g[B], gm, gv, args.cv_cheap)
    nB = B.stop - B.start
    sd_cv = float(r["sigma_cv"] * np.sqrt(nB))       # per-sample spread of the CV form
    sigma1_cv = Z * sd_cv * 27.211386245988
    plain_sd = float(np.std(y[B], ddof=1))
    sigma1_plain_b = Z * plain_sd * 27.211386245988   # plain spread on the same set B
    return {"gpu_s_per_qp": t_sample * (sigma1_cv / 0.03) ** 2 + t_cv, "samples": n,
            "plain_gpu_s_per_qp_same_set": t_sample * (sigma1_plain_b / 0.03) ** 2,
            "rho2_A": r["rho2"], "variance_ratio_B": (sd_cv / plain_sd) ** 2,
            "fallback": r["fallback"], "sigma1_eV": sigma1_cv, "plain_sigma1_eV": sigma1,
            "feature_and_training_s": t_cv, "cheap_samples": args.cv_cheap,
            "sample_time_s": t_samples}


def hbm_ceilings(nbytes=2 << 30, reps=10):
    """Streaming rates that library kernels reach on plain access patterns
    (torch's elementwise kernels and the runtime's copy on buffers of nbytes):
    write only (fill), read-modify-write in place (add) and a copy between two
    buffers, in GB/s of algorithmic bytes.  They are lower bounds of what the
    device can stream, set beside the nominal 8 TB/s: a kernel that reads and
    rewrites psi in place, like the projector scatter, is held to the
    read-modify-write rate."""
    import torch
    n = nbytes // 8
    a = torch.zeros(n, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    f = a.view(torch.float32)

    def rate(fn, moved):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    out = {"write": rate(lambda: a.fill_(0), nbytes),
           "rmw": rate(lambda: f.add_(1.0), 2 * nbytes),
           "copy": rate(lambda: b.copy_(a), 2 * nbytes), "unit": "GB/s",
           "bytes": nbytes, "method": "torch fill_ / add_ / copy_ on complex64 buffers"}
    del a, b, f
    torch.cuda.empty_cache()
    return out


def rocfft_comparison(s, nv=256, reps=10):
    """The library's three FFT passes against rocFFT on the same batch: H
    applied by a local-only context (forward xy plane, z pencil with the
    kinetic multiplier and the inverse, inverse xy plane with V psi) against
    torch.fft.fftn + ifftn (rocFFT) on 256 complex FP32 vectors of the 64^3
    grid, HIP events on the default stream that both run on."""
    import torch
    from paper_2601_21005_amd import sgw
    n = s.grid.n
    ctx = sgw.Context(n, s.grid.h, s.v_loc, None, precision=sgw.SGW_C64, ecut=s.ecut,
                      max_nvec=nv)
    x = torch.randn((nv, s.grid.N), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    x3 = x.view(nv, n, n, n)

    def timed(f):
        f()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    ours = timed(lambda: ctx.apply_H(x, y))
    roc = timed(lambda: torch.fft.ifftn(torch.fft.fftn(x3, dim=(1, 2, 3)), dim=(1, 2, 3)))
    ctx.close()
    del x, y
    ptv = nv * s.grid.N
    return {"vectors": nv, "grid": n, "library_local_H_ms": ours,
            "rocfft_fftn_ifftn_ms": roc, "library_gptvec_per_s": ptv / ours / 1e6,
            "rocfft_gptvec_per_s": ptv / roc / 1e6, "speedup": roc / ours,
            "note": "library: forward FFT, T(k), inverse FFT and V psi in three passes; "
                    "rocFFT: forward and inverse transforms only (no multiplier, no V psi)"}


def filter_coefficient_dump(sgw, homo, lumo, eps, emin, emax, ncoef):
    """Magnitudes |a_n| of the occupied-space filter's Chebyshev coefficients
    at log-spaced n (the analogue of the paper's coefficient plot, Fig. 3):
    the gapped filter in use (erfc step, 1 - eps / eps at the band edges)
    beside a Fermi function with the same edge values (beta = 2 ln((1-eps)/
    eps) / gap), each with the length at which its discarded tail drops below
    1e-7."""
    import numpy as np
    nmax = 4 * ncoef
    ag = np.abs(sgw.sgw_gapped_coefficients(homo, lumo, eps, emin, emax, nmax))
    mu, beta = 0.5 * (homo + lumo), 2.0 * np.log((1 - eps) / eps) / (lumo - homo)
    fer = 8192
    while True:
        af = np.abs(sgw.sgw_fermi_coefficients(mu, beta, emin, emax, fer))
        tail = np.cumsum(af[::-1])[::-1]
        ok = np.nonzero(tail < 1e-7)[0]
        if (ok.size and ok[0] < fer // 2) or fer >= 65536:
            break
        fer *= 2
    nf = int(ok[0]) if ok.size else None
    pts = sorted({0, 1} | {int(round(x)) for x in np.geomspace(2, nmax - 1, 24)})
    return {"gapped_ncoef": ncoef, "fermi_beta": beta, "fermi_ncoef": nf,
            "n": pts, "gapped_abs": [float(ag[i]) for i in pts],
            "fermi_abs": [float(af[i]) if i < af.size else None for i in pts]}


def qp_spread(sgw, sig, x, p, eks):
    """QP energy (graphical root of Eq. 6), Z and the per-sample spread sigma_1
    (eV) of the linearised per-sample QP correction Z (X_i + Re Sigma_i(w))."""
    import numpy as np
    gam = 3.0 / (p["n_tau"] * p["dt"])
    eg, el, Z = sgw.sgw_qp_solve(sig.mean(0), p["dt"], gam, eks, x.mean())
    re_i = np.array([sgw.sgw_sigma_omega(si, p["dt"], gam, eg)[0].real for si in sig])
    return eg, Z, float(Z * np.std(x + re_i, ddof=1) * HA_EV)


def cfg1_form(args):
    """Plain sGW in complex FP64 on the 32^3 Gaussian-well system (8 wells of
    2 Ha, width 1 bohr; 8 occupied states): 8 samples per step, N_eta = 8,
    Fermi filter (beta = 50/Ha, mu mid-gap, coefficient tail < 1e-10), 100
    output steps of 0.2 au (TDH: 4 Strang substeps of 0.05), N_xi = 10000 at
    f_g = 0.003.  GPU-s per HOMO QP energy at +-0.03 eV."""
    import numpy as np
    import torch
    from paper_2601_21005_amd import ksinput, sgw, systems
    s = systems.gaussian_wells()
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, None, precision=sgw.SGW_C128, max_nvec=96)
    emin, emax = ctx.lanczos_bounds(60, seed=1, pad=0.01)
    ev, phis, _ = ksinput.lowest_states(ctx, s.n_occ + 1, emin, emax, s.grid.h ** 3)
    homo, lumo = float(ev[s.n_occ - 1]), float(ev[s.n_occ])
    phi = phis[s.n_occ - 1].cpu().numpy()
    mu, beta = 0.5 * (homo + lumo), 50.0
    ncoef = 2048
    while True:
        a = sgw.sgw_fermi_coefficients(mu, beta, emin, emax, ncoef)
        tail = np.cumsum(np.abs(a[::-1]))[::-1]
        ok = np.nonzero(tail < 1e-10)[0]
        if ok.size and ok[0] < ncoef // 2:
            ncoef = int(ok[0])
            break
        ncoef *= 2
    p = dict(seed=1001, n_eta=8, n_tau=100, dt=0.2, m_sub=4, mu=mu, beta=beta, ncoef=ncoef,
             emin=emin, emax=emax, n_xi=10000, f_g=0.003, mode=0, filter=0)
    B, K = 8, max(2, args.form_steps)
    ctx.sigma_estimate(phi, n_zeta=B, first_sample=0, **p)         # warm-up
    torch.cuda.synchronize()
    sigs, xs = [], []
    t0 = time.perf_counter()
    for k in range(K):
        sig, x, _ = ctx.sigma_estimate(phi, n_zeta=B, first_sample=(1 + k) * B, **p)
        sigs.append(sig)
        xs.append(x)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / (K * B)
    ctx.close()
    eg, Z, s1 = qp_spread(sgw, np.concatenate(sigs), np.concatenate(xs), p, homo)
    return {"workload": "32^3 Gaussian wells, complex FP64, N_eta=8, Fermi beta=50, "
                        "100 x 0.2 au (4 TDH substeps each), N_xi=10000",
            "samples": K * B, "ncoef": ncoef, "gpu_s_per_sample": t, "sigma1_eV": s1,
            "gpu_s_per_qp": t * (s1 / 0.03) ** 2, "eqp_homo_eV": eg * HA_EV,
            "eps_ks_homo_eV": homo * HA_EV}


def cfg3_form(args):
    """The 128^3 cluster shape (Si357H204 stand-in for Si353H196, h = 0.6
    bohr, 1632 projectors, 816 occupied states): 32 samples x N_eta = 8, so
    the TDH batch is 32 x 8 x 2 = 512 orbitals in one launch; gapped filter
    (transition over >= 0.3 Ha around mid-gap, tail < 1e-7); N_xi = 10000 at
    f_g = 0.003; the time axis shortened to --cfg3-ntau steps of 0.05 au.
    The same samples in complex FP64 (the reference), and with the projector
    GEMMs on BF16 MFMA (split BF16 x 2 and plain BF16) in complex FP32:
    per-sample time, GPU-s per HOMO QP energy at +-0.03 eV and the QP error
    against the FP64 run."""
    import numpy as np
    import torch
    from paper_2601_21005_amd import ksinput, sgw, systems
    s = systems.si357h204()
    dV = s.grid.h ** 3

    def ctx_of(prec):
        return sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=prec,
                           ecut=s.ecut, max_nvec=512)
    c64 = ctx_of(sgw.SGW_C64)
    emin, emax = c64.lanczos_bounds(60, seed=1, pad=0.01)
    t0 = time.perf_counter()
    ev, phis, _ = ksinput.lowest_states(c64, s.n_occ + 1, emin, emax, dV, tol=1e-4, maxit=80)
    t_ks = time.perf_counter() - t0
    c64.close()
    homo, lumo = float(ev[s.n_occ - 1]), float(ev[s.n_occ])
    phi = phis[s.n_occ - 1].cpu().numpy()
    del phis
    mid, half = 0.5 * (homo + lumo), max(0.5 * (lumo - homo), 0.15)
    eh, el = mid - half, mid + half
    ncoef = suggested_ncoef(sgw, eh, el, 1e-7, emin, emax, 1e-7)
    p = dict(seed=1003, n_eta=8, n_tau=args.cfg3_ntau, dt=0.05, m_sub=1, ncoef=ncoef,
             emin=emin, emax=emax, n_xi=10000, f_g=0.003, mode=0, filter=1, e_homo=eh,
             e_lumo=el, filter_eps=1e-7)
    out = {"workload": f"Si357H204 stand-in, 128^3 h=0.6, 1632 KB projectors, 32 samples x "
                       f"N_eta=8 (512 TDH orbitals per launch), N_tau={p['n_tau']} x 0.05 au "
                       f"(shortened from 400), N_xi=10000, gapped filter",
           "ncoef": ncoef, "ks_states_s": t_ks, "forms": {}}
    ref = None
    for prec, name in ((sgw.SGW_C128, "c128"), (sgw.SGW_C64_BF16X2KB, "c64_bf16x2kb"),
                       (sgw.SGW_C64_BF16KB, "c64_bf16kb")):
        ctx = ctx_of(prec)
        ctx.sigma_estimate(phi, n_zeta=2, first_sample=1000, **dict(p, n_tau=2))   # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sig, x, ms = ctx.sigma_estimate(phi, n_zeta=32, first_sample=0, **p)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t1) / 32
        ctx.close()
        eg, Z, s1 = qp_spread(sgw, sig, x, p, homo)
        f = {"gpu_s_per_sample": t, "sigma1_eV": s1, "gpu_s_per_qp": t * (s1 / 0.03) ** 2,
             "eqp_homo_eV": eg * HA_EV, "phase_ms": {"filter": ms[0], "tdh": ms[1]}}
        if ref is None:
            ref = (eg, sig)
        else:
            f["qp_err_vs_c128_meV"] = abs(eg - ref[0]) * HA_EV * 1e3
            f["sigma_t_max_rel_diff_vs_c128"] = float(np.max(np.abs(sig - ref[1])) /
                                                      np.max(np.abs(ref[1])))
        out["forms"][name] = f
        progress(f"cfg3 {name}: {t:.3f} s per sample")
    return out


def cfg4_mode(args):
    """Uneven batch as configured: 32 seeded H-capped Si clusters (17 to 147
    Si) on grids 40^3 ... 112^3 (h = 0.6 bohr) with 16 to 128 stochastic
    orbitals each, complex FP32, one Monte Carlo sample per cluster, N_tau =
    400 x 0.05 au, N_xi = 10000 at f_g = 0.003, gapped filter.  Times the
    clusters one after another (one stream each, eager) and through
    sgw_batch_sigma_estimate (host workers, one stream per cluster, graph
    replay), checks that every result is bitwise the sequential one, then
    does the same for 32 small clusters (Si17H36 on 40^3 with 16 orbitals),
    the regime where single launches leave most of the chip idle.  Prints
    one JSON line."""
    import numpy as np
    import torch
    from paper_2601_21005_amd import sgw, systems

    def run(batch, label, n_tau, workers):
        jobs, meta = [], []
        for i, (s, neta) in enumerate(batch):
            st = torch.cuda.Stream()
            ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors,
                              precision=sgw.SGW_C64, ecut=s.ecut, max_nvec=256,
                              stream=st.cuda_stream)
            lo, hi = ctx.lanczos_bounds(30, seed=1, pad=0.01)
            mid = lo + 0.12 * (hi - lo)
            ncoef = suggested_ncoef(sgw, mid - 0.15, mid + 0.15, 1e-7, lo, hi, 1e-7)
            rs = np.random.default_rng(i)
            phi = rs.standard_normal(s.grid.N)
            phi /= np.sqrt(s.grid.h ** 3 * np.sum(phi * phi))
            kw = dict(seed=1005 + i, n_zeta=1, n_eta=neta, n_tau=n_tau, dt=0.05, m_sub=1,
                      ncoef=ncoef, emin=lo, emax=hi, n_xi=10000, f_g=0.003, mode=0, filter=1,
                      e_homo=mid - 0.15, e_lumo=mid + 0.15, filter_eps=1e-7)
            jobs.append((ctx, phi, kw))
            meta.append({"name": s.name, "grid": s.grid.n, "n_eta": neta, "ncoef": ncoef})
        torch.cuda.synchronize()
        # warm-up of every context (autotuning, allocation) on a short time axis
        for ctx, phi, kw in jobs:
            ctx.sigma_estimate(phi, **dict(kw, n_tau=2))
        torch.cuda.synchronize()
        progress(f"{label}: {len(jobs)} contexts ready")
        t0 = time.perf_counter()
        seq = []
        for k, (ctx, phi, kw) in enumerate(jobs):
            t1 = time.perf_counter()
            seq.append(ctx.sigma_estimate(phi, **kw))
            torch.cuda.synchronize()
            meta[k]["alone_s"] = time.perf_counter() - t1
        t_seq = time.perf_counter() - t0
        progress(f"{label}: sequential {t_seq:.1f} s")
        for ctx, phi, kw in jobs:
            # capture the graphs: the filter pair, one TDH output step and the
            # zeta sweep of 8 output steps (every sweep of n_tau = 400 reuses it)
            ctx.use_graphs(True)
            ctx.sigma_estimate(phi, **dict(kw, n_tau=16))
            ctx.sigma_estimate(phi, **dict(kw, n_tau=16))
        torch.cuda.synchronize()
        progress(f"{label}: graphs captured")
        t0 = time.perf_counter()
        bat = sgw.batch_sigma_estimate(jobs, nworkers=workers)
        torch.cuda.synchronize()
        t_bat = time.perf_counter() - t0
        progress(f"{label}: batched {t_bat:.1f} s")
        same = all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
                   for a, b in zip(seq, bat))
        for m, b in zip(meta, bat):
            m["batched_ms"] = b[2]
        for ctx, _, _ in jobs:
            ctx.close()
        return {"clusters": len(jobs), "workers": workers, "n_tau": n_tau,
                "sequential_s": t_seq, "batched_s": t_bat, "speedup": t_seq / t_bat,
                "bitwise_equal": bool(same), "per_cluster": meta}

    out = {"mode": "cfg4", "workers": args.cfg4_workers,
           "gpu_max_hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "runtime default")}
    if not args.cfg4_small_only:
        out["uneven_32"] = run(systems.uneven_batch_spread(32), "uneven", args.cfg4_ntau,
                               args.cfg4_workers)
    small = [systems.cluster_model(*systems.si_cluster(17, seed=2000 + i), n=40, h=0.6,
                                   ecut=28.0, name="Si17H36") for i in range(32)]
    out["small_32_at_40"] = run([(s, 16) for s in small], "small", args.cfg4_ntau,
                                args.cfg4_workers)
    print(json.dumps(out), flush=True)


def cfg5_mode(args):
    """Learned control variate on the Si705H300-shaped cluster (160^3, h = 0.6
    bohr, 3120 projectors, 1560 occupied states), complex FP32.  Plain sGW
    samples (N_eta = 8, N_tau = 400 x 0.05 au, N_xi = 10000 at f_g = 0.003,
    gapped filter with its transition over >= 0.3 Ha around mid-gap) in
    batches of 32 (512 TDH orbitals per launch), with the features of every
    sample ([|<phi_k|zeta-bar>|^2, mean_l |<phi_k|eta-bar_l>|^2] over the 32
    states HOMO - 15 ... LUMO + 15).  Samples computed in earlier calls are
    read from --cfg5-load (npz files written by --cfg5-out); with
    --cfg5-cheap M > 0 the network is trained and evaluated (3/8 train, 1/8
    validation, 1/4 fit of c, 1/4 evaluation) and E[g] taken over M cheap
    samples.  Prints one JSON line."""
    import hashlib
    import numpy as np
    import torch
    from paper_2601_21005_amd import ksinput, sgw, systems
    t0 = time.perf_counter()
    s = systems.si705h300()
    dV = s.grid.h ** 3
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=sgw.SGW_C64,
                      ecut=s.ecut, max_nvec=512)
    emin, emax = ctx.lanczos_bounds(60, seed=1, pad=0.01)
    progress(f"cfg5: context and interval [{emin:.4f}, {emax:.4f}] "
             f"({time.perf_counter() - t0:.1f} s)")
    t1 = time.perf_counter()
    ev, phis, res, its = ksinput.lowest_states_lean(ctx, s.n_occ + 16, emin, emax, dV)
    t_ks = time.perf_counter() - t1
    torch.cuda.empty_cache()
    homo, lumo = float(ev[s.n_occ - 1]), float(ev[s.n_occ])
    sel = phis[s.n_occ - 16:s.n_occ + 16].contiguous()
    phi = phis[s.n_occ - 1].double().cpu().numpy()
    del phis
    torch.cuda.empty_cache()
    digest = hashlib.sha256(sel.cpu().numpy().tobytes()).hexdigest()[:16]
    progress(f"cfg5: {s.n_occ + 16} KS states in {t_ks:.1f} s ({its} iterations, max residual "
             f"{res.max():.1e}); HOMO {homo:.6f} LUMO {lumo:.6f} Ha; states digest {digest}")
    mid, half = 0.5 * (homo + lumo), max(0.5 * (lumo - homo), 0.15)
    eh, el = mid - half, mid + half
    ncoef = suggested_ncoef(sgw, eh, el, 1e-7, emin, emax, 1e-7)
    p = dict(seed=1006, n_eta=8, n_tau=400, dt=0.05, m_sub=1, ncoef=ncoef, emin=emin,
             emax=emax, n_xi=10000, f_g=0.003, mode=0, filter=1, e_homo=eh, e_lumo=el,
             filter_eps=1e-7)
    B = 32
    sig_l, x_l, f_l, idx_l = [], [], [], []
    t_samples, n_new = 0.0, 0
    for f in (args.cfg5_load.split(",") if args.cfg5_load else []):
        d = np.load(f)
        if str(d["digest"]) != digest:
            raise RuntimeError(f"{f}: KS states differ from this run's ({d['digest']} != {digest})")
        sig_l.append(d["sig"]); x_l.append(d["x"]); f_l.append(d["feat"]); idx_l.append(d["idx"])
        t_samples += float(d["seconds"])
    for b0 in range(args.cfg5_first, args.cfg5_first + args.cfg5_count, B):
        nb = min(B, args.cfg5_first + args.cfg5_count - b0)
        t2 = time.perf_counter()
        sig, x, _ = ctx.sigma_estimate(phi, n_zeta=nb, first_sample=b0, **p)
        torch.cuda.synchronize()
        t_samples += time.perf_counter() - t2
        n_new += nb
        feats = torch.empty((nb, 64), dtype=torch.float32, device="cuda")
        feats[:, :32] = sgw.cv_features(ctx, sel, p["seed"], b0, nb)
        sgw.cv_features_eta(ctx, sel, p["seed"], b0, nb, p["n_eta"], out=feats, col0=32)
        sig_l.append(sig); x_l.append(x); f_l.append(feats.cpu().numpy())
        idx_l.append(np.arange(b0, b0 + nb))
        progress(f"cfg5: samples {b0} .. {b0 + nb - 1} ({(time.perf_counter() - t2) / nb:.2f} s "
                 f"each)")
    sig, x = np.concatenate(sig_l), np.concatenate(x_l)
    feat, idx = np.concatenate(f_l), np.concatenate(idx_l)
    if args.cfg5_out and n_new:
        new = slice(sig.shape[0] - n_new, sig.shape[0])
        np.savez_compressed(args.cfg5_out, sig=sig[new], x=x[new], feat=feat[new], idx=idx[new],
                            digest=digest, seconds=t_samples - sum(
                                float(np.load(f)["seconds"]) for f in
                                (args.cfg5_load.split(",") if args.cfg5_load else [])))
    n = sig.shape[0]
    t_sample = t_samples / n
    out = {"mode": "cfg5", "workload": "Si705H300-shaped cluster, 160^3 h=0.6, 3120 KB "
                                       "projectors, N_eta=8, TDH 400 x 0.05 au, N_xi=10000, "
                                       "gapped filter, complex FP32",
           "samples": n, "ncoef": ncoef, "homo_lumo_Ha": [homo, lumo],
           "interval_Ha": [emin, emax], "ks_states_s": t_ks, "states_digest": digest,
           "gpu_s_per_sample": t_sample}
    gam = 3.0 / (p["n_tau"] * p["dt"])
    eg, el, Z = sgw.sgw_qp_solve(sig.mean(0), p["dt"], gam, homo, x.mean())
    y = x + np.array([sgw.sgw_sigma_omega(si, p["dt"], gam, eg)[0].real for si in sig])
    sd = float(Z * np.std(y, ddof=1) * HA_EV)
    out.update({"eqp_homo_eV": eg * HA_EV, "Z": Z, "plain_sigma1_eV": sd,
                "plain_gpu_s_per_qp": t_sample * (sd / 0.03) ** 2})
    if args.cfg5_cheap > 0 and n >= 64:
        t3 = time.perf_counter()
        n8 = n - n % 8
        tr, va = slice(0, 3 * n8 // 8), slice(3 * n8 // 8, n8 // 2)
        A, Bs = slice(n8 // 2, 3 * n8 // 4), slice(3 * n8 // 4, n8)
        mean, std = feat[tr].mean(axis=0), feat[tr].std(axis=0)
        std[std == 0] = 1.0
        ym, ysd = y[tr].mean(), y[tr].std()
        xt = torch.from_numpy(feat.astype(np.float32)).cuda()
        yt = torch.from_numpy(((y - ym) / ysd).astype(np.float32)).cuda()
        net = sgw.Mlp(systems.mlp_init(3))
        net.set_standardization(mean, std)
        best, best_loss = None, np.inf
        for _ in range(30):
            net.train(xt[tr].contiguous(), yt[tr].contiguous(), 10, lr=1e-3)
            gv = net.forward(xt[va].contiguous()).cpu().numpy().astype(np.float64)
            loss = float(np.mean((gv - (y[va] - ym) / ysd) ** 2))
            if loss < best_loss:
                best, best_loss = net.params(), loss
        net.close()
        net = sgw.Mlp(best)
        net.set_standardization(mean, std)
        g = net.forward(xt).cpu().numpy().astype(np.float64)
        t_train = time.perf_counter() - t3
        t4 = time.perf_counter()
        # cheap samples: fresh sample indices from 4096 on (the plain ones are below)
        M = min(args.cfg5_cheap, (1 << 20) - 4096)
        gm, gv = sgw.cv_cheap_moments_mixed(ctx, net, sel, sel, p["seed"], p["n_eta"], 4096, M,
                                            chunk=8192)
        torch.cuda.synchronize()
        t_cheap = time.perf_counter() - t4
        net.close()
        r = sgw.sgw_cv_estimate(y[A], g[A], y[Bs], g[Bs], gm, gv, M)
        nB = Bs.stop - Bs.start
        sd_cv = float(r["sigma_cv"] * np.sqrt(nB))
        plain_B = float(np.std(y[Bs], ddof=1))
        s_cv, s_pl = Z * sd_cv * HA_EV, Z * plain_B * HA_EV
        out["control_variate"] = {
            "train": tr.stop, "validation": va.stop - va.start, "fit_A": A.stop - A.start,
            "eval_B": nB, "cheap_samples": M, "rho2_A": r["rho2"],
            "variance_ratio_B": (sd_cv / plain_B) ** 2, "fallback": r["fallback"],
            "cv_estimate": r["estimate"], "plain_estimate": r["plain"],
            "sigma1_cv_eV": s_cv, "sigma1_plain_B_eV": s_pl,
            "train_s": t_train, "cheap_s": t_cheap,
            "gpu_s_per_qp_cv": t_sample * (s_cv / 0.03) ** 2 + t_train + t_cheap,
            "gpu_s_per_qp_plain_same_set": t_sample * (s_pl / 0.03) ** 2}
        progress(f"cfg5: control variate ratio {(sd_cv / plain_B) ** 2:.3f}")
    ctx.close()
    print(json.dumps(out), flush=True)


def ecut_mode(args):
    """Kinetic-cutoff tuning on the 64^3 cluster (Sec. 3 clips T(k) to bound
    the spectral width): for each cutoff the Lanczos interval, the lengths of
    the gapped filter and of the one-step propagator, the KS HOMO/LUMO, the
    time per sample and the HOMO QP energy from the same 16 samples (N_eta =
    64, N_tau = 100, N_xi = 10000), against the unclipped operator."""
    import numpy as np
    import torch
    from paper_2601_21005_amd import ksinput, sgw, systems
    rows = []
    for ecut in args.ecut_list:
        s = systems.si35h36(ecut=ecut)
        ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=sgw.SGW_C64,
                          ecut=s.ecut, max_nvec=256)
        emin, emax = ctx.lanczos_bounds(60, seed=1, pad=0.01)
        ev, phis, _ = ksinput.lowest_states(ctx, s.n_occ + 1, emin, emax, s.grid.h ** 3)
        homo, lumo = float(ev[s.n_occ - 1]), float(ev[s.n_occ])
        phi = phis[s.n_occ - 1].cpu().numpy()
        del phis
        ncoef = suggested_ncoef(sgw, homo, lumo, 1e-7, emin, emax, 1e-7)
        nprop = len(sgw.sgw_propagator_coefficients(emin, emax, 0.05, 1e-14))
        p = dict(seed=1002, n_eta=64, n_tau=100, dt=0.05, m_sub=1, ncoef=ncoef, emin=emin,
                 emax=emax, n_xi=10000, f_g=0.003, mode=0, filter=1, e_homo=homo, e_lumo=lumo,
                 filter_eps=1e-7)
        ctx.sigma_estimate(phi, n_zeta=8, first_sample=1000, **dict(p, n_tau=2))   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sig, x = [], []
        for b in range(2):
            a, xx, _ = ctx.sigma_estimate(phi, n_zeta=8, first_sample=8 * b, **p)
            sig.append(a)
            x.append(xx)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / 16
        ctx.close()
        sig, x = np.concatenate(sig), np.concatenate(x)
        eg, Z, s1 = qp_spread(sgw, sig, x, p, homo)
        rows.append({"ecut_Ha": ecut, "interval_Ha": [emin, emax], "ncoef": ncoef,
                     "prop_terms": nprop, "homo_Ha": homo, "lumo_Ha": lumo,
                     "gpu_s_per_sample": t, "eqp_homo_eV": eg * HA_EV, "sigma1_eV": s1})
        progress(f"ecut {ecut}: [{emin:.3f}, {emax:.3f}] ncoef {ncoef} eqp {eg * HA_EV:.4f} eV "
                 f"{t:.3f} s/sample")
    print(json.dumps({"mode": "ecut", "rows": rows}), flush=True)


def counters_driver(args):
    """Workload for rocprofv3 counter runs (one counter set per run): a plain
    256 MiB device copy (the reference that scales FETCH_SIZE / WRITE_SIZE to
    bytes), the filter on the bench launch shape (260 complex vectors = 8
    samples x 65 real orbitals; terms - 1 launches of the Chebyshev plane
    pass) and three H applications on --hpsi-nvec vectors (the TDH's launch
    shape of the projector kernels is 1024)."""
    import numpy as np
    import torch
    from paper_2601_21005_amd import sgw, systems
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy bytes read {a.numel() * 4} written {b.numel() * 4}", flush=True)
    del a, b
    s = systems.si35h36()
    nvec = 260
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=sgw.SGW_C64,
                      ecut=s.ecut, max_nvec=max(nvec, args.hpsi_nvec))
    print(f"kb layout {ctx.kb_stats()}", flush=True)
    lo, hi = ctx.bounds(0.01)
    coef = sgw.sgw_fermi_coefficients(-4.65, 66.0, lo, hi, args.terms)
    x = torch.randn((nvec, s.grid.N), dtype=torch.complex64, device="cuda")
    x /= float(np.sqrt(s.grid.N))
    ctx.fermi_filter(x, coef, lo, hi)
    torch.cuda.synchronize()
    print(f"filter nvec {nvec} terms {args.terms} N {s.grid.N}", flush=True)
    del x
    if args.hpsi_nvec > 0:
        y = torch.randn((args.hpsi_nvec, s.grid.N), dtype=torch.complex64, device="cuda")
        hy = torch.empty_like(y)
        for _ in range(3):
            ctx.apply_H(y, hy)
        torch.cuda.synchronize()
        print(f"H psi nvec {args.hpsi_nvec}: 3 applications", flush=True)
    ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the samples are independent, so several GPUs would each run their own "
              "share of them and only the final sums would be combined)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2601_21005_amd import ksinput, sgw, systems
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.counters:
        counters_driver(args)
        return
    if args.cfg4:
        cfg4_mode(args)
        return
    if args.cfg5:
        cfg5_mode(args)
        return
    if args.ecut_study:
        ecut_mode(args)
        return
    if args.quick:
        args.n_tau, args.n_eta, args.batch = 20, 8, 2

    s = systems.si35h36()
    dV = s.grid.h ** 3
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=sgw.SGW_C64,
                      ecut=s.ecut, max_nvec=256)
    # spectral interval by Lanczos on the device (60 steps, 1% pad), as the
    # paper obtains it by power iteration; the rigorous interval is ~17% wider
    emin, emax = ctx.lanczos_bounds(60, seed=1, pad=0.01)
    nst = s.n_occ + 16 if args.cv else s.n_occ + 1
    ev, phis, res = ksinput.lowest_states(ctx, nst, emin, emax, dV)
    homo, lumo = float(ev[s.n_occ - 1]), float(ev[s.n_occ])
    gap = lumo - homo
    phi = phis[s.n_occ - 1].cpu().numpy()
    eps = 1e-7
    ncoef = suggested_ncoef(sgw, homo, lumo, eps, emin, emax, 1e-7)
    fcoef = filter_coefficient_dump(sgw, homo, lumo, eps, emin, emax, ncoef)
    if args.quick:
        ncoef = min(ncoef, 400)
    p = dict(seed=1002, n_eta=args.n_eta, n_tau=args.n_tau, dt=0.05, m_sub=1, ncoef=ncoef,
             emin=emin, emax=emax, n_xi=10000, f_g=0.003, mode=0, filter=1, e_homo=homo,
             e_lumo=lumo, filter_eps=eps)
    B = args.batch

    progress(f"setup done: interval [{emin:.4f}, {emax:.4f}], {ncoef} filter terms")
    for w in range(args.warmup):
        ctx.sigma_estimate(phi, n_zeta=B, first_sample=w * B, **p)
        progress(f"warm-up {w + 1}/{args.warmup}")
    torch.cuda.synchronize()
    ctx.kernel_timer(sgw.SGW_TIMER_CHEB_PLANE | sgw.SGW_TIMER_KB_SCATTER |
                     sgw.SGW_TIMER_KB_GATHER)
    sigs, xs, phases = [], [], np.zeros(6)
    t0 = time.perf_counter()
    for k in range(args.steps):
        sig, x, ms = ctx.sigma_estimate(phi, n_zeta=B, first_sample=(args.warmup + k) * B, **p)
        sigs.append(sig)
        xs.append(x)
        phases += ms
        progress(f"step {k + 1}/{args.steps}: {ms[5]:.0f} ms")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ctx.kernel_timer(0)
    k_ms, k_launch, k_pts = ctx.kernel_timer_read(sgw.SGW_TIMER_CHEB_PLANE)
    s_ms, s_launch, s_pts = ctx.kernel_timer_read(sgw.SGW_TIMER_KB_SCATTER)
    g_ms, g_launch, g_pts = ctx.kernel_timer_read(sgw.SGW_TIMER_KB_GATHER)
    kbs = ctx.kb_stats()
    # timer points are touched-tile points x vectors; the method's are the
    # support points x vectors
    support_frac = kbs["support_points"] / kbs["tile_points"]

    sig = np.concatenate(sigs)
    x = np.concatenate(xs)
    nsamp = sig.shape[0]
    gam = 3.0 / (p["n_tau"] * p["dt"])
    eg, el, Z = sgw.sgw_qp_solve(sig.mean(0), p["dt"], gam, homo, x.mean())
    re_i = np.array([sgw.sgw_sigma_omega(si, p["dt"], gam, eg)[0].real for si in sig])
    sigma1 = Z * np.std(x + re_i, ddof=1) * HA_EV
    err = sigma1 / np.sqrt(nsamp)
    t_sample = t_total / nsamp
    gpu_s_per_qp = t_sample * (sigma1 / 0.03) ** 2

    # H psi throughput (local + KB), batch of 256 complex FP32 vectors
    nv, reps = 256, 20
    xh = torch.randn((nv, s.grid.N), dtype=torch.complex64, device="cuda")
    yh = torch.empty_like(xh)
    ctx.apply_H(xh, yh)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        ctx.apply_H(xh, yh)
    torch.cuda.synchronize()
    hpsi_rate = nv * reps * s.grid.N / (time.perf_counter() - t1)
    del xh, yh
    fft_cmp = rocfft_comparison(s)
    ceilings = hbm_ceilings()
    feat = features_roofline(ctx, phis, s)
    progress("H psi, rocFFT and feature-GEMM lines done")

    forms = {"plain": {"gpu_s_per_qp": gpu_s_per_qp, "gpu_s_per_sample": t_sample}}
    if not args.no_bf16:
        forms["c64_graphs"] = graph_form(args, s, phi, p, sigma1, sig, homo, gam,
                                         sgw.SGW_C64)
        progress("graph form done")
        forms["bf16x2kb_graphs"] = graph_form(args, s, phi, p, sigma1, sig, homo, gam,
                                             sgw.SGW_C64_BF16X2KB)
    if not args.no_states:
        phi2 = np.stack([phi, phis[s.n_occ].cpu().numpy()])
        forms["homo_lumo_shared"] = states_form(args, ctx, phi2, p, homo, lumo, gam, t_sample)
        progress("states form done")
    if not args.no_cfg1 and not args.quick:
        forms["cfg1_32_c128_plain"] = cfg1_form(args)
        progress("cfg1 form done")
    if not args.no_cfg3 and not args.quick:
        forms["cfg3_128_bf16"] = cfg3_form(args)
    if args.cv:
        forms["control_variate"] = cv_form(args, ctx, s, phis, ev, phi, p, homo, eg, gam,
                                          t_sample, sigma1, Z)

    achieved = CHEB_ALGO_BYTES * k_pts / (k_ms * 1e-3) / 1e9 if k_ms > 0 else None

    def kb_line(kernel, algo, measured, ms, launches, pts):
        """HBM roofline of a projector kernel on the method's bytes (support
        points) with the tile-granular figures beside it."""
        if not ms > 0:
            return None
        sup = pts * support_frac                      # support pt x vec over the launches
        a = algo * sup / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": kernel, "achieved": a, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": a / HBM_PEAK_GBS,
                "traffic": (measured * pts / launches if measured else None),
                "traffic_unit": "B per launch (counters)",
                "algo_bytes_per_support_ptvec": algo,
                "traffic_bytes_per_support_ptvec": (measured / support_frac if measured
                                                    else None),
                "support_points": kbs["support_points"], "tile_points": kbs["tile_points"],
                "achieved_on_tile_points": algo * pts / (ms * 1e-3) / 1e9,
                "launches": launches, "avg_launch_us": 1e3 * ms / launches,
                "support_ptvec_per_launch": sup / launches}
    line = {
        "metric": METRIC,
        "value": gpu_s_per_qp,
        "unit": "GPU-s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "Si35H36-shaped cluster, 64^3 grid h=0.5, KB s/p "
                               "projectors, N_eta=64, TDH 400 x 0.05 au, N_xi=10000, "
                               "f_g=0.003, gapped filter (1e-7 at the gap edges), "
                               "complex FP32",
                   "samples_per_step": B, "n_tau": p["n_tau"], "n_eta": p["n_eta"],
                   "ncoef": ncoef, "quick": bool(args.quick)},
        "qp": {"eps_ks_homo_eV": homo * HA_EV, "gap_eV": gap * HA_EV,
               "spectral_interval_Ha": [emin, emax],
               "eqp_homo_eV": eg * HA_EV, "eqp_lin_eV": el * HA_EV, "Z": Z,
               "stat_err_eV": err, "sigma1_eV": sigma1, "samples": nsamp,
               "gpu_s_per_sample": t_sample},
        "forms": forms,
        "hpsi_gptvec_per_s": hpsi_rate / 1e9,
        "hpsi_algo_roofline_frac": hpsi_rate * HPSI_ALGO_BYTES / (HBM_PEAK_GBS * 1e9),
        "phase_ms": {"filter": phases[0], "tdh": phases[1], "time_order": phases[2],
                     "zeta_contract": phases[3], "other": phases[4], "total": phases[5]},
        "roofline": kb_line("k_kb_scatter_mma[_w8]<OpF32,NVB,MJ,LX> (autotuned)",
                            KB_SCATTER_ALGO_BYTES, KB_SCATTER_MEASURED_BYTES, s_ms, s_launch,
                            s_pts),
        "roofline_gather": kb_line("k_kb_gather_mma<OpF32,NVB,MT,LX> (autotuned; the "
                                   "TDH's 1024-vector launches: the filter's run untimed "
                                   "on the second stream beside the FFT passes)",
                                   KB_GATHER_ALGO_BYTES, KB_GATHER_MEASURED_BYTES, g_ms,
                                   g_launch, g_pts),
        "fft_vs_rocfft": fft_cmp,
        "hbm_ceilings": ceilings,
        "filter_coefficients": fcoef,
        "kb_layout": kbs,
        "roofline_cheb": {"bound": "hbm", "kernel": "k_plane<float,64,64,PLANE_INV_CHEB>",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": (CHEB_MEASURED_BYTES * k_pts / k_launch
                                 if k_launch and CHEB_MEASURED_BYTES else None),
                     "traffic_unit": "B per launch",
                     "algo_bytes_per_ptvec": CHEB_ALGO_BYTES,
                     "traffic_bytes_per_ptvec": CHEB_MEASURED_BYTES,
                     "launches": k_launch,
                     "avg_launch_us": 1e3 * k_ms / k_launch if k_launch else None},
        "roofline_features": feat,
    }
    if not args.no_cpu_baseline:
        progress("cpu baseline")
        tcpu, parts, cores, sample = cpu_baseline(s, phi, p, args.cpu_terms, ncoef)
        progress("cpu baseline done")
        line["cpu_baseline"] = {"value": tcpu * (sigma1 / 0.03) ** 2, "unit": "CPU-s",
                                "cores": cores, "kind": "oracle", "sample": sample,
                                "seconds_per_sample": tcpu, "parts_s": parts}
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
