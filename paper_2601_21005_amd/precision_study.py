"""Precision of the QP energies on the large-cluster shape, against an FP64 run.

On the Si357H204 stand-in (128^3, h = 0.6 bohr, 1632 KB projectors, 816
occupied states) this runs the same Monte Carlo samples (identical seeds)
with complex FP64 (the reference), complex FP32, and complex FP32 with BF16
projector GEMMs, for the HOMO and the LUMO, and prints one JSON line with the
QP energies and their differences from the FP64 run.  Every step runs on the
device through the library; the KS input states come from ksinput.

  python -m paper_2601_21005_amd.precision_study [--n-zeta 32] [--n-eta 8] [--n-tau 100]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HA_EV = 27.211386245988


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-zeta", type=int, default=32)
    ap.add_argument("--n-eta", type=int, default=8)
    ap.add_argument("--n-tau", type=int, default=100)
    ap.add_argument("--dt", type=float, default=0.05)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--window", type=float, default=0.3,
                    help="minimum width (Ha) of the filter's transition window")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    from paper_2601_21005_amd import ksinput, sgw, systems
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    s = systems.si357h204(n=args.n)
    dV = s.grid.h ** 3
    print(f"system {s.name}: N {s.grid.N}, projectors {len(s.projectors.l)}, "
          f"n_occ {s.n_occ} ({time.perf_counter() - t0:.1f} s)", flush=True)

    def ctx_of(prec):
        return sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=prec,
                           ecut=s.ecut, max_nvec=512)

    c64 = ctx_of(sgw.SGW_C64)
    emin, emax = c64.lanczos_bounds(60, seed=1, pad=0.01)
    t1 = time.perf_counter()
    ev, phis, res = ksinput.lowest_states(c64, s.n_occ + 1, emin, emax, dV, tol=1e-4,
                                           maxit=80)
    homo, lumo = float(ev[s.n_occ - 1]), float(ev[s.n_occ])
    print(f"interval [{emin:.4f}, {emax:.4f}] Ha; HOMO {homo:.6f} LUMO {lumo:.6f} Ha "
          f"(states {time.perf_counter() - t1:.1f} s, max residual {res.max():.1e})", flush=True)
    states = {"HOMO": (phis[s.n_occ - 1].cpu().numpy(), homo),
              "LUMO": (phis[s.n_occ].cpu().numpy(), lumo)}
    # The model's gap at this size is far smaller than the real cluster's, so
    # the filter's transition is spread over a window of at least
    # args.window Ha centred mid-gap -- the same filter in every precision.
    mid, half = 0.5 * (homo + lumo), max(0.5 * (lumo - homo), 0.5 * args.window)
    eh, el = mid - half, mid + half
    a = sgw.sgw_gapped_coefficients(eh, el, 1e-7, emin, emax, 16384)
    tail = np.cumsum(np.abs(a[::-1]))[::-1]
    ncoef = int(np.nonzero(tail < 1e-7)[0][0])
    p = dict(seed=1003, n_eta=args.n_eta, n_tau=args.n_tau, dt=args.dt, m_sub=1, ncoef=ncoef,
             emin=emin, emax=emax, n_xi=10000, f_g=0.003, mode=0, filter=1, e_homo=eh,
             e_lumo=el, filter_eps=1e-7)
    gam = 3.0 / (args.n_tau * args.dt)
    out = {"system": s.name, "grid": list(s.grid.n) if hasattr(s.grid.n, "__len__") else s.grid.n,
           "h": s.grid.h, "projectors": int(len(s.projectors.l)), "n_occ": s.n_occ,
           "samples": args.n_zeta, "n_eta": args.n_eta, "n_tau": args.n_tau, "ncoef": ncoef,
           "interval_Ha": [emin, emax], "homo_lumo_Ha": [homo, lumo],
           "filter_window_Ha": [eh, el], "results": {}}
    c64.close()
    for prec, name in ((sgw.SGW_C128, "c128"), (sgw.SGW_C64, "c64"),
                       (sgw.SGW_C64_BF16KB, "c64_bf16kb"), (sgw.SGW_C64_BF16X2KB, "c64_bf16x2kb")):
        ctx = ctx_of(prec)
        for st, (phi, eks) in states.items():
            t2 = time.perf_counter()
            sig, x, _ = ctx.sigma_estimate(phi, n_zeta=args.n_zeta, first_sample=0, **p)
            torch.cuda.synchronize()
            eg, el, Z = sgw.sgw_qp_solve(sig.mean(0), args.dt, gam, eks, x.mean())
            out["results"].setdefault(st, {})[name] = {
                "eqp_eV": eg * HA_EV, "eqp_lin_eV": el * HA_EV, "Z": Z,
                "sigma_t": [sig.mean(0).real.tolist()[::10], sig.mean(0).imag.tolist()[::10]],
                "x": float(x.mean()), "seconds": time.perf_counter() - t2}
            print(f"{name} {st}: eqp {eg * HA_EV:.6f} eV ({time.perf_counter() - t2:.1f} s)",
                  flush=True)
        ctx.close()
    summary = {}
    for st, r in out["results"].items():
        ref = r["c128"]
        s_ref = np.array(ref["sigma_t"][0]) + 1j * np.array(ref["sigma_t"][1])
        for name in ("c64", "c64_bf16kb", "c64_bf16x2kb"):
            s_x = np.array(r[name]["sigma_t"][0]) + 1j * np.array(r[name]["sigma_t"][1])
            summary[f"{st}_{name}"] = {
                "d_eqp_meV": 1e3 * abs(r[name]["eqp_eV"] - ref["eqp_eV"]),
                "d_x_rel": abs(r[name]["x"] - ref["x"]) / abs(ref["x"]),
                "sigma_t_max_rel": float(np.max(np.abs(s_x - s_ref)) / np.max(np.abs(s_ref)))}
    for r in out["results"].values():
        for v in r.values():
            v.pop("sigma_t")
    out["errors_vs_c128"] = summary
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
