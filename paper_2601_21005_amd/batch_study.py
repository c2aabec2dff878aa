"""Uneven batch of clusters: sequential calls against the batched entry point.

32 seeded H-capped Si clusters (5 to 147 Si atoms, grids 48^3 to 96^3 at
h = 0.6 bohr, 16 to 128 stochastic orbitals each, from systems.uneven_batch)
each get a context on a stream of their own and a short Sigma_c(t) estimate
(2 samples, 20 output steps, gapped filter).  The script times the clusters
one after another on one stream without graphs, then all of them through
sgw_batch_sigma_estimate (host workers, one stream per cluster, graph replay
on), checks that every result is bitwise the sequential one, and prints one
JSON line.

  python -m paper_2601_21005_amd.batch_study [--count 32] [--workers 4]
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=32)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--n-tau", type=int, default=20)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    from paper_2601_21005_amd import sgw, systems
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    batch = systems.uneven_batch(args.count)
    print(f"{len(batch)} clusters built ({time.perf_counter() - t0:.1f} s)", flush=True)
    jobs, meta = [], []
    for i, (s, neta) in enumerate(batch):
        st = torch.cuda.Stream()
        ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=sgw.SGW_C64,
                          ecut=s.ecut, max_nvec=256, stream=st.cuda_stream)
        lo, hi = ctx.lanczos_bounds(30, seed=1, pad=0.01)
        mid = lo + 0.12 * (hi - lo)
        a = sgw.sgw_gapped_coefficients(mid - 0.15, mid + 0.15, 1e-7, lo, hi, 16384)
        tail = np.cumsum(np.abs(a[::-1]))[::-1]
        ncoef = int(np.nonzero(tail < 1e-6)[0][0])
        rs = np.random.default_rng(i)
        phi = rs.standard_normal(s.grid.N)
        phi /= np.sqrt(s.grid.h ** 3 * np.sum(phi * phi))
        kw = dict(seed=1004 + i, n_zeta=2, n_eta=neta, n_tau=args.n_tau, dt=0.05, m_sub=1,
                  ncoef=ncoef, emin=lo, emax=hi, n_xi=2000, f_g=0.003, mode=0, filter=1,
                  e_homo=mid - 0.15, e_lumo=mid + 0.15, filter_eps=1e-7)
        jobs.append((ctx, phi, kw))
        meta.append({"name": s.name, "grid": s.grid.n, "n_eta": neta, "ncoef": ncoef})
    torch.cuda.synchronize()
    print(f"contexts and intervals ready ({time.perf_counter() - t0:.1f} s)", flush=True)
    # warm-up: autotuning and allocation of every context, eagerly
    for ctx, phi, kw in jobs:
        ctx.sigma_estimate(phi, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    seq = []
    for ctx, phi, kw in jobs:
        seq.append(ctx.sigma_estimate(phi, **kw))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    print(f"sequential: {t_seq:.2f} s", flush=True)
    for ctx, phi, kw in jobs:                                   # capture the graphs
        ctx.use_graphs(True)
        ctx.sigma_estimate(phi, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bat = sgw.batch_sigma_estimate(jobs, nworkers=args.workers)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t2
    print(f"batched ({args.workers} workers, graphs): {t_bat:.2f} s", flush=True)
    same = all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
               for a, b in zip(seq, bat))
    for m, b in zip(meta, bat):
        m["batched_ms"] = b[2]
    for ctx, _, _ in jobs:
        ctx.close()
    print(json.dumps({"clusters": len(jobs), "workers": args.workers, "n_tau": args.n_tau,
                      "sequential_s": t_seq, "batched_s": t_bat, "speedup": t_seq / t_bat,
                      "bitwise_equal": bool(same), "per_cluster": meta}), flush=True)


if __name__ == "__main__":
    main()
