"""Plain FP64 CPU oracle for the stochastic-GW (sGW / sROI) hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
definition that the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path (no kernels, headers, tables
or helpers) and never imports the product package.

Every function cites the passage of the paper it follows (arXiv 2601.21005,
"StochasticGW-GPU").  Where the paper is silent the module states the reading
it takes.  Arithmetic is numpy/scipy float64 / complex128 throughout.

Modules
-------
rng          counter-based SplitMix64 white noise and sparse xi supports
grid         periodic real-space grid, FFT conventions, inner products
hamiltonian  kinetic, local and Kleinman-Bylander parts of H, H|psi>, bounds
chebyshev    Fermi-filter coefficients and recurrence, Chebyshev propagator
tdh          Hartree potential and the linear-response TDH Strang step
sroi         sparse stochastic xi basis and its overlaps
timeorder    retarded -> time-ordered conversion by conjugating omega<0
sigma        per-sample Sigma_c(t), exchange X, the full estimator
qp           damped Fourier transform Sigma(omega) and the QP equation
eigen        reference eigensolvers (dense and iterative) for the inputs

Parity status: every function is pinned by a ``-m "not gpu"`` test under
``tests/`` (see the ``test_oracle_*`` files); none is "parity unpinned".
"""
