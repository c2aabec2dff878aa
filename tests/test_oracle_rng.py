"""Pins for the counter-based random numbers and the sparse xi basis."""
import numpy as np

from oracle import rng
from oracle.sroi import XiBasis, n_segments, supports


def test_splitmix64_published_sequence():
    # Reference outputs of SplitMix64 seeded with 1234567 (the sequence
    # printed by the authors' reference implementation, splitmix64.c).
    assert rng.splitmix64_sequence(1234567, 5) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_vectorised_mix_matches_scalar():
    xs = [0, 1, 2 ** 63, 2 ** 64 - 1, 123456789123456789]
    v = rng.sm64(np.array(xs, dtype=np.uint64))
    assert [int(a) for a in v] == [rng.sm64(x) for x in xs]


def test_white_noise_values_and_norm():
    dV = 0.125
    z = rng.white_noise(7, rng.ZETA, 3, 0, 4096, dV)
    assert np.allclose(np.abs(z), 1 / np.sqrt(dV))
    # <z|z> = dV sum z^2 = N exactly for +-1/sqrt(dV) noise
    assert abs(dV * np.sum(z * z) - 4096) < 1e-9


def test_white_noise_unbiased_and_decorrelated():
    n = 1 << 18
    a = rng.white_noise_signs(11, rng.stream_id(rng.ETA, 0, 0), n)
    b = rng.white_noise_signs(11, rng.stream_id(rng.ETA, 0, 1), n)
    c = rng.white_noise_signs(12, rng.stream_id(rng.ETA, 0, 0), n)
    tol = 5.0 / np.sqrt(n)
    assert abs(np.mean(a)) < tol
    assert abs(np.mean(a * b)) < tol
    assert abs(np.mean(a * c)) < tol
    # neighbouring points use neighbouring bits of one word: no correlation
    assert abs(np.mean(a[1:] * a[:-1])) < tol


def test_xi_supports_distinct_and_in_range():
    N, n_xi, fg = 32768, 2000, 0.003
    bl = supports(5, 2, N, n_xi, fg)
    assert bl.shape == (n_xi, n_segments(N, fg))
    assert bl.min() >= 0 and bl.max() < N // 32
    for row in bl:
        assert len(set(row.tolist())) == row.size


def test_xi_supports_force_collisions():
    # many segments out of few blocks: linear probing must give distinct,
    # complete rows
    bl = supports(9, 0, 32 * 8, 50, 0.7)   # n_seg = 6 of 8 blocks
    assert bl.shape[1] == 6
    for row in bl:
        assert len(set(row.tolist())) == 6


def test_xi_marginal_coverage_uniform():
    N, n_xi, fg = 32 * 64, 4000, 0.1     # n_seg = 6 of 64 blocks
    bl = supports(3, 1, N, n_xi, fg)
    counts = np.bincount(bl.ravel(), minlength=N // 32)
    expect = bl.size / (N // 32)
    # multinomial-like counts: all within 5 sigma of the mean
    assert np.all(np.abs(counts - expect) < 5 * np.sqrt(expect))


def test_xi_resolution_of_identity():
    """E_xi[ sum_m <xi_m|a><xi_m|b> ] = <a|b>  (sROI completeness)."""
    N, dV, n_xi, fg = 512, 0.343, 40, 0.125
    rs = np.random.default_rng(0)
    a = rs.standard_normal(N)
    b = a + 0.5 * rs.standard_normal(N)
    exact = dV * np.sum(a * b)
    vals = []
    for s in range(600):
        X = XiBasis(100 + s, s % 7, N, n_xi, fg, dV)
        vals.append(np.sum(X.overlaps(a) * X.overlaps(b)))
    vals = np.array(vals)
    err = np.std(vals) / np.sqrt(len(vals))
    assert abs(np.mean(vals) - exact) < 4 * err
    # and the dense form gives the same numbers as the gather form
    X = XiBasis(1, 0, N, n_xi, fg, dV)
    assert np.allclose(dV * X.dense() @ a, X.overlaps(a), rtol=1e-13, atol=1e-13)
