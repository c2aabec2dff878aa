"""Counter-based random numbers for the stochastic orbitals (oracle side).

The paper draws its white-noise orbitals and sparse xi functions with KISS on
the CPU and cuRAND on the GPU (Sec. 2.3, and the discussion of Table 4).  The
method only needs independent random signs; to make the CPU oracle and the GPU
library draw *identical* numbers, both sides implement the same counter-based
generator from its published definition, independently:

* SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom
  number generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the
  output mix  z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
  z *= 0x94D049BB133111EB; z ^= z>>31.

Reading (the paper is silent on the generator's structure):
  key(seed, stream)      = sm64(seed XOR sm64(stream))
  word(seed, stream, i)  = sm64(key + i)               (mod 2**64)
  sign of grid point r   = bit (r mod 64) of word(seed, stream, r div 64):
                           0 -> +1, 1 -> -1
  white noise value      = sign / sqrt(dV)   so that E[z z^T] = I / dV
  stream(kind, s, l)     = kind * 2**40 + s * 2**20 + l

where ``sm64(x)`` is the first output of SplitMix64 started in state x.
"""
import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB

# stream kinds
ZETA = 1        # white noise zeta-bar_i (one per Monte Carlo sample)
ETA = 2         # white noise eta-bar_{i,l}
XI_SUPPORT = 3  # segment positions of the sparse xi_{i,m}
XI_SIGN = 4     # point signs of the sparse xi_{i,m}
BOUNDS = 5      # start vector of the Lanczos estimate of the spectral interval


def sm64(x):
    """First SplitMix64 output from state ``x`` (python int or uint64 array)."""
    if isinstance(x, np.ndarray):
        with np.errstate(over="ignore"):
            z = x.astype(np.uint64) + np.uint64(GAMMA)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
            return z ^ (z >> np.uint64(31))
    z = (int(x) + GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def splitmix64_sequence(seed, count):
    """The plain SplitMix64 stream of ``count`` outputs from ``seed``."""
    out = []
    state = int(seed) & MASK64
    for _ in range(count):
        state = (state + GAMMA) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * MIX1) & MASK64
        z = ((z ^ (z >> 27)) * MIX2) & MASK64
        out.append(z ^ (z >> 31))
    return out


def stream_id(kind, sample, l=0):
    assert 0 <= sample < (1 << 20) and 0 <= l < (1 << 20)
    return (kind << 40) | (sample << 20) | l


def stream_key(seed, stream):
    return sm64((int(seed) & MASK64) ^ sm64(stream))


def words(seed, stream, idx):
    """word(seed, stream, i) for an integer array of counters ``idx``."""
    key = stream_key(seed, stream)
    with np.errstate(over="ignore"):
        x = np.asarray(idx, dtype=np.uint64) + np.uint64(key)
    return sm64(x)


def white_noise_signs(seed, stream, n):
    """+1/-1 (float64) for grid points 0..n-1."""
    r = np.arange(n, dtype=np.uint64)
    w = words(seed, stream, r >> np.uint64(6))
    bit = (w >> (r & np.uint64(63))) & np.uint64(1)
    return 1.0 - 2.0 * bit.astype(np.float64)


def white_noise(seed, kind, sample, l, n, dV):
    """Stochastic orbital of +-1/sqrt(dV) values (Sec. 2.1)."""
    return white_noise_signs(seed, stream_id(kind, sample, l), n) / np.sqrt(dV)
