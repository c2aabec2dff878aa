// Counter-based random numbers (library side).
//
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state += 0x9E3779B97F4A7C15,
// output z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
// z *= 0x94D049BB133111EB; z ^= z >> 31.  sm64(x) is the first output from
// state x.  Streams: key(seed, stream) = sm64(seed ^ sm64(stream)),
// word(key, i) = sm64(key + i), stream = kind << 40 | sample << 20 | l.
// White-noise sign of point r: bit (r mod 64) of word(key, r / 64), 0 -> +1.
#pragma once

#include <cstdint>

namespace sgw {

enum RngKind : uint64_t {
  RNG_ZETA = 1, RNG_ETA = 2, RNG_XI_SUPPORT = 3, RNG_XI_SIGN = 4,
  RNG_BOUNDS = 5   // start vector of the Lanczos interval
};

__host__ __device__ __forceinline__ uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ uint64_t rng_stream(uint64_t kind, uint64_t sample,
                                                        uint64_t l) {
  return (kind << 40) | (sample << 20) | l;
}

__host__ __device__ __forceinline__ uint64_t rng_key(uint64_t seed, uint64_t stream) {
  return sm64(seed ^ sm64(stream));
}

// +1 / -1 white-noise sign of grid point r
__device__ __forceinline__ int noise_bit(uint64_t key, int64_t r) {
  const uint64_t w = sm64(key + (uint64_t)(r >> 6));
  return (int)((w >> (r & 63)) & 1ull);
}

}  // namespace sgw
