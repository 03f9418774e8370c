// Bit-string actions of the ring groups on basis states (host and device).
//
// A basis index x holds the spin at bit position p.  rho^l rotates positions by
// l*stride (p -> p + l*s mod n); phi is the site-centred reflection p -> -p (mod n),
// written as a bit reversal within n bits followed by a rotation by one position.
// Element (l, f) is rho^l phi^f.  All arithmetic is integer, so representatives are
// bit exact.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qoc {

__host__ __device__ inline uint64_t nmask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

__host__ __device__ inline uint64_t rotl_n(uint64_t x, int r, int n) {
  r %= n;
  if (r == 0) return x;
  return ((x << r) | (x >> (n - r))) & nmask(n);
}

__host__ __device__ inline uint64_t reverse_n(uint64_t x, int n) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __brevll(x) >> (64 - n);
#else
  uint64_t y = 0;
  for (int p = 0; p < n; ++p) y |= ((x >> p) & 1ull) << (n - 1 - p);
  return y;
#endif
}

__host__ __device__ inline uint64_t reflect_n(uint64_t x, int n) { return rotl_n(reverse_n(x, n), 1, n); }

// Image of x under rho^l phi^f.
__host__ __device__ inline uint64_t group_act(uint64_t x, int l, int f, int n, int s) {
  uint64_t y = f ? reflect_n(x, n) : x;
  return rotl_n(y, l * s, n);
}

// Minimum over the orbit, with the element (l, f) that maps x onto it.
struct Canon {
  uint64_t rep;
  int l;
  int f;
};

__host__ __device__ inline Canon canonicalize(uint64_t x, int n, int s, int L, bool refl) {
  Canon c{x, 0, 0};
  uint64_t y = x;
  for (int l = 1; l < L; ++l) {
    y = rotl_n(y, s, n);
    if (y < c.rep) { c.rep = y; c.l = l; c.f = 0; }
  }
  if (refl) {
    y = reflect_n(x, n);
    for (int l = 0; l < L; ++l) {
      if (y < c.rep) { c.rep = y; c.l = l; c.f = 1; }
      y = rotl_n(y, s, n);
    }
  }
  return c;
}

__host__ __device__ inline int popc64(uint64_t v) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __popcll(v);
#else
  return __builtin_popcountll(v);
#endif
}

}  // namespace qoc
