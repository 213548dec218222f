// Host-side draws of the method's randomness: hash/sign tables and start
// vectors, from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).  Integer
// work only for the tables, FP64 Box-Muller for the start vectors.
#include <math.h>
#include <stdint.h>

#include "../../include/tsk.h"
#include "status.hpp"

namespace {

inline uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" tsk_status tsk_hash_generate(uint64_t seed, int n, int b, int B, uint32_t* h_host,
                                        int8_t* xi_host) {
  if (!h_host || !xi_host) return tsk::fail(TSK_EINVAL, "tsk_hash_generate: null output pointer");
  if (n < 1 || b < 1 || B < 1)
    return tsk::fail(TSK_EINVAL, "tsk_hash_generate: n=%d b=%d B=%d must be >= 1", n, b, B);
  if (B > (1 << 29)) return tsk::fail(TSK_EINVAL, "tsk_hash_generate: B too large");
  const uint64_t base = mix64(seed ^ 0x68617368ull);
  for (int m = 0; m < B; ++m)
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < n; ++i) {
        const uint64_t key = ((uint64_t)m << 34) | ((uint64_t)j << 32) | (uint64_t)(uint32_t)i;
        const uint64_t r = mix64(base + key);
        const size_t e = ((size_t)m * 3 + j) * n + i;
        h_host[e] = (uint32_t)(((r >> 32) * (uint64_t)(uint32_t)b) >> 32);
        xi_host[e] = ((r >> 31) & 1u) ? (int8_t)-1 : (int8_t)1;
      }
  return TSK_OK;
}

extern "C" tsk_status tsk_init_vectors(uint64_t seed, int comp, int L, int n, double* u0_host) {
  if (!u0_host) return tsk::fail(TSK_EINVAL, "tsk_init_vectors: null output pointer");
  if (L < 1 || n < 1 || comp < 0 || L >= (1 << 20) || n >= (1 << 19) || comp >= (1 << 23))
    return tsk::fail(TSK_EINVAL, "tsk_init_vectors: comp=%d L=%d n=%d out of range", comp, L, n);
  const uint64_t base = mix64(seed ^ 0x75307530ull);
  const double two53 = 1.0 / 9007199254740992.0;
  const double two_pi = 6.283185307179586476925286766559;
  for (int tau = 0; tau < L; ++tau) {
    double* u = u0_host + (size_t)tau * n;
    double ss = 0.0;
    for (int i = 0; i < n; ++i) {
      const uint64_t key = ((uint64_t)comp << 40) | ((uint64_t)tau << 20) | (uint64_t)(2 * i);
      const uint64_t r0 = mix64(base + key);
      const uint64_t r1 = mix64(base + key + 1);
      const double U0 = (double)(r0 >> 11) * two53;
      const double U1 = (double)(r1 >> 11) * two53;
      const double z = sqrt(-2.0 * log(1.0 - U0)) * cos(two_pi * U1);
      u[i] = z;
      ss += z * z;
    }
    const double nrm = sqrt(ss);
    for (int i = 0; i < n; ++i) u[i] /= nrm;
  }
  return TSK_OK;
}
