// sbm_fastdiv.h -- division by a run-time constant through one multiply, used
// to decode linear node and cell indices without integer division.
//
// For n < 2^31 and a divisor d >= 1: with s = ceil(log2 d), L = 32 + s and
// M = floor(2^L / d) + 1, floor(n / d) = floor(n M / 2^L).  Writing
// M = 2^L/d + e with 0 < e <= 1, n M / 2^L = n/d + n e / 2^L and the error
// term is below 2^(31-32-s) <= 1/(2d), which never lifts n/d past the next
// integer (its fractional part is at most (d-1)/d); M <= 2^33 + 1 keeps the
// product n M below 2^64.
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#ifndef __forceinline__
#define __forceinline__ inline
#endif
#endif

namespace sbm {

struct FastDiv {
  uint32_t d;
  uint32_t L;
  uint64_t M;
  __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return (uint32_t)(((uint64_t)n * M) >> L);
  }
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  FastDiv f;
  f.d = d;
  f.L = 32 + s;
  f.M = (uint64_t)((((unsigned __int128)1) << f.L) / d) + 1;
  return f;
}

}  // namespace sbm
