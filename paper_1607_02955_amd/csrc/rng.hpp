// Counter-based random draws of the estimators (library side).
//
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) as a keyed hash
// H(seed, tag, a, b) = s(s(s(seed ^ tag) ^ a) ^ b), s(x) = SplitMix64 output
// for state x; bounded integers by Lemire's multiply-shift with rejection
// (ACM TOMACS 2019); k-subsets by Floyd's algorithm (CACM 1987).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define CFC_HD __host__ __device__ __forceinline__
#else
#define CFC_HD inline
#endif

namespace cfc {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kTagJL = 0x4A4Cull;
constexpr uint64_t kTagSample = 0x5350ull;
constexpr uint64_t kTagShared = 0x5348ull;
constexpr uint64_t kTagPairs = 0x4346ull;

CFC_HD uint64_t sm_step(uint64_t x) {
  uint64_t z = x + kGolden;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

CFC_HD uint64_t key_hash(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b) {
  return sm_step(sm_step(sm_step(seed ^ tag) ^ a) ^ b);
}

// Sign word for projection rows 64*word .. 64*word+63 on edge {lo < hi}.
CFC_HD uint64_t jl_word(uint64_t seed, uint64_t word, uint64_t lo, uint64_t hi) {
  return key_hash(seed, kTagJL, word, (lo << 32) | hi);
}

}  // namespace cfc
