// Fixed-width byte-string keys (the paper's measured workload, Section 3:
// random strings of 32 bytes in memcmp order), sorted through the index:
// the strings stay where they are and the sort moves their 64-bit prefix
// words with the index as payload, most significant word first.
//
//   round 0   word 0 (bytes 0..7, read big-endian so that unsigned order is
//             memcmp order) of every string, sorted stably with the index
//             as payload (the pairs sort: sample, splitters, classify on
//             the word, stable split, stable bucket sort);
//   round k   the runs of strings whose words 0..k-1 are all equal (groups
//             of two or more) are gathered with their word k and sorted as
//             segments (one segment per group, stable), then scattered back
//             into place.  A round without such runs ends the sort.
//
// Strings equal in every word keep their input order (every sort is
// stable), so the result is the stable memcmp order.
#pragma once
#include "ss_kernels.h"

namespace ss {

__device__ __forceinline__ uint64_t str_word(const uint8_t* recs, uint32_t width, uint64_t i, uint32_t k) {
  const uint64_t v = *(const uint64_t*)(recs + i * width + 8ull * k);
  return __builtin_bswap64(v);
}

// w[i] = word k of string perm[i] (perm == nullptr: string i)
__global__ void __launch_bounds__(256) k_str_word(const uint8_t* recs, uint32_t width, uint32_t k,
                                                  const uint32_t* perm, uint64_t* w, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    w[i] = str_word(recs, width, perm ? perm[i] : i, k);
}

// Group boundaries after sorting by words 0..k-1 (w: word k-1 of the
// sorted strings; bprev: the boundaries of the rounds before, or null):
// b[i] = 1 where a new run of equal prefixes starts.  f[i] = 1 for strings
// in runs of two or more, g[i] = 1 at the first string of such a run; both
// arrays have n + 1 entries (the last 0) so that their exclusive scans end
// with the totals.
__global__ void __launch_bounds__(256) k_str_flags(const uint64_t* w, const uint8_t* bprev, uint8_t* b,
                                                   uint32_t* f, uint32_t* g, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i <= n; i += (uint64_t)gridDim.x * 256) {
    if (i == n) {
      f[n] = 0;
      g[n] = 0;
      continue;
    }
    const bool st = i == 0 || w[i] != w[i - 1] || (bprev && bprev[i]);
    const bool nx = i + 1 == n || w[i + 1] != w[i] || (bprev && bprev[i + 1]);
    const bool tie = !(st && nx);
    b[i] = st ? 1 : 0;
    f[i] = tie ? 1u : 0u;
    g[i] = (tie && st) ? 1u : 0u;
  }
}

// Gather the strings of the runs: word k, index, position; run g starts at
// off[g] (f, g scanned; tot[0] = strings in runs, tot[1] = runs).
__global__ void __launch_bounds__(256) k_str_gather(const uint8_t* recs, uint32_t width, uint32_t k,
                                                    const uint8_t* b, const uint32_t* f, const uint32_t* g,
                                                    const uint32_t* perm, uint64_t* key_t, uint32_t* val_t,
                                                    uint32_t* pos_t, int64_t* off, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i <= n; i += (uint64_t)gridDim.x * 256) {
    if (i == n) {
      off[g[n]] = (int64_t)f[n];
      continue;
    }
    const bool tie = f[i + 1] != f[i];
    if (!tie) continue;
    const uint32_t c = f[i];
    const uint32_t s = perm[i];
    key_t[c] = str_word(recs, width, s, k);
    val_t[c] = s;
    pos_t[c] = (uint32_t)i;
    if (b[i]) off[g[i]] = (int64_t)c;
  }
}

// Put the sorted runs back: index and word k at their positions.
__global__ void __launch_bounds__(256) k_str_scatter(const uint64_t* key_s, const uint32_t* val_s,
                                                     const uint32_t* pos_t, uint32_t* perm, uint64_t* w,
                                                     const uint32_t* f, uint64_t n) {
  const uint64_t tot = f[n];
  for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < tot; c += (uint64_t)gridDim.x * 256) {
    const uint32_t i = pos_t[c];
    perm[i] = val_s[c];
    w[i] = key_s[c];
  }
}

// Sorted strings: out[i] = recs[perm[i]], 8 bytes per thread step.
__global__ void __launch_bounds__(256) k_str_permute(const uint8_t* recs, uint8_t* out, const uint32_t* perm,
                                                     uint32_t width, uint64_t n) {
  const uint32_t wpr = width / 8;
  const uint64_t tot = n * wpr;
  for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < tot; q += (uint64_t)gridDim.x * 256) {
    const uint64_t i = q / wpr, k = q - i * wpr;
    ((uint64_t*)out)[q] = *(const uint64_t*)(recs + (uint64_t)perm[i] * width + 8 * k);
  }
}

}  // namespace ss
