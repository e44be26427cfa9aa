// Device building blocks of the sample sort (gfx950, wave64).
//
//  - order-preserving key maps (the sort compares unsigned images "ord")
//  - wave and work-group scans / reductions
//  - a work-group stable LSD radix sort held in registers + LDS that sorts
//    only the bit range that varies inside the group of keys
//  - a merge-path split for stable two-way merges
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace ss {

constexpr int WAVE = 64;

// ------------------------------------------------------------------ keys

// kind: 0 unsigned, 1 signed (two's complement), 2 IEEE float (totalOrder)
__device__ __forceinline__ uint32_t to_ord(uint32_t x, int kind) {
  uint32_t m = kind ? 0x80000000u : 0u;
  if (kind == 2 && (x >> 31)) m = 0xFFFFFFFFu;
  return x ^ m;
}
__device__ __forceinline__ uint64_t to_ord(uint64_t x, int kind) {
  uint64_t m = kind ? 0x8000000000000000ull : 0ull;
  if (kind == 2 && (x >> 63)) m = ~0ull;
  return x ^ m;
}
__device__ __forceinline__ uint32_t from_ord(uint32_t o, int kind) {
  uint32_t m = kind ? 0x80000000u : 0u;
  if (kind == 2 && !(o >> 31)) m = 0xFFFFFFFFu;
  return o ^ m;
}
__device__ __forceinline__ uint64_t from_ord(uint64_t o, int kind) {
  uint64_t m = kind ? 0x8000000000000000ull : 0ull;
  if (kind == 2 && !(o >> 63)) m = ~0ull;
  return o ^ m;
}

template <typename T>
__device__ __forceinline__ int bit_width(T x) {  // number of bits needed for x
  if (x == 0) return 0;
  if constexpr (sizeof(T) == 8) return 64 - __clzll((long long)x);
  else return 32 - __clz((int)x);
}

// ------------------------------------------------------------ SplitMix64
// Steele, Lea & Flood (OOPSLA 2014), finaliser with shifts 30/27/31.
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t SM64_GAMMA = 0x9E3779B97F4A7C15ull;
// (j+1)-th output of the generator with state `seed`
__device__ __forceinline__ uint64_t sm64_at(uint64_t seed, uint64_t j) {
  return sm64_mix(seed + (j + 1) * SM64_GAMMA);
}
// floor(r * n / 2^64)
__device__ __forceinline__ uint64_t scale_to(uint64_t r, uint64_t n) { return __umul64hi(r, n); }

// ------------------------------------------------------------- scans

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / WAVE; }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T y = __shfl_up(x, d, WAVE);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan over the work-group (NT threads); `sh` needs NT/64 + 1
// elements.  Returns the thread's exclusive prefix; *total gets the sum.
template <int NT, typename T = uint32_t>
__device__ __forceinline__ T block_excl_scan(T v, T* sh, T* total) {
  constexpr int NW = NT / WAVE;
  const int lane = lane_id(), w = wave_id();
  T inc = wave_incl_scan(v);
  if (lane == WAVE - 1) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x < WAVE) {
    T t = (lane < NW) ? sh[lane] : T(0);
    T ti = wave_incl_scan(t);
    if (lane < NW) sh[lane] = ti - t;
    if (lane == NW - 1) sh[NW] = ti;
  }
  __syncthreads();
  T r = sh[w] + inc - v;
  *total = sh[NW];
  __syncthreads();
  return r;
}

template <typename T>
__device__ __forceinline__ T wave_min(T x) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) { T y = __shfl_xor(x, d, WAVE); x = y < x ? y : x; }
  return x;
}
template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) { T y = __shfl_xor(x, d, WAVE); x = y > x ? y : x; }
  return x;
}

// min and max over the work-group; `sh` needs 2*NT/64 elements of T
template <int NT, typename T>
__device__ __forceinline__ void block_minmax(T& mn, T& mx, T* sh) {
  constexpr int NW = NT / WAVE;
  mn = wave_min(mn);
  mx = wave_max(mx);
  if (lane_id() == 0) { sh[wave_id()] = mn; sh[NW + wave_id()] = mx; }
  __syncthreads();
  mn = sh[0];
  mx = sh[NW];
#pragma unroll
  for (int i = 1; i < NW; i++) {
    T a = sh[i], b = sh[NW + i];
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  __syncthreads();
}

// ------------------------------------------------- work-group radix sort

struct NoVal {};

// LDS slot of item i in an exchange buffer: one padding slot after every K
// items so a thread reading its K consecutive items hits distinct banks.
template <int K>
__device__ __forceinline__ int pad_idx(int i) { return i + i / K; }

template <int NT, int K>
struct SortShape {
  static constexpr int C = NT * K;           // items per work-group
  static constexpr int SLOTS = C + C / K;    // exchange slots incl. padding
};

// Digits of R bits; counters are 16-bit, two digits packed per 32-bit word.
constexpr int RADIX_BITS = 4;
constexpr int RADIX_HALF = 1 << (RADIX_BITS - 1);  // digits per packed half

template <int NT>
struct RadixLds {
  static constexpr int CNT_WORDS = RADIX_HALF * NT;
};

// Stable LSD radix sort of NT*K items held blocked in registers (item
// i = t*K + k of thread t), ordered by (hi, lo) [lo only if LO], over the
// bit ranges that actually vary among the first `nvalid` items.  Items with
// i >= nvalid must carry all-ones keys: they sort after every real item.
// A payload (VT != NoVal) travels with its key.
//
// On return the sorted items are in LDS: xh[pad_idx<K>(j)] (and xl, xv),
// j = 0..NT*K-1, and the function ends with a barrier.
//
// LDS: cnt = RadixLds<NT>::CNT_WORDS words; xh/xl/xv = SortShape::SLOTS
// elements each; red >= 2*NT/64 HT elements + NT/64+1 words (aligned 8).
//
// hi_skip: low bits of hi that are not part of the key (they may vary but
// are already in the required order among equal keys, e.g. a packed index).
template <int NT, int K, typename HT, bool LO, typename VT>
__device__ __forceinline__ void block_radix_sort(HT (&hi)[K], uint32_t (&lo)[K], VT (&val)[K], int nvalid,
                                 uint32_t* cnt, HT* xh, uint32_t* xl, VT* xv, void* red,
                                 int hi_skip = 0) {
  constexpr bool HASV = !std::is_same<VT, NoVal>::value;
  constexpr int H = RADIX_HALF;
  static_assert(K <= 255, "per-thread counts are kept as bytes");
  const int t = threadIdx.x;

  // bit ranges that vary among the real items
  HT mnh = ~HT(0), mxh = 0;
  uint32_t mnl = ~0u, mxl = 0;
#pragma unroll
  for (int k = 0; k < K; k++) {
    if (t * K + k < nvalid) {
      mnh = hi[k] < mnh ? hi[k] : mnh;
      mxh = hi[k] > mxh ? hi[k] : mxh;
      if constexpr (LO) {
        mnl = lo[k] < mnl ? lo[k] : mnl;
        mxl = lo[k] > mxl ? lo[k] : mxl;
      }
    }
  }
  block_minmax<NT>(mnh, mxh, (HT*)red);
  int nb_hi = bit_width<HT>((HT)((mnh ^ mxh) >> hi_skip));
  int nb_lo = 0;
  if constexpr (LO) {
    block_minmax<NT>(mnl, mxl, (uint32_t*)red);
    nb_lo = bit_width<uint32_t>(mnl ^ mxl);
  }
  const int np_lo = (nb_lo + RADIX_BITS - 1) / RADIX_BITS;
  const int np_hi = (nb_hi + RADIX_BITS - 1) / RADIX_BITS;
  const int npass = np_lo + np_hi;
  uint32_t* scan_sh = (uint32_t*)((HT*)red + 2 * (NT / WAVE) + 2);

  if (npass == 0) {  // all real keys equal: the input order is the sorted order
#pragma unroll
    for (int k = 0; k < K; k++) {
      int j = pad_idx<K>(t * K + k);
      xh[j] = hi[k];
      if constexpr (LO) xl[j] = lo[k];
      if constexpr (HASV) xv[j] = val[k];
    }
    __syncthreads();
    return;
  }

  for (int pass = 0; pass < npass; pass++) {
    const bool on_lo = pass < np_lo;
    const int rel = (on_lo ? pass : pass - np_lo) * RADIX_BITS;
    const int nbits = min(RADIX_BITS, (on_lo ? nb_lo : nb_hi) - rel);
    const int shift = on_lo ? rel : rel + hi_skip;
    const uint32_t mask = (1u << nbits) - 1u;

    // 1. zero this thread's counter column
#pragma unroll
    for (int j = 0; j < H; j++) cnt[j * NT + t] = 0;

    // 2. count: digits of this thread's items, in item order.  The number
    // of earlier items of this thread with the same digit (< K <= 255) is
    // kept as a byte, four to a register.
    uint32_t locp[(K + 3) / 4];
#pragma unroll
    for (int q = 0; q < (K + 3) / 4; q++) locp[q] = 0;
#pragma unroll
    for (int k = 0; k < K; k++) {
      uint32_t d = on_lo ? ((lo[k] >> shift) & mask) : ((uint32_t)(hi[k] >> shift) & mask);
      int word = (d & (H - 1)) * NT + t;
      int sh = (d / H) * 16;
      uint32_t c = cnt[word];
      locp[k / 4] |= ((c >> sh) & 0xFFu) << (8 * (k % 4));
      cnt[word] = c + (1u << sh);
      if (k % 16 == 15) __builtin_amdgcn_sched_barrier(0);  // bound the batch of LDS reads in flight
    }
    __syncthreads();

    // 3. exclusive scan of the packed counters in (digit, thread) order
    {
      uint32_t v[H];
      uint32_t sum = 0;
#pragma unroll
      for (int i = 0; i < H; i++) { v[i] = cnt[t * H + i]; sum += v[i]; }
      uint32_t tot;
      uint32_t run = block_excl_scan<NT>(sum, scan_sh, &tot);
#pragma unroll
      for (int i = 0; i < H; i++) { cnt[t * H + i] = run; run += v[i]; }
      if (t == 0) scan_sh[NT / WAVE + 1] = tot & 0xFFFFu;  // items whose digit < H
    }
    __syncthreads();
    const uint32_t total_low = scan_sh[NT / WAVE + 1];
    // Recompute each item's digit below instead of keeping the count loop's
    // K digit/word/shift values live across the scan (register pressure).
#pragma unroll
    for (int k = 0; k < K; k++) {
      asm volatile("" : "+v"(hi[k]));
      if constexpr (LO) asm volatile("" : "+v"(lo[k]));
    }

    // 4. rank and exchange
#pragma unroll
    for (int k = 0; k < K; k++) {
      uint32_t d = on_lo ? ((lo[k] >> shift) & mask) : ((uint32_t)(hi[k] >> shift) & mask);
      int word = (d & (H - 1)) * NT + t;
      int sh = (d / H) * 16;
      uint32_t base = (cnt[word] >> sh) & 0xFFFFu;
      if (d >= (uint32_t)H) base += total_low;
      int j = pad_idx<K>((int)(base + ((locp[k / 4] >> (8 * (k % 4))) & 0xFFu)));
      xh[j] = hi[k];
      if constexpr (LO) xl[j] = lo[k];
      if constexpr (HASV) xv[j] = val[k];
      if (k % 16 == 15) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();

    if (pass + 1 < npass) {  // back to registers, blocked
#pragma unroll
      for (int k = 0; k < K; k++) {
        int j = pad_idx<K>(t * K + k);
        hi[k] = xh[j];
        if constexpr (LO) lo[k] = xl[j];
        if constexpr (HASV) val[k] = xv[j];
      }
      // the next pass zeroes only this thread's counter column, which no
      // other thread reads before the next barrier
    }
  }
}

// ------------------------------------------------------------ merge path

// Number of elements taken from A among the first `diag` outputs of the
// stable merge of sorted A[0..la) and B[0..lb) (A wins ties).  le(a, b)
// must return a <= b.
template <typename GetA, typename GetB, typename Le>
__device__ __forceinline__ uint64_t merge_path(uint64_t diag, uint64_t la, uint64_t lb, GetA ga, GetB gb,
                                               Le le) {
  uint64_t lo = diag > lb ? diag - lb : 0;
  uint64_t hi = diag < la ? diag : la;
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    // take A[mid] before B[diag-1-mid] iff A[mid] <= B[diag-1-mid]
    if (le(ga(mid), gb(diag - 1 - mid))) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// XCD-aware work-group order: consecutive tiles go to the same XCD (whose
// L2 then sees neighbouring writes), instead of the hardware's round-robin
// of work-group ids over the 8 XCDs.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t grid) {
  constexpr uint32_t NX = 8;
  uint32_t x = bid % NX, i = bid / NX;
  uint32_t q = grid / NX, r = grid % NX;
  uint32_t start = x * q + (x < r ? x : r);
  return start + i;
}

// ------------------------------------------------- LDS counters

// LDS atomic increments by the active lanes of a wave, each on counter
// cnt[b].  When every active lane has the same b (sorted or constant input),
// one atomic serves the whole wave instead of 64 on one address.
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// cnt[b] += 1 per active lane
__device__ __forceinline__ void lds_count(uint32_t* cnt, uint32_t b) {
  const uint64_t act = __ballot(1);
  const uint32_t first = __builtin_amdgcn_readfirstlane(b);
  if (__ballot(b == first) == act) {
    if (lane_rank(act) == 0) atomicAdd(&cnt[b], (uint32_t)__popcll(act));
  } else {
    atomicAdd(&cnt[b], 1u);
  }
}

// old = cnt[b]++ per active lane (distinct slots; order among lanes free)
__device__ __forceinline__ uint32_t lds_claim(uint32_t* cnt, uint32_t b) {
  const uint64_t act = __ballot(1);
  const uint32_t first = __builtin_amdgcn_readfirstlane(b);
  if (__ballot(b == first) == act) {
    const uint32_t r = lane_rank(act);
    uint32_t base = 0;
    if (r == 0) base = atomicAdd(&cnt[b], (uint32_t)__popcll(act));
    return __builtin_amdgcn_readfirstlane(base) + r;
  }
  return atomicAdd(&cnt[b], 1u);
}

// ------------------------------------------------- work-group merge sort

// Sorts the NTH*K u64 values a work-group holds (K per thread, in any
// order) ascending.  Each thread first sorts its K values with an odd-even
// transposition network; then log2(NTH) passes merge pairs of sorted runs
// through LDS, each thread producing K consecutive outputs of its pair
// (its starting point found by a binary search along the merge path).  On
// return thread t holds sorted[t*K .. t*K+K) in v and buf holds the whole
// sorted sequence (buf: NTH*K entries).
template <int NTH, int K>
__device__ __forceinline__ void block_merge_sort_u64(uint64_t (&v)[K], uint64_t* buf) {
#pragma unroll
  for (int pass = 0; pass < K; pass++) {
#pragma unroll
    for (int i = pass & 1; i + 1 < K; i += 2) {
      const uint64_t a = v[i], b = v[i + 1];
      v[i] = a < b ? a : b;
      v[i + 1] = a < b ? b : a;
    }
  }
  const int t = threadIdx.x;
  for (int r = K; r < NTH * K; r *= 2) {
#pragma unroll
    for (int k = 0; k < K; k++) buf[t * K + k] = v[k];
    __syncthreads();
    const int tpg = 2 * r / K;               // threads per merged pair of runs
    const int g = t / tpg, o = (t % tpg) * K;
    const uint64_t* A = buf + g * 2 * r;
    const uint64_t* B = A + r;
    // a = number of A elements among the first o outputs (ties: A first)
    int lo = o > r ? o - r : 0, hi = o < r ? o : r;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (A[mid] <= B[o - 1 - mid]) lo = mid + 1;
      else hi = mid;
    }
    int ia = lo, ib = o - lo;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const bool ha = ia < r, hb = ib < r;
      const uint64_t x = ha ? A[ia] : ~0ull;
      const uint64_t y = hb ? B[ib] : ~0ull;
      const bool takeA = ha && (!hb || x <= y);
      v[k] = takeA ? x : y;
      ia += takeA ? 1 : 0;
      ib += takeA ? 0 : 1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < K; k++) buf[t * K + k] = v[k];
  __syncthreads();
}

}  // namespace ss
