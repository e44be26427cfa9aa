// Kernels of the oversampling sample sort (gfx950).
//
// One split level partitions a list of segments (each an independent sort
// problem) into buckets:
//   k_plan          per-segment bucket count p, sample size and offsets
//   k_sample_*      draw the sample: random positions (Alg. 2 step 2) or the
//                   regular order statistics of sorted blocks (Alg. 1 step 2)
//   k_sample_sort_* sort the sample by (key, position), then lay the p-1
//                   splitters (Alg. 1/2 step 3) out as an implicit search tree
//   k_classify      count, per tile, the keys of each bucket (step 4)
//   k_scan_*        exclusive scan of the bucket-major counts -> offsets
//   k_scatter       stable split of the keys into their buckets (step 4)
//   k_bucket_sort_* sort every bucket in LDS (slot sorts; ss_pairs.h for
//                   pairs); buckets too large for one work-group go to the
//                   next level's list (or, past the last planned level, to
//                   a one-work-group merge sort)
// Keys are compared through their order-preserving unsigned image (ord);
// ties are broken by the index inside the segment (Section 2.2's tags), so
// every key is distinct for the split and the result is the stable order.
#pragma once
#include "ss_device.h"

namespace ss {

constexpr int NT = 512;          // threads per work-group (8 waves)
constexpr int MAX_LEVELS = 6;    // split levels including the top one
constexpr int SCAN_ITEMS = 8;    // scan: items per thread
constexpr int SCAN_BLOCK = NT * SCAN_ITEMS;
constexpr int MERGE_V = 4;       // merge: outputs per thread

template <int KW> struct KeyOf;
template <> struct KeyOf<4> { using T = uint32_t; };
template <> struct KeyOf<8> { using T = uint64_t; };
template <int VW> struct ValOf;
template <> struct ValOf<0> { using T = NoVal; };
template <> struct ValOf<4> { using T = uint32_t; };
template <> struct ValOf<8> { using T = uint64_t; };

// Items per thread of the one-work-group sort, by key and payload width;
// NT * KMAX items fit in the 160 KB LDS of a CU.
template <int KW, int VW> struct SmallCap {
  static constexpr int KMAX = (KW + VW <= 4) ? 64 : ((KW + VW <= 8) ? 32 : 16);
  static constexpr int C = NT * KMAX;
};
// Sample records (ord, tag): 4-byte keys pack into one u64.
template <int KW> struct SampleCap {
  static constexpr int KMAX = (KW == 4) ? 32 : 16;
  static constexpr int C = NT * KMAX;
};

// Chunks of a sample too large for one work-group: sorted one per
// work-group, then merged (4-byte keys: small chunks, so many work-groups
// share the sort).
template <int KW> struct SampleChunk {
  static constexpr int K = (KW == 4) ? 4 : SampleCap<KW>::KMAX;
  static constexpr int C = NT * K;
};
// 4-byte samples of up to this many chunks are ranked by chunk pairs
constexpr uint32_t SAMPLE_PAIR_MAXCH = 64;

// Keys per thread in one chunk of the stable split.
template <int KW, int VW, int PMAX = 256> struct SplitChunk {
  static constexpr int KS = (KW + VW <= 4) ? 8 : 4;
  static constexpr int CH = NT * KS;
};

struct SegDesc {          // one sort problem at one split level
  uint64_t beg;           // first element in the level's buffers
  uint64_t seed;          // SplitMix64 state for its random sample
  uint64_t hist_off;      // first entry of its bucket-major counts
  uint32_t len;           // elements
  uint32_t p;             // buckets (power of two; 0 = chosen by k_plan)
  uint32_t lgp;
  uint32_t m;             // sample records
  uint32_t stride;        // splitter i = sample record i*stride - 1
  uint32_t samp_off;      // first sample record
  uint32_t tile_off;      // first tile (global tile index of the level)
  uint32_t ntiles;
  uint32_t bkt_off;       // first bucket (global bucket index of the level)
  uint32_t tree_off;      // first tree slot (p slots, slot 0 unused)
  uint32_t depth;         // split depth (0 = top)
  uint32_t parent_bkt;    // bucket index inside the parent segment
};

struct LevelCtl {
  uint32_t nsegs;
  uint32_t total_samples;
  uint32_t total_tiles;
  uint32_t total_buckets;
  uint64_t total_hist;
  uint32_t total_tree;
  uint32_t max_m;
  uint64_t keys;          // keys in the level's segments (the input of its split)
  uint64_t bucket_keys;   // keys its bucket kernel sorted in place (not handed on)
};

struct SmallEnt { uint64_t beg; uint32_t len; uint32_t pad; };

struct Ctl {              // device control block at the start of the workspace
  uint32_t status;        // SS_ST_* bits
  uint32_t nsmall;        // entries in the small-segment list (up to one work-group's capacity)
  uint32_t ntiny;         // entries in the tiny-segment list (up to 64 keys: one wave each)
  uint32_t nmid;          // entries in the mid-segment list (up to MID_CAP keys: a small work-group each)
  uint32_t nsmall_fb;     // small segments with an index payload the stable slot sort handed to the radix sort
  LevelCtl lv[MAX_LEVELS];
  uint32_t nleft[MAX_LEVELS];   // buckets the slot sort handed on, per level
  uint32_t nleft2[MAX_LEVELS];  // of those, buckets the round-based slot sort handed on
};

enum : uint32_t {
  ST_LIST_FULL = 1u,      // a next-level list was full (the bucket was sorted by the fallback)
  ST_FALLBACK = 2u,       // a bucket larger than one work-group was sorted by the fallback
  ST_BAD_OFFSETS = 4u,    // a segment's offsets decrease, leave [0, total) or exceed max_seg_len (skipped)
};

// Everything one split level needs.
struct LevelArgs {
  SegDesc* segs;
  LevelCtl* ctl;
  SegDesc* next_segs;      // null at the last planned level
  LevelCtl* next_ctl;
  uint32_t next_cap;
  uint32_t seg_cap;
  Ctl* gctl;
  const void* src;         // keys before the split
  const void* vsrc;        // payload before the split (null if none / iota)
  void* dst;               // keys after the split (bucketed)
  void* vdst;
  void* out;               // final output
  void* vout;
  void* tmp;               // workspace copy of the data (scratch for the fallback)
  void* vtmp;
  void* s_ord;             // sample key images (KW bytes each)
  uint32_t* s_tag;         // sample tags
  uint64_t* s_pack;        // 4-byte keys, sorted sample chunks: (ord << 32) | tag per record, or null
  void* tree;              // splitter trees
  uint32_t* tree_tag;      // tags of the tree (8-byte keys)
  uint32_t* hist;          // counts, then offsets (in place)
  uint32_t* scan_part;     // per-block partial sums of the scan
  uint64_t* exp_smp_ord;   // stage export (top level), may be null
  uint64_t* exp_smp_tag;
  uint64_t* exp_spl_ord;
  uint64_t* exp_spl_tag;
  uint64_t* exp_counts;
  SmallEnt* left;          // buckets the slot sort handed on (keys only)
  uint32_t* nleft;
  SmallEnt* left2;         // buckets the round-based slot sort handed on (4-byte keys only)
  uint32_t* nleft2;
  uint32_t tile;           // keys per tile in the split passes
  uint32_t s;              // oversampling factor for automatically sized segments
  uint32_t p_cap;          // largest p for automatically sized segments
  uint32_t target;         // aimed-at bucket size for automatically sized segments
  int kin;                 // key map of src: 0 unsigned, 1 signed, 2 float (the top level reads the
                           // caller's keys; every deeper buffer holds the unsigned images, kin = 0)
  int kout;                // key map of the final output (the caller's key type)
  int iota;                // 1: payload = index in segment, generated (top level)
  uint32_t use_tab;        // 1: automatically sized segments take p and s from tab_* by size class
  uint16_t tab_p[33];      // by size class c (lengths in (2^(c-1), 2^c]): buckets
  uint16_t tab_s[33];      //   and oversampling factor
};

// ------------------------------------------------------------ helpers

// index of the last segment whose field `off` is <= x (segments sorted by it)
template <typename F>
__device__ __forceinline__ uint32_t find_seg(const SegDesc* segs, uint32_t nsegs, uint64_t x, F off) {
  uint32_t lo = 0, hi = nsegs;    // find first with off > x
  while (lo < hi) {
    uint32_t mid = (lo + hi) / 2;
    if (off(segs[mid]) <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

// rank (1-based) among the p-1 splitters of Eytzinger slot k (tree of
// depth lgp: slot 1 is the root, slots 2k and 2k+1 its children)
__device__ __forceinline__ uint32_t eytz_rank(uint32_t k, uint32_t lgp) {
  uint32_t d = 31 - __clz(k);
  uint32_t i = k - (1u << d);
  return (2 * i + 1) << (lgp - 1 - d);
}

__device__ __forceinline__ uint64_t derive_seed(uint64_t seed, uint32_t depth, uint32_t bucket) {
  return sm64_mix(seed ^ sm64_mix(((uint64_t)depth << 32) + bucket));
}

// Keys in flight per thread in the counting and split passes.
// (halved in the split for p > 256, whose per-bucket counters and tree fill the LDS)
template <int KW, int PMAX = 256> struct SplitU {
  static constexpr int U = (KW == 4 ? 16 : 8) / (PMAX > 256 ? 2 : 1);
  static constexpr int CH = U * NT;
};

// search tree in LDS: 4-byte keys as packed u64, 8-byte keys as (ord, tag)
template <int KW, int PMAX>
struct TreeLds;
template <int PMAX>
struct TreeLds<4, PMAX> {
  uint64_t node[PMAX];
  // (every load issued before the first LDS store)
  __device__ void load(const void* tree, const uint32_t*, uint32_t off, uint32_t p) {
    constexpr int R = (PMAX + NT - 1) / NT;
    const uint64_t* t = (const uint64_t*)tree + off;
    uint64_t v[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const uint32_t k = r * NT + threadIdx.x;
      v[r] = k < p ? t[k] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
      const uint32_t k = r * NT + threadIdx.x;
      if (k < p) node[k] = v[r];
    }
  }
  // bucket = #{splitters < (ord, tag)}: walk lgp levels from the root
  __device__ __forceinline__ uint32_t classify(uint32_t ord, uint32_t tag, uint32_t lgp, uint32_t p) const {
    uint64_t e = ((uint64_t)ord << 32) | tag;
    uint32_t k = 1;
    for (uint32_t l = 0; l < lgp; l++) k = 2 * k + (node[k] < e ? 1u : 0u);
    return k - p;
  }
  // U independent walks advanced level by level, so their LDS reads overlap
  template <int U>
  __device__ __forceinline__ void classify_many(const uint32_t (&ord)[U], const uint32_t (&tag)[U], uint32_t lgp,
                                                uint32_t p, uint32_t (&b)[U]) const {
    uint64_t e[U];
#pragma unroll
    for (int u = 0; u < U; u++) { e[u] = ((uint64_t)ord[u] << 32) | tag[u]; b[u] = 1; }
    for (uint32_t l = 0; l < lgp; l++) {
#pragma unroll
      for (int u = 0; u < U; u++) b[u] = 2 * b[u] + (node[b[u]] < e[u] ? 1u : 0u);
    }
#pragma unroll
    for (int u = 0; u < U; u++) b[u] -= p;
  }
};
template <int PMAX>
struct TreeLds<8, PMAX> {
  uint64_t node[PMAX];
  uint32_t tag[PMAX];
  __device__ void load(const void* tree, const uint32_t* ttag, uint32_t off, uint32_t p) {
    constexpr int R = (PMAX + NT - 1) / NT;
    const uint64_t* t = (const uint64_t*)tree + off;
    uint64_t v[R];
    uint32_t g[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const uint32_t k = r * NT + threadIdx.x;
      v[r] = k < p ? t[k] : 0ull;
      g[r] = k < p ? ttag[off + k] : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
      const uint32_t k = r * NT + threadIdx.x;
      if (k < p) {
        node[k] = v[r];
        tag[k] = g[r];
      }
    }
  }
  __device__ __forceinline__ uint32_t classify(uint64_t ord, uint32_t tg, uint32_t lgp, uint32_t p) const {
    uint32_t k = 1;
    for (uint32_t l = 0; l < lgp; l++) {
      uint64_t a = node[k];
      bool less = (a < ord) || (a == ord && tag[k] < tg);
      k = 2 * k + (less ? 1u : 0u);
    }
    return k - p;
  }
  template <int U>
  __device__ __forceinline__ void classify_many(const uint64_t (&ord)[U], const uint32_t (&tg)[U], uint32_t lgp,
                                                uint32_t p, uint32_t (&b)[U]) const {
#pragma unroll
    for (int u = 0; u < U; u++) b[u] = 1;
    for (uint32_t l = 0; l < lgp; l++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        uint64_t a = node[b[u]];
        bool less = (a < ord[u]) || (a == ord[u] && tag[b[u]] < tg[u]);
        b[u] = 2 * b[u] + (less ? 1u : 0u);
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) b[u] -= p;
  }
};

// ------------------------------------------------------- one-WG sort

// LDS of the one-work-group sort of (key, payload) items.
template <int KW, int VW, int KMAX>
struct SmallLds {
  using KT = typename KeyOf<KW>::T;
  static constexpr int SLOTS = SortShape<NT, KMAX>::SLOTS;
  uint32_t cnt[RadixLds<NT>::CNT_WORDS];
  KT xh[SLOTS];
  typename std::conditional<VW == 0, char, typename std::conditional<VW == 4, uint32_t, uint64_t>::type>::type
      xv[VW == 0 ? 1 : SLOTS];
  alignas(8) uint64_t red[64];
};

// Sort src[beg, beg+len) (len <= NT*K) into out[beg, beg+len).  The payload
// comes from vsrc, or is the index inside the segment (iota_base + i) when
// vsrc is null and the payload type is not NoVal.
template <int KW, int VW, int K, int KMAX>
__device__ __forceinline__ void sort_small_k(const typename KeyOf<KW>::T* src, const void* vsrc,
                             typename KeyOf<KW>::T* out, void* vout, uint64_t beg, uint32_t len,
                             uint64_t iota_base, int kin, int kout, SmallLds<KW, VW, KMAX>& sm) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  constexpr bool HASV = VW != 0;
  const int t = threadIdx.x;
  VT* xv = (VT*)(void*)sm.xv;
  // striped (coalesced) load into LDS, then blocked registers; a bounded
  // unroll keeps the number of in-flight load addresses in check (each
  // element is read and written once: streaming loads and stores)
#pragma unroll 8
  for (int r = 0; r < K; r++) {
    int i = r * NT + t;
    int j = pad_idx<K>(i);
    if (i < (int)len) {
      sm.xh[j] = to_ord(__builtin_nontemporal_load(&src[beg + i]), kin);
      if constexpr (HASV) {
        if (vsrc) xv[j] = __builtin_nontemporal_load(&((const VT*)vsrc)[beg + i]);
        else xv[j] = (VT)(iota_base + i);
      }
    } else {
      sm.xh[j] = ~KT(0);
    }
  }
  __syncthreads();
  KT hi[K];
  uint32_t lo[K];
  VT val[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    int j = pad_idx<K>(t * K + k);
    hi[k] = sm.xh[j];
    if constexpr (HASV) val[k] = xv[j];
  }
  // (the sort's first LDS exchange comes after its internal barriers)
  block_radix_sort<NT, K, KT, false, VT>(hi, lo, val, (int)len, sm.cnt, sm.xh, nullptr, xv, sm.red);
#pragma unroll 8
  for (int r = 0; r < K; r++) {
    int i = r * NT + t;
    if (i < (int)len) {
      int j = pad_idx<K>(i);
      __builtin_nontemporal_store(from_ord(sm.xh[j], kout), &out[beg + i]);
      if constexpr (HASV) __builtin_nontemporal_store(xv[j], &((VT*)vout)[beg + i]);
    }
  }
  __syncthreads();
}

template <int KW, int VW>
__device__ __forceinline__ void sort_small(const typename KeyOf<KW>::T* src, const void* vsrc, typename KeyOf<KW>::T* out,
                           void* vout, uint64_t beg, uint32_t len, uint64_t iota_base, int kin, int kout,
                           SmallLds<KW, VW, SmallCap<KW, VW>::KMAX>& sm) {
  constexpr int KMAX = SmallCap<KW, VW>::KMAX;
  if (len <= (uint32_t)NT * 1) sort_small_k<KW, VW, 1, KMAX>(src, vsrc, out, vout, beg, len, iota_base, kin, kout, sm);
  else if (len <= (uint32_t)NT * 4) sort_small_k<KW, VW, 4, KMAX>(src, vsrc, out, vout, beg, len, iota_base, kin, kout, sm);
  else if (len <= (uint32_t)NT * 8) sort_small_k<KW, VW, 8, KMAX>(src, vsrc, out, vout, beg, len, iota_base, kin, kout, sm);
  else if (len <= (uint32_t)NT * 16) sort_small_k<KW, VW, 16, KMAX>(src, vsrc, out, vout, beg, len, iota_base, kin, kout, sm);
  else if (KMAX > 32 && len <= (uint32_t)NT * 32)
    sort_small_k<KW, VW, (KMAX > 32 ? 32 : KMAX), KMAX>(src, vsrc, out, vout, beg, len, iota_base, kin, kout, sm);
  else sort_small_k<KW, VW, KMAX, KMAX>(src, vsrc, out, vout, beg, len, iota_base, kin, kout, sm);
}

// One work-group sorts a segment of any length: LDS-sorted chunks of C
// items, then stable two-way merges (merge path) through global memory,
// alternating between `out` and `alt`, ending in `out`.  `cur` holds the
// data (it may be `out` or `alt`).
template <int KW, int VW>
__device__ void sort_big_wg(const typename KeyOf<KW>::T* cur, const void* vcur, typename KeyOf<KW>::T* out,
                            void* vout, typename KeyOf<KW>::T* alt, void* valt, uint64_t beg, uint64_t len,
                            uint64_t iota_base, int kin, int kout, SmallLds<KW, VW, SmallCap<KW, VW>::KMAX>& sm) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  constexpr bool HASV = VW != 0;
  constexpr uint64_t C = SmallCap<KW, VW>::C;
  uint64_t nch = (len + C - 1) / C;
  int passes = 0;
  while ((C << passes) < len) passes++;
  // the merges alternate buffers; pick the chunk-sort target so the last lands in out
  KT* b0 = (passes % 2 == 0) ? out : alt;
  void* vb0 = (passes % 2 == 0) ? vout : valt;
  KT* b1 = (passes % 2 == 0) ? alt : out;
  void* vb1 = (passes % 2 == 0) ? valt : vout;
  for (uint64_t c = 0; c < nch; c++) {
    uint64_t cb = c * C;
    uint32_t cl = (uint32_t)((len - cb) < C ? (len - cb) : C);
    sort_small<KW, VW>(cur, vcur, b0, vb0, beg + cb, cl, iota_base + cb, kin, kout, sm);
  }
  if (passes == 0) return;
  __threadfence_block();
  for (int ps = 0; ps < passes; ps++) {
    __syncthreads();
    uint64_t run = C << ps;
    const KT* a = b0;
    const VT* va = (const VT*)vb0;
    KT* o = b1;
    VT* vo = (VT*)vb1;
    for (uint64_t pb = 0; pb < len; pb += 2 * run) {
      uint64_t la = (len - pb) < run ? (len - pb) : run;
      uint64_t lb = (len - pb - la) < run ? (len - pb - la) : run;
      const KT* A = a + beg + pb;
      const KT* B = A + la;
      uint64_t tot = la + lb;
      for (uint64_t d0 = 0; d0 < tot; d0 += (uint64_t)NT * MERGE_V) {
        uint64_t d = d0 + (uint64_t)threadIdx.x * MERGE_V;
        if (d < tot) {
          auto ga = [&](uint64_t i) { return to_ord(A[i], kout); };
          auto gb = [&](uint64_t i) { return to_ord(B[i], kout); };
          uint64_t i = merge_path(d, la, lb, ga, gb, [](KT x, KT y) { return x <= y; });
          uint64_t j = d - i;
          for (int v = 0; v < MERGE_V && d + v < tot; v++) {
            bool takeA;
            if (i >= la) takeA = false;
            else if (j >= lb) takeA = true;
            else takeA = to_ord(A[i], kout) <= to_ord(B[j], kout);
            uint64_t dst = beg + pb + d + v;
            if (takeA) {
              o[dst] = A[i];
              if constexpr (HASV) vo[dst] = va[beg + pb + i];
              i++;
            } else {
              o[dst] = B[j];
              if constexpr (HASV) vo[dst] = va[beg + pb + la + j];
              j++;
            }
          }
        }
      }
    }
    __threadfence_block();
    // swap roles
    KT* tk = b0; b0 = b1; b1 = tk;
    void* tv = vb0; vb0 = vb1; vb1 = tv;
  }
  __syncthreads();
}

// ------------------------------------------------------------ kernels

// Per segment: bucket count, sample size, tile count and prefix offsets.
// One work-group.  Segments with p == 0 are sized here from their length:
// enough buckets for about `target` keys each (at most p_cap), and an
// oversampling factor cut so that p*s < len/2 (Claim 1's precondition) and
// the sample fits one work-group.
__global__ void __launch_bounds__(NT) k_plan(LevelArgs a, uint32_t samp_cap) {
  __shared__ uint64_t sh64[NT / WAVE + 2];
  __shared__ uint32_t sh32[NT / WAVE + 2];
  const uint32_t n = min(a.ctl->nsegs, a.seg_cap);
  uint32_t run_s = 0, run_t = 0, run_b = 0, max_m = 0;
  uint64_t run_h = 0, run_k = 0;
  for (uint32_t base = 0; base < n; base += NT) {
    const uint32_t i = base + threadIdx.x;
    uint32_t m = 0, nt = 0, p = 0;
    uint64_t h = 0;
    SegDesc d = {};
    if (i < n) {
      d = a.segs[i];
      if (d.p == 0) {
        uint32_t want = (d.len + a.target - 1) / a.target;
        uint32_t q = 2;
        while (q < want && q < a.p_cap) q *= 2;
        uint32_t sv = a.s;
        if (a.use_tab) {
          // the tuned p of the segment's size class (never above the target
          // rule's, which sized the level's bucket arrays; 0 = that rule)
          uint32_t c = 0;
          while (c < 32 && (1ull << c) < (uint64_t)d.len) c++;
          if (a.tab_p[c]) q = min(q, max(2u, (uint32_t)a.tab_p[c]));
          if (a.tab_s[c]) sv = a.tab_s[c];
        }
        if ((uint64_t)q * sv > (uint64_t)samp_cap + 1) sv = (samp_cap + 1) / q;
        if ((uint64_t)2 * q * sv >= d.len) sv = (d.len - 1) / (2 * q);
        if (sv < 1) sv = 1;
        d.p = q;
        d.m = q * sv - 1;
        d.stride = sv;
      }
      d.lgp = 31 - __clz(d.p);
      d.ntiles = (d.len + a.tile - 1) / a.tile;
      m = d.m;
      nt = d.ntiles;
      p = d.p;
      h = (uint64_t)p * nt;
    }
    uint32_t ts, tt, tb;
    uint64_t th;
    const uint32_t so = block_excl_scan<NT>(m, sh32, &ts);
    const uint32_t to = block_excl_scan<NT>(nt, sh32, &tt);
    const uint32_t bo = block_excl_scan<NT>(p, sh32, &tb);
    const uint64_t ho = block_excl_scan<NT, uint64_t>(h, sh64, &th);
    uint64_t tk;
    block_excl_scan<NT, uint64_t>(i < n ? (uint64_t)d.len : 0ull, sh64, &tk);
    const uint32_t wm = wave_max(m);
    if (lane_id() == 0) sh32[wave_id()] = wm;
    __syncthreads();
    for (int w = 0; w < NT / WAVE; w++) max_m = sh32[w] > max_m ? sh32[w] : max_m;
    __syncthreads();
    if (i < n) {
      d.samp_off = run_s + so;
      d.tile_off = run_t + to;
      d.bkt_off = run_b + bo;
      d.tree_off = run_b + bo;
      d.hist_off = run_h + ho;
      a.segs[i] = d;
    }
    run_s += ts;
    run_t += tt;
    run_b += tb;
    run_h += th;
    run_k += tk;
  }
  if (threadIdx.x == 0) {
    a.ctl->nsegs = n;
    a.ctl->total_samples = run_s;
    a.ctl->total_tiles = run_t;
    a.ctl->total_buckets = run_b;
    a.ctl->total_tree = run_b;
    a.ctl->total_hist = run_h;
    a.ctl->max_m = max_m;
    a.ctl->keys = run_k;
    a.ctl->bucket_keys = 0;
  }
}

// Random sample (Alg. 2 step 2): record j of segment g is the key at
// in-segment position floor(r_j * len / 2^64), r_j the (j+1)-th output of
// the segment's SplitMix64 generator; tag = that position.
template <int KW>
__global__ void __launch_bounds__(256) k_sample_random(LevelArgs a) {
  using KT = typename KeyOf<KW>::T;
  const uint32_t total = a.ctl->total_samples, nsegs = a.ctl->nsegs;
  for (uint32_t g = blockIdx.x * 256 + threadIdx.x; g < total; g += gridDim.x * 256) {
    uint32_t si = find_seg(a.segs, nsegs, g, [](const SegDesc& d) { return (uint64_t)d.samp_off; });
    SegDesc d = a.segs[si];
    uint32_t j = g - d.samp_off;
    uint64_t pos = scale_to(sm64_at(d.seed, j), d.len);
    KT key = to_ord(((const KT*)a.src)[d.beg + pos], a.kin);
    ((KT*)a.s_ord)[g] = key;
    a.s_tag[g] = (uint32_t)pos;
  }
}

// LDS of the one-work-group sample sort.
template <int KW>
struct SampleLds {
  static constexpr int KMAX = SampleCap<KW>::KMAX;
  static constexpr int SLOTS = SortShape<NT, KMAX>::SLOTS;
  uint32_t cnt[RadixLds<NT>::CNT_WORDS];
  uint64_t xh[SLOTS];
  uint32_t xl[KW == 8 ? SLOTS : 1];
  alignas(8) uint64_t red[64];
};

// Write splitter tree slot k from sorted record (ord, tag), and export.
template <int KW>
__device__ __forceinline__ void put_tree(const LevelArgs& a, const SegDesc& d, uint32_t k,
                                         typename KeyOf<KW>::T ord, uint32_t tag, bool exp) {
  if constexpr (KW == 4) ((uint64_t*)a.tree)[d.tree_off + k] = ((uint64_t)ord << 32) | tag;
  else {
    ((uint64_t*)a.tree)[d.tree_off + k] = ord;
    a.tree_tag[d.tree_off + k] = tag;
  }
  if (exp) {
    uint32_t r = eytz_rank(k, d.lgp);
    a.exp_spl_ord[r - 1] = (uint64_t)ord;
    a.exp_spl_tag[r - 1] = tag;
  }
}

// One work-group per segment: sort its sample (m <= SampleCap) by (key,
// tag) in LDS, then write the splitter tree: splitter i = sorted record
// i*stride - 1 (1-based i, Alg. 1/2 step 3).
template <int KW, int K>
__device__ __forceinline__ void sample_sort_one(const LevelArgs& a, const SegDesc& d, SampleLds<KW>& sm, bool exp) {
  using KT = typename KeyOf<KW>::T;
  constexpr int KM = SampleLds<KW>::KMAX;
  const int t = threadIdx.x;
  const KT* so = (const KT*)a.s_ord + d.samp_off;
  const uint32_t* st = a.s_tag + d.samp_off;
  const int m = (int)d.m;
  if constexpr (KW == 4) {
    // 4-byte keys: (ord, tag) packed in a u64, merge-sorted in LDS
    uint64_t v[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = t * K + k;
      v[k] = i < m ? (((uint64_t)so[i] << 32) | st[i]) : ~0ull;
    }
    block_merge_sort_u64<NT, K>(v, sm.xh);
    for (int i = t; i < m; i += NT) {
      const uint64_t x = sm.xh[i];
      ((KT*)a.s_ord)[d.samp_off + i] = (KT)(x >> 32);
      a.s_tag[d.samp_off + i] = (uint32_t)x;
      if (a.s_pack) a.s_pack[d.samp_off + i] = x;
      if (exp) { a.exp_smp_ord[i] = x >> 32; a.exp_smp_tag[i] = (uint32_t)x; }
    }
    for (uint32_t k = 1 + t; k < d.p; k += NT) {
      const uint32_t r = eytz_rank(k, d.lgp);
      const uint64_t x = sm.xh[r * d.stride - 1];
      put_tree<KW>(a, d, k, (KT)(x >> 32), (uint32_t)x, exp);
    }
    __syncthreads();
    return;
  }
  uint64_t hi[K];
  uint32_t lo[K];
  NoVal nv[K];
  // striped load to LDS then blocked registers
#pragma unroll
  for (int r = 0; r < K; r++) {
    int i = r * NT + t;
    int j = pad_idx<K>(i);
    if (i < m) {
      if constexpr (KW == 4) sm.xh[j] = ((uint64_t)so[i] << 32) | st[i];
      else { sm.xh[j] = so[i]; sm.xl[j] = st[i]; }
    } else {
      sm.xh[j] = ~0ull;
      if constexpr (KW == 8) sm.xl[j] = ~0u;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) {
    int j = pad_idx<K>(t * K + k);
    hi[k] = sm.xh[j];
    if constexpr (KW == 8) lo[k] = sm.xl[j];
  }
  block_radix_sort<NT, K, uint64_t, KW == 8, NoVal>(hi, lo, nv, m, sm.cnt, sm.xh, sm.xl, nullptr, sm.red);
  (void)KM;
  // sorted records back to global (kept for the stage export)
  for (int i = t; i < m; i += NT) {
    int j = pad_idx<K>(i);
    KT ord;
    uint32_t tag;
    if constexpr (KW == 4) { ord = (KT)(sm.xh[j] >> 32); tag = (uint32_t)sm.xh[j]; }
    else { ord = sm.xh[j]; tag = sm.xl[j]; }
    ((KT*)a.s_ord)[d.samp_off + i] = ord;
    a.s_tag[d.samp_off + i] = tag;
    if (exp) { a.exp_smp_ord[i] = (uint64_t)ord; a.exp_smp_tag[i] = tag; }
  }
  for (uint32_t k = 1 + t; k < d.p; k += NT) {
    uint32_t r = eytz_rank(k, d.lgp);
    int j = pad_idx<K>((int)(r * d.stride - 1));
    KT ord;
    uint32_t tag;
    if constexpr (KW == 4) { ord = (KT)(sm.xh[j] >> 32); tag = (uint32_t)sm.xh[j]; }
    else { ord = sm.xh[j]; tag = sm.xl[j]; }
    put_tree<KW>(a, d, k, ord, tag, exp);
  }
  __syncthreads();
}

template <int KW>
__global__ void __launch_bounds__(NT) k_sample_sort_wg(LevelArgs a, int export_stages) {
  __shared__ SampleLds<KW> sm;
  const uint32_t g = blockIdx.x;
  if (g >= a.ctl->nsegs) return;
  SegDesc d = a.segs[g];
  constexpr int KM = SampleLds<KW>::KMAX;
  if (d.m > (uint32_t)NT * KM) return;  // sorted by the multi-work-group path
  bool exp = export_stages && d.depth == 0 && g == 0;
  if (d.m <= (uint32_t)NT) sample_sort_one<KW, 1>(a, d, sm, exp);
  else if (d.m <= (uint32_t)NT * 4) sample_sort_one<KW, 4>(a, d, sm, exp);
  else if (d.m <= (uint32_t)NT * 16) sample_sort_one<KW, 16>(a, d, sm, exp);
  else sample_sort_one<KW, KM>(a, d, sm, exp);
}

// Large top-level sample (one segment): chunk sorts (then k_sample_rank).
template <int KW>
__global__ void __launch_bounds__(NT) k_sample_chunk_sort(LevelArgs a) {
  __shared__ SampleLds<KW> sm;
  using KT = typename KeyOf<KW>::T;
  constexpr int KM = SampleChunk<KW>::K;
  constexpr int C = SampleChunk<KW>::C;
  SegDesc d = a.segs[0];
  uint32_t cb = blockIdx.x * C;
  if (cb >= d.m) return;
  SegDesc dc = d;
  dc.samp_off = d.samp_off + cb;
  dc.m = (d.m - cb) < (uint32_t)C ? (d.m - cb) : (uint32_t)C;
  dc.p = 1;  // no tree from a chunk
  sample_sort_one<KW, KM>(a, dc, sm, false);
  (void)sizeof(KT);
}

// The top level of a single sort whose 4-byte sample is ranked by chunk
// pairs, in one launch: work-group 0 also writes the level's descriptor and
// counters (as k_init_single), and every work-group draws its chunk of the
// sample itself -- record j is the key at position floor(r_j * n / 2^64),
// r_j the j-th output of the seeded generator, as k_sample_random draws it
// (Alg. 2 step 2) -- then sorts the chunk by (key, position) and writes the
// packed records the rank pass reads.
struct TopInit {
  uint64_t n, seed;
  uint32_t p, m, stride, tile;
};
__device__ __forceinline__ void init_single(Ctl* g, SegDesc* segs, uint64_t n, uint32_t p, uint32_t m,
                                            uint32_t stride, uint64_t seed, uint32_t tile);

__global__ void __launch_bounds__(NT) k_sample_draw_sort(LevelArgs a, Ctl* g, SegDesc* segs, TopInit ti) {
  __shared__ SampleLds<4> sm;
  constexpr int K = SampleChunk<4>::K;
  constexpr uint32_t C = SampleChunk<4>::C;
  if (blockIdx.x == 0 && threadIdx.x == 0) init_single(g, segs, ti.n, ti.p, ti.m, ti.stride, ti.seed, ti.tile);
  const uint32_t cb = blockIdx.x * C;
  if (cb >= ti.m) return;
  const uint32_t len = min(C, ti.m - cb);
  const int t = threadIdx.x;
  const uint32_t* src = (const uint32_t*)a.src;
  uint64_t pos[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const uint32_t i = t * K + k;
    pos[k] = i < len ? scale_to(sm64_at(ti.seed, cb + i), ti.n) : 0ull;
  }
  uint64_t v[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const uint32_t i = t * K + k;
    v[k] = i < len ? (((uint64_t)to_ord(src[pos[k]], a.kin) << 32) | (uint32_t)pos[k]) : ~0ull;
  }
  block_merge_sort_u64<NT, K>(v, sm.xh);
  for (uint32_t i = t; i < len; i += NT) a.s_pack[cb + i] = sm.xh[i];
}

// Sorted chunks of a large sample to splitters in one pass: the rank of a
// record among all m records is its index in its own (sorted) chunk plus,
// for every other chunk, the number of that chunk's records before it in
// (ord, tag) order -- records of earlier chunks that equal it count as
// before it, those of later chunks as after, so equal records (a position
// drawn twice) still get distinct ranks.  A record whose 1-based rank is a
// multiple of the stride below p * stride is splitter rank / stride (step
// 3) and goes to its slot of the implicit tree; with the stage export on
// every record is also written at its rank.
//
// 2^lgL lanes (aligned inside a wave, lgL <= 6) serve one record: lane j
// searches chunks j, j + 2^lgL, ..., and a butterfly sum over the group
// adds the counts, so the dependent reads of the binary searches are spread
// over many waves instead of one thread's long chain.
template <int KW>
__global__ void __launch_bounds__(256) k_sample_rank(LevelArgs a, int export_stages, uint32_t lgL) {
  using KT = typename KeyOf<KW>::T;
  constexpr uint32_t C = SampleChunk<KW>::C;
  const SegDesc d = a.segs[0];
  const uint64_t gt = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t L = 1u << lgL;
  const uint64_t g64 = gt >> lgL;
  const uint32_t lane = (uint32_t)gt & (L - 1);
  const bool live = g64 < d.m;
  const uint32_t g = live ? (uint32_t)g64 : 0u;
  const KT* so = (const KT*)a.s_ord + d.samp_off;
  const uint32_t* st = a.s_tag + d.samp_off;
  KT k = 0;
  uint32_t tg = 0, cnt = 0;
  if (live) {
    k = so[g];
    tg = st[g];
    const uint32_t c = g / C, nch = (d.m + C - 1) / C;
    // 4-byte keys with the packed copy: one 8-byte read per search step
    const uint64_t* pk = KW == 4 ? a.s_pack : nullptr;
    const uint64_t me = ((uint64_t)k << 32) | tg;
    for (uint32_t j = lane; j < nch; j += L) {
      if (j == c) {
        cnt += g - c * C;
        continue;
      }
      const uint32_t b = j * C, len = min(C, d.m - b);
      const bool le = j < c;                  // count records <= (k, tg), else < (k, tg)
      uint32_t lo = 0, hi = len;
      if (pk) {
        const uint64_t* q = pk + d.samp_off + b;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          const uint64_t x = q[mid];
          if (le ? x <= me : x < me) lo = mid + 1;
          else hi = mid;
        }
      } else {
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          const KT ok = so[b + mid];
          const uint32_t ot = st[b + mid];
          const bool before = ok < k || (ok == k && (le ? ot <= tg : ot < tg));
          if (before) lo = mid + 1;
          else hi = mid;
        }
      }
      cnt += lo;
    }
  }
  for (uint32_t o = L >> 1; o > 0; o >>= 1) cnt += __shfl_xor(cnt, (int)o, WAVE);
  if (!live || lane != 0) return;
  const uint32_t rank = cnt;
  const bool exp = export_stages != 0;
  if (exp) {
    a.exp_smp_ord[rank] = (uint64_t)k;
    a.exp_smp_tag[rank] = tg;
  }
  const uint32_t r1 = rank + 1;
  if (r1 % d.stride == 0) {
    const uint32_t r = r1 / d.stride;         // splitter rank, 1-based
    if (r >= 1 && r < d.p) {
      const uint32_t z = __builtin_ctz(r);
      const uint32_t slot = (1u << (d.lgp - 1 - z)) + (r >> (z + 1));
      put_tree<KW>(a, d, slot, k, tg, exp);
    }
  }
}

// The same ranks for a 4-byte sample of at most SAMPLE_PAIR_MAXCH chunks,
// in two launches.  First one work-group per ordered pair of chunks (c, j),
// j != c: chunk j's packed records (ord << 32 | tag, whose order is the
// records' order) are staged in LDS and every record of chunk c counts
// those before it by a binary search there (<= for an earlier chunk, < for
// a later one): cnt[j * m + g] for record g of chunk c.
__global__ void __launch_bounds__(NT) k_sample_pair_count(LevelArgs a, uint16_t* cnt) {
  constexpr uint32_t C = SampleChunk<4>::C;
  constexpr int KR = SampleChunk<4>::K;           // records of chunk c per thread
  static_assert((C & (C - 1)) == 0, "power-of-two chunks");
  __shared__ uint64_t sj[C];
  const SegDesc d = a.segs[0];
  const uint32_t m = d.m, nch = (m + C - 1) / C;
  const uint32_t c = blockIdx.x / nch, j = blockIdx.x % nch;
  if (c >= nch || j == c) return;
  const int t = threadIdx.x;
  const uint64_t* q = a.s_pack + d.samp_off;
  const uint32_t cb = c * C, clen = min(C, m - cb), jb = j * C, jlen = min(C, m - jb);
  // chunk j to LDS, padded with all-ones records (above every record: a tag
  // is a position below 2^32 - 1), and this thread's KR records of chunk c
  uint64_t v[KR], x[KR];
#pragma unroll
  for (int r = 0; r < KR; r++) {
    const uint32_t i = r * NT + t;
    v[r] = i < jlen ? q[jb + i] : ~0ull;
    const uint32_t ic = t * KR + r;
    x[r] = ic < clen ? q[cb + ic] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < KR; r++) sj[r * NT + t] = v[r];
  __syncthreads();
  const bool le = j < c;
  // records of chunk j before x: the predicate holds on a prefix of sj;
  // fixed-step binary lifting, the KR searches side by side
  uint32_t pos[KR];
#pragma unroll
  for (int r = 0; r < KR; r++) pos[r] = 0;
  for (uint32_t b = C; b > 0; b >>= 1) {
#pragma unroll
    for (int r = 0; r < KR; r++) {
      const uint32_t at = pos[r] + b;
      const uint64_t y = sj[min(at, C) - 1];
      const bool before = le ? y <= x[r] : y < x[r];
      pos[r] = (at <= C && before) ? at : pos[r];
    }
  }
#pragma unroll
  for (int r = 0; r < KR; r++) {
    const uint32_t ic = t * KR + r;
    if (ic < clen) cnt[(uint64_t)j * m + cb + ic] = (uint16_t)pos[r];
  }
}

// Second launch: rank of record g = its index in its chunk plus its counts
// in the other chunks; splitters to the tree, records to the stage export.
__global__ void __launch_bounds__(256) k_sample_rank_sum(LevelArgs a, const uint16_t* cnt, int export_stages) {
  constexpr uint32_t C = SampleChunk<4>::C;
  const SegDesc d = a.segs[0];
  const uint32_t g = blockIdx.x * 256 + threadIdx.x;
  if (g >= d.m) return;
  const uint32_t m = d.m, nch = (m + C - 1) / C, c = g / C;
  uint32_t rank = g - c * C;
  for (uint32_t j0 = 0; j0 < nch; j0 += 8) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const uint32_t j = j0 + u;
      v[u] = (j < nch && j != c) ? (uint32_t)cnt[(uint64_t)j * m + g] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; u++) rank += v[u];
  }
  const uint64_t x = a.s_pack[d.samp_off + g];
  const uint32_t k = (uint32_t)(x >> 32), tg = (uint32_t)x;
  const bool exp = export_stages != 0;
  if (exp) {
    a.exp_smp_ord[rank] = (uint64_t)k;
    a.exp_smp_tag[rank] = tg;
  }
  const uint32_t r1 = rank + 1;
  if (r1 % d.stride == 0) {
    const uint32_t r = r1 / d.stride;         // splitter rank, 1-based
    if (r >= 1 && r < d.p) {
      const uint32_t z = __builtin_ctz(r);
      const uint32_t slot = (1u << (d.lgp - 1 - z)) + (r >> (z + 1));
      put_tree<4>(a, d, slot, k, tg, exp);
    }
  }
}

// Splitter tree (and stage export) from a sorted sample in global memory.
template <int KW>
__global__ void __launch_bounds__(256) k_build_tree(LevelArgs a, const void* sord, const uint32_t* stag,
                                                    int export_stages) {
  using KT = typename KeyOf<KW>::T;
  SegDesc d = a.segs[0];
  bool exp = export_stages != 0;
  const KT* so = (const KT*)sord;
  uint32_t gid = blockIdx.x * 256 + threadIdx.x;
  for (uint32_t k = gid; k < d.p; k += gridDim.x * 256) {
    if (k == 0) continue;
    uint32_t r = eytz_rank(k, d.lgp);
    uint32_t idx = d.samp_off + r * d.stride - 1;
    put_tree<KW>(a, d, k, so[idx], stag[idx], exp);
  }
  if (exp) {
    for (uint32_t i = gid; i < d.m; i += gridDim.x * 256) {
      a.exp_smp_ord[i] = (uint64_t)so[d.samp_off + i];
      a.exp_smp_tag[i] = stag[d.samp_off + i];
    }
  }
}

// Widening of a 32-bit index payload into the caller's 64-bit one: all of
// [0, n) for an array; for segments, [off[0], off[nseg]) (off == nullptr:
// the whole range).
__global__ void __launch_bounds__(256) k_widen_index(const uint32_t* v32, int64_t* v64, const int64_t* off,
                                                     uint64_t nseg, uint64_t n) {
  uint64_t b = 0, e = n;
  if (off) {
    const int64_t ob = off[0], oe = off[nseg];
    b = ob < 0 ? 0 : (uint64_t)ob;
    e = oe < ob ? b : (uint64_t)oe;
    if (e > n) e = n;
  }
  for (uint64_t i = b + (uint64_t)blockIdx.x * 256 + threadIdx.x; i < e; i += (uint64_t)gridDim.x * 256)
    v64[i] = (int64_t)v32[i];
}

// A sample of 4-byte keys of 2^20 records or more (beyond what the chunk
// ranks handle well) is sorted as 64-bit keys (ord << 32) | tag, which
// order exactly as the records (key, tag): pack before, unpack after.
constexpr uint64_t SAMPLE_NESTED_MIN = 1ull << 20;

__global__ void __launch_bounds__(256) k_pack_sample(const uint32_t* so, const uint32_t* stag, uint64_t* pk,
                                                     uint64_t m) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (uint64_t)gridDim.x * 256)
    pk[i] = ((uint64_t)so[i] << 32) | stag[i];
}

__global__ void __launch_bounds__(256) k_unpack_sample(const uint64_t* pk, uint32_t* so, uint32_t* stag, uint64_t m) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (uint64_t)gridDim.x * 256) {
    const uint64_t v = pk[i];
    so[i] = (uint32_t)(v >> 32);
    stag[i] = (uint32_t)v;
  }
}

// Regular sample (Alg. 1 steps 1-2) from blocks already sorted by (key,
// in-block index): block k = [floor(k n/p), floor((k+1) n/p)); with
// S = s*p and x = ceil(ceil(n/p)/S), record j of block k is the block's
// record of rank min((j+1) x, |block|) - 1; tag = input position.
template <int KW>
__global__ void __launch_bounds__(256) k_sample_regular(LevelArgs a, const void* skeys, const uint32_t* sidx,
                                                        uint64_t n, uint32_t p, uint32_t S) {
  using KT = typename KeyOf<KW>::T;
  const uint64_t total = (uint64_t)p * S;
  const uint64_t blk_max = (n + p - 1) / p;
  const uint64_t x = (blk_max + S - 1) / S;
  for (uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (uint64_t)gridDim.x * 256) {
    uint64_t k = g / S, j = g % S;
    uint64_t b = (k * n) / p, e = ((k + 1) * n) / p, mk = e - b;
    uint64_t rank = (j + 1) * x;
    if (rank > mk) rank = mk;
    uint64_t at = b + rank - 1;
    ((KT*)a.s_ord)[g] = to_ord(((const KT*)skeys)[at], a.kin);
    a.s_tag[g] = (uint32_t)(b + sidx[at]);
  }
}

// Per-tile bucket counts (step 4), stored bucket-major per segment:
// hist[hist_off + b * ntiles + tile].  Each thread classifies U keys at a
// time (their tree walks advance level by level together) and adds runs of
// equal buckets to an LDS histogram.
template <int KW, int PMAX>
__device__ __forceinline__ void count_block(const LevelArgs& a, const TreeLds<KW, PMAX>& tr, const SegDesc& d,
                                            const typename KeyOf<KW>::T* src, uint32_t i0, uint32_t t1, bool full,
                                            uint32_t* cnt, uint32_t& cur, uint32_t& run) {
  using KT = typename KeyOf<KW>::T;
  constexpr int U = SplitU<KW>::U;
  KT key[U];
  uint32_t tag[U], b[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    uint32_t i = i0 + u * NT + threadIdx.x;
    tag[u] = i;
    key[u] = (full || i < t1) ? to_ord(__builtin_nontemporal_load(&src[i]), a.kin) : KT(0);
  }
  tr.template classify_many<U>(key, tag, d.lgp, d.p, b);
#pragma unroll
  for (int u = 0; u < U; u++) {
    if (full || i0 + u * NT + threadIdx.x < t1) {
      if (b[u] != cur) {
        if (run) atomicAdd(&cnt[cur], run);
        cur = b[u];
        run = 0;
      }
      run++;
    }
  }
}

template <int KW, int PMAX>
__global__ void __launch_bounds__(NT) k_classify(LevelArgs a) {
  using KT = typename KeyOf<KW>::T;
  constexpr int CH = SplitU<KW>::CH;
  __shared__ TreeLds<KW, PMAX> tr;
  __shared__ uint32_t cnt[PMAX];
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const LevelCtl c = *a.ctl;
  if (tile >= c.total_tiles) return;
  const uint32_t si = find_seg(a.segs, c.nsegs, tile, [](const SegDesc& d) { return (uint64_t)d.tile_off; });
  const SegDesc d = a.segs[si];
  const uint32_t tw = tile - d.tile_off;
  tr.load(a.tree, a.tree_tag, d.tree_off, d.p);
  for (uint32_t b = threadIdx.x; b < d.p; b += NT) cnt[b] = 0;
  __syncthreads();
  const uint32_t t0 = tw * a.tile;
  const uint32_t t1 = min(t0 + a.tile, d.len);
  const KT* src = (const KT*)a.src + d.beg;
  uint32_t cur = ~0u, run = 0;
  uint32_t i0 = t0;
  for (; i0 + CH <= t1; i0 += CH) {
    if (i0 + 2 * CH <= t1) {   // start fetching the next block (lands in L2 / L1)
#pragma unroll
      for (int u = 0; u < SplitU<KW>::U; u += 4) __builtin_prefetch(&src[i0 + CH + u * NT + threadIdx.x]);
    }
    count_block<KW, PMAX>(a, tr, d, src, i0, t1, true, cnt, cur, run);
  }
  if (i0 < t1) count_block<KW, PMAX>(a, tr, d, src, i0, t1, false, cnt, cur, run);
  if (run) atomicAdd(&cnt[cur], run);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < d.p; b += NT) a.hist[d.hist_off + (uint64_t)b * d.ntiles + tw] = cnt[b];
}

// Exclusive scan of an array of counts in place (u32, wrapping mod 2^32;
// only differences inside one sort problem are used, and those are < 2^32).
// The length is total_dev[0] when total_dev is given, else total.
__device__ __forceinline__ uint64_t scan_len(uint64_t total, const uint64_t* total_dev) {
  return total_dev ? *total_dev : total;
}

// Up to two arrays per launch: blocks [0, nb1) scan array 1 (h, part,
// total), the rest array 2 (h2, part2, total2; total2 given on the host).
struct ScanPair {
  uint32_t* h2 = nullptr;
  uint32_t* part2 = nullptr;
  uint64_t total2 = 0;
  uint32_t nb1 = 0xFFFFFFFFu;
};

__device__ __forceinline__ uint32_t scan_pick(uint32_t*& h, uint32_t*& part, uint64_t& total, const ScanPair& q,
                                              uint32_t bid) {
  if (bid < q.nb1) return bid;
  h = q.h2;
  part = q.part2;
  total = q.total2;
  return bid - q.nb1;
}

__global__ void __launch_bounds__(NT) k_scan_reduce(uint32_t* h, uint32_t* part, uint64_t total_h,
                                                    const uint64_t* total_dev, ScanPair q) {
  __shared__ uint32_t sh[NT / WAVE + 2];
  uint64_t total = scan_len(total_h, total_dev);
  const uint32_t bid = scan_pick(h, part, total, q, blockIdx.x);
  uint64_t b0 = (uint64_t)bid * SCAN_BLOCK;
  if (b0 >= total) return;
  uint32_t s = 0;
  if (b0 + SCAN_BLOCK <= total) {
    // a whole block: 16-byte loads (every scanned array starts 16-byte aligned)
    const uint4* hv = (const uint4*)(h + b0);
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS / 4; r++) {
      const uint4 v = hv[r * NT + threadIdx.x];
      s += v.x + v.y + v.z + v.w;
    }
  } else {
    for (int r = 0; r < SCAN_ITEMS; r++) {
      uint64_t i = b0 + (uint64_t)r * NT + threadIdx.x;
      if (i < total) s += h[i];
    }
  }
  uint32_t tot;
  block_excl_scan<NT>(s, sh, &tot);
  if (threadIdx.x == 0) part[bid] = tot;
}

__global__ void __launch_bounds__(NT) k_scan_partials(uint32_t* part, uint64_t total_h, const uint64_t* total_dev,
                                                      ScanPair q) {
  __shared__ uint32_t sh[NT / WAVE + 2];
  uint64_t total = scan_len(total_h, total_dev);
  uint32_t* hh = nullptr;
  if (blockIdx.x == 1) scan_pick(hh, part, total, q, q.nb1);
  const uint32_t nb = (uint32_t)((total + SCAN_BLOCK - 1) / SCAN_BLOCK);
  uint32_t run = 0;
  for (uint32_t base = 0; base < nb; base += NT) {
    uint32_t i = base + threadIdx.x;
    uint32_t v = i < nb ? part[i] : 0;
    uint32_t tot;
    uint32_t e = block_excl_scan<NT>(v, sh, &tot);
    if (i < nb) part[i] = run + e;
    run += tot;
  }
}

// self_prefix: part holds the blocks' plain sums (no k_scan_partials
// launch) and each block adds up those before it itself -- for arrays of a
// few thousand blocks at most, whose partials are a few KB read from L2.
__global__ void __launch_bounds__(NT) k_scan_down(uint32_t* h, uint32_t* part, uint64_t total_h,
                                                  const uint64_t* total_dev, ScanPair q, int self_prefix) {
  __shared__ uint32_t sh[NT / WAVE + 2];
  uint64_t total = scan_len(total_h, total_dev);
  const uint32_t bid = scan_pick(h, part, total, q, blockIdx.x);
  uint64_t b0 = (uint64_t)bid * SCAN_BLOCK;
  if (b0 >= total) return;
  uint32_t before;
  if (self_prefix) {
    uint32_t v = 0;
    for (uint32_t j = threadIdx.x; j < bid; j += NT) v += part[j];
    block_excl_scan<NT>(v, sh, &before);
  } else {
    before = part[bid];
  }
  // thread t owns the SCAN_ITEMS consecutive entries starting at b0 + t*SCAN_ITEMS
  static_assert(SCAN_ITEMS == 8, "two 16-byte vectors per thread");
  const bool whole = b0 + SCAN_BLOCK <= total;
  uint32_t v[SCAN_ITEMS];
  uint32_t s = 0;
  if (whole) {
    const uint4* hv = (const uint4*)(h + b0) + 2 * threadIdx.x;
    const uint4 a = hv[0], b = hv[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    for (int k = 0; k < SCAN_ITEMS; k++) {
      uint64_t i = b0 + (uint64_t)threadIdx.x * SCAN_ITEMS + k;
      v[k] = i < total ? h[i] : 0;
    }
  }
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; k++) s += v[k];
  uint32_t tot;
  uint32_t run = block_excl_scan<NT>(s, sh, &tot) + before;
  if (whole) {
    uint32_t o[SCAN_ITEMS];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
      o[k] = run;
      run += v[k];
    }
    uint4* hv = (uint4*)(h + b0) + 2 * threadIdx.x;
    hv[0] = make_uint4(o[0], o[1], o[2], o[3]);
    hv[1] = make_uint4(o[4], o[5], o[6], o[7]);
  } else {
    for (int k = 0; k < SCAN_ITEMS; k++) {
      uint64_t i = b0 + (uint64_t)threadIdx.x * SCAN_ITEMS + k;
      if (i < total) h[i] = run;
      run += v[k];
    }
  }
}

// Stable split (step 4): every key moves to its bucket, keeping input order
// inside each (tile, bucket); tiles keep their order through the offsets.
template <int KW, int VW, int PMAX>
struct ScatterLds {
  using KT = typename KeyOf<KW>::T;
  static constexpr int KS = SplitChunk<KW, VW, PMAX>::KS;
  static constexpr int CH = SplitChunk<KW, VW, PMAX>::CH;
  static constexpr int SLOTS = SortShape<NT, KS>::SLOTS;
  TreeLds<KW, PMAX> tr;
  uint32_t gofs[PMAX];   // next free in-segment position of each bucket
  uint32_t adj[PMAX];    // gofs - first sorted index of the bucket in the chunk
  uint32_t cnt[RadixLds<NT>::CNT_WORDS];
  uint32_t xw[SLOTS];    // (bucket << 16 | chunk index), sorted by bucket
  KT ck[SLOTS];          // the chunk's keys (raw)
  typename std::conditional<VW == 0, char, typename std::conditional<VW == 4, uint32_t, uint64_t>::type>::type
      cv[VW == 0 ? 1 : SLOTS];
  alignas(8) uint64_t red[64];
};

template <int KW, int VW, int PMAX>
__global__ void __launch_bounds__(NT) k_scatter(LevelArgs a) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  using L = ScatterLds<KW, VW, PMAX>;
  constexpr int KS = L::KS;
  constexpr int CH = L::CH;
  constexpr bool HASV = VW != 0;
  __shared__ L sm;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const LevelCtl c = *a.ctl;
  if (tile >= c.total_tiles) return;
  const uint32_t si = find_seg(a.segs, c.nsegs, tile, [](const SegDesc& d) { return (uint64_t)d.tile_off; });
  const SegDesc d = a.segs[si];
  const uint32_t tw = tile - d.tile_off;
  const int t = threadIdx.x;
  sm.tr.load(a.tree, a.tree_tag, d.tree_off, d.p);
  const uint32_t base = a.hist[d.hist_off];
  for (uint32_t b = t; b < d.p; b += NT) sm.gofs[b] = a.hist[d.hist_off + (uint64_t)b * d.ntiles + tw] - base;
  __syncthreads();
  const uint32_t t0 = tw * a.tile;
  const uint32_t t1 = min(t0 + a.tile, d.len);
  const KT* src = (const KT*)a.src + d.beg;
  const VT* vsrc = (const VT*)a.vsrc;
  KT* dst = (KT*)a.dst + d.beg;
  VT* vdst = (VT*)a.vdst;
  VT* cv = (VT*)(void*)sm.cv;
  for (uint32_t c0 = t0; c0 < t1; c0 += CH) {
    const int cn = (int)min((uint32_t)CH, t1 - c0);
    // striped load of the chunk
#pragma unroll
    for (int r = 0; r < KS; r++) {
      int i = r * NT + t;
      if (i < cn) {
        int j = pad_idx<KS>(i);
        sm.ck[j] = to_ord(src[c0 + i], a.kin);
        if constexpr (HASV) {
          if (a.iota) cv[j] = (VT)(c0 + i);
          else cv[j] = vsrc[d.beg + c0 + i];
        }
      }
    }
    __syncthreads();
    // classify blocked items, pack (bucket, chunk index)
    uint32_t w[KS];
    uint32_t lo[KS];
    NoVal nv[KS];
    {
      KT key[KS];
      uint32_t tag[KS], bk[KS];
#pragma unroll
      for (int k = 0; k < KS; k++) {
        int i = t * KS + k;
        key[k] = sm.ck[pad_idx<KS>(i)];   // slots past cn hold stale keys: ignored below
        tag[k] = c0 + i;
      }
      sm.tr.template classify_many<KS>(key, tag, d.lgp, d.p, bk);
#pragma unroll
      for (int k = 0; k < KS; k++) {
        int i = t * KS + k;
        w[k] = (i < cn) ? ((bk[k] << 16) | (uint32_t)i) : ~0u;
      }
    }
    block_radix_sort<NT, KS, uint32_t, false, NoVal>(w, lo, nv, cn, sm.cnt, sm.xw, nullptr, nullptr, sm.red, 16);
    // first element of each bucket's run
    for (int j = t; j < cn; j += NT) {
      uint32_t b = sm.xw[pad_idx<KS>(j)] >> 16;
      uint32_t pb = j ? (sm.xw[pad_idx<KS>(j - 1)] >> 16) : ~0u;
      if (b != pb) sm.adj[b] = sm.gofs[b] - (uint32_t)j;
    }
    __syncthreads();
    for (int j = t; j < cn; j += NT) {
      uint32_t wv = sm.xw[pad_idx<KS>(j)];
      uint32_t b = wv >> 16, i = wv & 0xFFFFu;
      uint32_t pos = sm.adj[b] + (uint32_t)j;
      dst[pos] = sm.ck[pad_idx<KS>(i)];
      if constexpr (HASV) vdst[d.beg + pos] = cv[pad_idx<KS>(i)];
      uint32_t nb = (j + 1 < cn) ? (sm.xw[pad_idx<KS>(j + 1)] >> 16) : ~0u;
      if (b != nb) sm.gofs[b] = pos + 1;
    }
    __syncthreads();
  }
}

// Hand a bucket too large for one work-group to the next level's list, or
// sort it with the one-work-group merge sort when no level is left.
template <int KW, int VW, typename SM>
__device__ __forceinline__ void bucket_overflow(const LevelArgs& a, const SegDesc& d, uint32_t b, uint64_t gb,
                                                uint32_t sz, SM& sm) {
  using KT = typename KeyOf<KW>::T;
  if (a.next_segs) {
    __shared__ uint32_t slot;
    if (threadIdx.x == 0) {
      slot = atomicAdd(&a.next_ctl->nsegs, 1u);
      if (slot < a.next_cap) {
        SegDesc nd = {};
        nd.beg = gb;
        nd.len = sz;
        nd.p = 0;
        nd.seed = derive_seed(d.seed, d.depth + 1, b);
        nd.depth = d.depth + 1;
        nd.parent_bkt = b;
        a.next_segs[slot] = nd;
      } else {
        atomicOr(&a.gctl->status, ST_LIST_FULL);
      }
    }
    __syncthreads();
    if (slot < a.next_cap) return;
  }
  if (threadIdx.x == 0) atomicOr(&a.gctl->status, ST_FALLBACK);
  KT* alt = (a.dst == a.out) ? (KT*)a.tmp : (KT*)a.dst;
  void* valt = (a.dst == a.out) ? a.vtmp : a.vdst;
  sort_big_wg<KW, VW>((const KT*)a.dst, a.vdst, (KT*)a.out, a.vout, alt, valt, gb, sz, 0, 0, a.kout, sm);
}

// ------------------------------------------- keys-only (unstable) paths
//
// With no payload, keys that compare equal have identical bits, so the
// output does not depend on the order equal keys take inside a bucket; only
// bucket membership has to be exact (it is: classification still compares
// key then position).  These kernels therefore place keys with LDS atomics
// instead of a stable ranking.

// Split: every key goes to its bucket's region for this tile.  Each chunk
// of U*NT keys is grouped by bucket in LDS (slots reserved with LDS
// atomics), then every bucket's run is written out contiguously.  Per-bucket
// chunk counters alternate between two sets so a chunk needs three barriers:
// after counting, after the scan, after grouping.
template <int KW, int PMAX>
struct ScatterKeysLds {
  using KT = typename KeyOf<KW>::T;
  using BT = typename std::conditional<(PMAX <= 256), uint8_t, uint16_t>::type;
  static constexpr int CH = SplitU<KW, PMAX>::CH;
  TreeLds<KW, PMAX> tr;
  uint32_t gofs[PMAX];      // before the first chunk: in-segment position of each bucket's run;
                            // then that position - chunk position of the current chunk's run
  uint32_t cur[2][PMAX];    // chunk counts, then cursors (alternating chunks)
  KT sk[CH];                // chunk keys grouped by bucket
  BT sb[CH];                // their buckets
  alignas(8) uint32_t red[32];
};

template <int KW, int PMAX, bool FULL>
__device__ __forceinline__ void split_chunk(const LevelArgs& a, const SegDesc& d, ScatterKeysLds<KW, PMAX>& sm,
                                            const typename KeyOf<KW>::T* src, typename KeyOf<KW>::T* dst,
                                            uint32_t c0, uint32_t cn, int x, bool first) {
  using KT = typename KeyOf<KW>::T;
  using BT = typename ScatterKeysLds<KW, PMAX>::BT;
  constexpr int U = SplitU<KW, PMAX>::U;
  constexpr int CH = SplitU<KW, PMAX>::CH;
  const int t = threadIdx.x;
  KT key[U];
  uint32_t tag[U], b[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    uint32_t i = u * NT + t;
    tag[u] = c0 + i;
    key[u] = (FULL || i < cn) ? to_ord(__builtin_nontemporal_load(&src[c0 + i]), a.kin) : KT(0);
  }
  sm.tr.template classify_many<U>(key, tag, d.lgp, d.p, b);
  // sorted or constant input puts a wave's row of 64 keys into one bucket:
  // then (tested on the first row) each row claims its slots with one
  // atomic instead of 64 on one address
  const bool rows = __ballot(b[0] == __builtin_amdgcn_readfirstlane(b[0])) == __ballot(1);
  if (rows) {
#pragma unroll
    for (int u = 0; u < U; u++)
      if (FULL || (uint32_t)(u * NT + t) < cn) lds_count(sm.cur[x], b[u]);
  } else {
#pragma unroll
    for (int u = 0; u < U; u++)
      if (FULL || (uint32_t)(u * NT + t) < cn) atomicAdd(&sm.cur[x][b[u]], 1u);
  }
  __syncthreads();
  // close the previous chunk's bookkeeping, then chunk starts of this one
  {
    constexpr int PER = (PMAX + NT - 1) / NT;
    const int o = x ^ 1;
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (int j = 0; j < PER; j++) {
      uint32_t bb = t * PER + j;
      v[j] = 0;
      if (bb < d.p) {
        if (!first) {
          sm.gofs[bb] += sm.cur[o][bb];    // (previous delta + previous chunk's end of the run)
          sm.cur[o][bb] = 0;
        }
        v[j] = sm.cur[x][bb];
      }
      sum += v[j];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<NT>(sum, sm.red, &tot);
#pragma unroll
    for (int j = 0; j < PER; j++) {
      uint32_t bb = t * PER + j;
      if (bb < d.p) { sm.cur[x][bb] = run; sm.gofs[bb] -= run; }
      run += v[j];
    }
  }
  __syncthreads();
  if (rows) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (FULL || (uint32_t)(u * NT + t) < cn) {
        uint32_t pos = lds_claim(sm.cur[x], b[u]);
        sm.sk[pos] = key[u];
        sm.sb[pos] = (BT)b[u];
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (FULL || (uint32_t)(u * NT + t) < cn) {
        uint32_t pos = atomicAdd(&sm.cur[x][b[u]], 1u);
        sm.sk[pos] = key[u];
        sm.sb[pos] = (BT)b[u];
      }
    }
  }
  __syncthreads();
  const uint32_t lim = FULL ? (uint32_t)CH : cn;
#pragma unroll 4
  for (uint32_t j = t; j < lim; j += NT) dst[sm.gofs[sm.sb[j]] + j] = sm.sk[j];
}

template <int KW, int PMAX>
__global__ void __launch_bounds__(NT) k_scatter_keys(LevelArgs a) {
  using KT = typename KeyOf<KW>::T;
  using L = ScatterKeysLds<KW, PMAX>;
  constexpr int CH = L::CH;
  __shared__ L sm;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const LevelCtl c = *a.ctl;
  if (tile >= c.total_tiles) return;
  const uint32_t si = find_seg(a.segs, c.nsegs, tile, [](const SegDesc& d) { return (uint64_t)d.tile_off; });
  const SegDesc d = a.segs[si];
  const uint32_t tw = tile - d.tile_off;
  const int t = threadIdx.x;
  sm.tr.load(a.tree, a.tree_tag, d.tree_off, d.p);
  const uint32_t base = a.hist[d.hist_off];
  for (uint32_t b = t; b < d.p; b += NT) {
    sm.gofs[b] = a.hist[d.hist_off + (uint64_t)b * d.ntiles + tw] - base;
    sm.cur[0][b] = 0;
    sm.cur[1][b] = 0;
  }
  __syncthreads();
  const uint32_t t0 = tw * a.tile;
  const uint32_t t1 = min(t0 + a.tile, d.len);
  const KT* src = (const KT*)a.src + d.beg;
  KT* dst = (KT*)a.dst + d.beg;
  uint32_t c0 = t0;
  int x = 0;
  bool first = true;
  for (; c0 + CH <= t1; c0 += CH, x ^= 1, first = false)
    split_chunk<KW, PMAX, true>(a, d, sm, src, dst, c0, CH, x, first);
  if (c0 < t1) split_chunk<KW, PMAX, false>(a, d, sm, src, dst, c0, t1 - c0, x, first);
}

// Bucket sort of one bucket by counting into S value slots: slot(key) =
// (key - min) >> sh is monotone in the key, so ordering the slots and then
// each slot's few keys orders the bucket.  The bucket is read three times
// (min/max, count, place); the re-reads hit L2.  Slot counts are 16-bit,
// two per word.  Returns false (having written nothing) when a slot is too
// crowded; the caller then radix-sorts.
// LDS of the slot sort stays under 80 KB so two work-groups share a CU.
// Rank phase of the slot sorts: placed[0, len) holds the keys grouped by
// slot; bounds(k, s0, s1) gives the range of k's slot.  A key's final
// position = s0 + #{keys of its slot that are smaller, or equal and placed
// earlier}.
template <int KW, int NTH, typename F>
__device__ __forceinline__ void slot_rank_write(const typename KeyOf<KW>::T* placed, uint32_t len,
                                                typename KeyOf<KW>::T* out, int kout, F bounds) {
  using KT = typename KeyOf<KW>::T;
  for (uint32_t i = threadIdx.x; i < len; i += NTH) {
    const KT k = placed[i];
    uint32_t s0, s1;
    bounds(k, s0, s1);
    uint32_t rank = 0;
    if constexpr (KW == 4) {
      // (key, position) as one 64-bit number: smaller, or equal and placed
      // earlier, is one compare; two keys of the slot per step, the second
      // read clamped into the slot and not counted past its end
      const uint64_t me = ((uint64_t)k << 32) | i;
      for (uint32_t j = s0; j < s1; j += 2) {
        const uint32_t j1 = min(j + 1, s1 - 1);
        const uint64_t o0 = ((uint64_t)placed[j] << 32) | j;
        const uint64_t o1 = ((uint64_t)placed[j1] << 32) | j1;
        rank += o0 < me ? 1u : 0u;
        rank += (j + 1 < s1 && o1 < me) ? 1u : 0u;
      }
    } else {
      for (uint32_t j = s0; j < s1; j++) {
        const KT o = placed[j];
        rank += (o < k || (o == k && j < i)) ? 1u : 0u;
      }
    }
    // (streaming store: the output is not read again here, and the bucket's
    // keys, which other rounds re-read, keep their place in L2)
    __builtin_nontemporal_store(from_ord(k, kout), &out[s0 + rank]);
  }
}

// a 16-bit view of 32-bit LDS words (two slot counters per word)
typedef uint16_t __attribute__((may_alias)) u16_alias;

template <int KW> struct SlotCap { static constexpr int C = KW == 4 ? 16128 : 8064; };
constexpr int SLOT_LOG2 = 13;                   // S = 8192 slots
constexpr uint32_t SLOT_MAX_FILL = 48;          // crowded-slot limit

template <int KW, int CAP>
struct SlotLdsT {
  using KT = typename KeyOf<KW>::T;
  static constexpr int C = CAP;
  KT placed[C];
  uint32_t scnt[(1 << SLOT_LOG2) / 2];          // two 16-bit slot counters per word
  alignas(8) uint64_t red[64];
  uint32_t flag;
};
template <int KW>
using SlotLds = SlotLdsT<KW, SlotCap<KW>::C>;

//
// lo_known / hi_known: a bound on the bucket's keys is already known (from
// its splitters: keys of bucket b lie between splitter b's key and splitter
// b+1's key); otherwise it is found with one pass over the bucket.
// NTH threads per work-group, at most CAP keys.
template <int KW, int NTH, int CAP>
__device__ __forceinline__ bool slot_sort(const typename KeyOf<KW>::T* src, typename KeyOf<KW>::T* out, uint64_t beg,
                                          uint32_t len, int kin, int kout, SlotLdsT<KW, CAP>& sm,
                                          bool lo_known = false, typename KeyOf<KW>::T lo = 0, bool hi_known = false,
                                          typename KeyOf<KW>::T hi = 0) {
  using KT = typename KeyOf<KW>::T;
  constexpr int S = 1 << SLOT_LOG2;
  constexpr int W = S / 2;
  const int t = threadIdx.x;
  const KT* in = src + beg;
  // every key of the bucket to fn, eight per thread per step: whole steps
  // load without bounds tests, the last one clamps its index into the bucket
  auto each_key = [&](auto&& fn) {
    uint32_t i0 = 0;
    for (; i0 + 8 * NTH <= len; i0 += 8 * NTH) {
      KT k[8];
#pragma unroll
      for (int u = 0; u < 8; u++) k[u] = to_ord(in[i0 + u * NTH + t], kin);
#pragma unroll
      for (int u = 0; u < 8; u++) fn(k[u]);
    }
    if (i0 < len) {
      KT k[8] = {};
#pragma unroll
      for (int u = 0; u < 8; u++)   // (rows wholly past the end load nothing)
        if (i0 + u * NTH < len) k[u] = to_ord(in[min(i0 + u * NTH + t, len - 1)], kin);
#pragma unroll
      for (int u = 0; u < 8; u++)
        if (i0 + u * NTH + t < len) fn(k[u]);
    }
  };
  KT mn = ~KT(0), mx = 0;
  if (!(lo_known && hi_known))
    each_key([&](KT k) {
      mn = k < mn ? k : mn;
      mx = k > mx ? k : mx;
    });
  for (int q = t; q < W; q += NTH) sm.scnt[q] = 0;
  if (!(lo_known && hi_known)) block_minmax<NTH>(mn, mx, (KT*)sm.red);   // (ends with a barrier)
  else __syncthreads();
  if (lo_known) mn = lo;
  if (hi_known) mx = hi;
  if (mn == mx) {                          // one key value: already sorted
    for (uint32_t i = t; i < len; i += NTH) out[beg + i] = from_ord(mn, kout);
    return true;
  }
  const int bw = bit_width<KT>((KT)(mx - mn));
  const int sh = bw > SLOT_LOG2 ? bw - SLOT_LOG2 : 0;
  auto slot = [&](KT k) { return (uint32_t)((KT)(k - mn) >> sh); };
  each_key([&](KT k) {
    const uint32_t q = slot(k);
    atomicAdd(&sm.scnt[q >> 1], 1u << (16 * (q & 1)));
  });
  __syncthreads();
  // exclusive scan of the slot counts (16-bit halves), and the fullest slot
  {
    constexpr int PER = W / NTH;
    uint32_t v[PER], sum = 0, mxc = 0;
#pragma unroll
    for (int j = 0; j < PER; j++) {
      v[j] = sm.scnt[t * PER + j];
      uint32_t lo = v[j] & 0xFFFFu, hi = v[j] >> 16;
      sum += lo + hi;
      mxc = max(mxc, max(lo, hi));
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<NTH>(sum, (uint32_t*)sm.red, &tot);
    uint32_t wm = wave_max(mxc);
    if (t == 0) sm.flag = 0;
    __syncthreads();
    if (lane_id() == 0 && wm > SLOT_MAX_FILL) atomicOr(&sm.flag, 1u);
#pragma unroll
    for (int j = 0; j < PER; j++) {
      uint32_t lo = v[j] & 0xFFFFu;
      sm.scnt[t * PER + j] = run | ((run + lo) << 16);   // starts of slots 2w and 2w+1
      run += lo + (v[j] >> 16);
    }
  }
  __syncthreads();
  // every thread reads the flag before any thread leaves (the caller reuses
  // this LDS for the radix sort)
  const bool crowded = sm.flag != 0;
  __syncthreads();
  if (crowded) return false;
  // place: afterwards each slot's counter holds the slot's end
  auto place = [&](KT k) {
    const uint32_t q = slot(k);
    const uint32_t sft = 16 * (q & 1);
    const uint32_t old = atomicAdd(&sm.scnt[q >> 1], 1u << sft);
    sm.placed[(old >> sft) & 0xFFFFu] = k;
  };
  each_key(place);
  __syncthreads();
  // order each slot: a key's rank = keys of its slot that are smaller, or
  // equal and placed earlier
  auto slot_end = [&](uint32_t q) -> uint32_t { return ((const u16_alias*)sm.scnt)[q]; };
  slot_rank_write<KW, NTH>(sm.placed, len, out + beg, kout, [&](KT k, uint32_t& s0, uint32_t& s1) {
    const uint32_t q = slot(k);
    const uint32_t e0 = slot_end(q ? q - 1 : 0u);
    s0 = q ? e0 : 0u;
    s1 = slot_end(q);
  });
  __syncthreads();
  return true;
}

// Keys only: slot-sort every bucket that fits; hand the others on.
template <int KW>
__global__ void __launch_bounds__(NT) k_bucket_sort_keys(LevelArgs a, int export_stages) {
  using KT = typename KeyOf<KW>::T;
  __shared__ SlotLds<KW> sm;
  const LevelCtl c = *a.ctl;
  const uint32_t x = blockIdx.x;
  if (x >= c.total_buckets) return;
  const uint32_t si = find_seg(a.segs, c.nsegs, x, [](const SegDesc& d) { return (uint64_t)d.bkt_off; });
  const SegDesc d = a.segs[si];
  const uint32_t b = x - d.bkt_off;
  const uint32_t base = a.hist[d.hist_off];
  const uint32_t st = a.hist[d.hist_off + (uint64_t)b * d.ntiles] - base;
  const uint32_t en = (b + 1 < d.p) ? a.hist[d.hist_off + (uint64_t)(b + 1) * d.ntiles] - base : d.len;
  const uint32_t sz = en - st;
  if (export_stages && d.depth == 0 && si == 0 && threadIdx.x == 0) a.exp_counts[b] = sz;
  if (sz == 0) return;
  const uint64_t gb = d.beg + st;
  // the bucket's key range from its splitters (ranks b and b+1), when both exist
  auto spl_key = [&](uint32_t r) -> KT {          // key of splitter of rank r (1-based)
    uint32_t z = __builtin_ctz(r);
    uint32_t k = (1u << (d.lgp - 1 - z)) + (r >> (z + 1));
    uint64_t node = ((const uint64_t*)a.tree)[d.tree_off + k];
    if constexpr (KW == 4) return (KT)(node >> 32);
    else return (KT)node;
  };
  const bool lo_k = b >= 1, hi_k = b + 1 < d.p;
  const KT lo = lo_k ? spl_key(b) : KT(0);
  const KT hi = hi_k ? spl_key(b + 1) : KT(0);
  if (sz <= (uint32_t)SlotLds<KW>::C &&
      slot_sort<KW, NT, SlotCap<KW>::C>((const KT*)a.dst, (KT*)a.out, gb, sz, 0, a.kout, sm, lo_k, lo, hi_k, hi)) {
    if (threadIdx.x == 0) atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)sz);
    return;
  }
  if (sz > (uint32_t)SlotLds<KW>::C && a.next_segs) {   // larger than the slot sort takes: split it again
    if (threadIdx.x == 0) {
      uint32_t slot = atomicAdd(&a.next_ctl->nsegs, 1u);
      if (slot < a.next_cap) {
        SegDesc nd = {};
        nd.beg = gb;
        nd.len = sz;
        nd.seed = derive_seed(d.seed, d.depth + 1, b);
        nd.depth = d.depth + 1;
        nd.parent_bkt = b;
        a.next_segs[slot] = nd;
      } else {
        atomicOr(&a.gctl->status, ST_LIST_FULL);
        uint32_t k = atomicAdd(a.nleft, 1u);
        a.left[k] = SmallEnt{gb, sz, x};
      }
    }
    return;
  }
  if (threadIdx.x == 0) {
    // (bucket index kept in pad: the next level derives its seed from it)
    uint32_t k = atomicAdd(a.nleft, 1u);
    a.left[k] = SmallEnt{gb, sz, x};
  }
}

// Keys only: buckets handed on by the slot sorts (list 0: by the slot sort,
// list 1: by the round-based one) -- radix sort in LDS, or the next level /
// fallback when larger than one work-group.
template <int KW>
__global__ void __launch_bounds__(NT) k_bucket_leftover_keys(LevelArgs a, int list) {
  using KT = typename KeyOf<KW>::T;
  constexpr uint32_t C = SmallCap<KW, 0>::C;
  __shared__ SmallLds<KW, 0, SmallCap<KW, 0>::KMAX> sm;
  const SmallEnt* left = list ? a.left2 : a.left;
  const uint32_t nl = list ? *a.nleft2 : *a.nleft;
  for (uint32_t li = blockIdx.x; li < nl; li += gridDim.x) {
    const SmallEnt e = left[li];
    if (e.len <= C) {
      sort_small<KW, 0>((const KT*)a.dst, nullptr, (KT*)a.out, nullptr, e.beg, e.len, 0, 0, a.kout, sm);
      continue;
    }
    const LevelCtl c = *a.ctl;
    const uint32_t si = find_seg(a.segs, c.nsegs, e.pad, [](const SegDesc& d) { return (uint64_t)d.bkt_off; });
    const SegDesc d = a.segs[si];
    bucket_overflow<KW, 0>(a, d, e.pad - d.bkt_off, e.beg, e.len, sm);
    __syncthreads();
  }
}

// ------------------------------------------------- entry kernels

// Zero the control block and write the single top-level segment, planned
// (the offsets and totals the level-planning kernel would give one segment
// of n keys split into p buckets over tiles of `tile` keys).
__device__ __forceinline__ void init_single(Ctl* g, SegDesc* segs, uint64_t n, uint32_t p, uint32_t m,
                                            uint32_t stride, uint64_t seed, uint32_t tile) {
  {
    *g = Ctl{};
    SegDesc d = {};
    d.beg = 0;
    d.len = (uint32_t)n;
    d.p = p;
    d.lgp = 31 - __clz(p);
    d.m = m;
    d.stride = stride;
    d.seed = seed;
    d.ntiles = (uint32_t)((n + tile - 1) / tile);
    segs[0] = d;
    LevelCtl& c = g->lv[0];
    c.nsegs = 1;
    c.total_samples = m;
    c.total_tiles = d.ntiles;
    c.total_buckets = p;
    c.total_tree = p;
    c.total_hist = (uint64_t)p * d.ntiles;
    c.max_m = m;
    c.keys = n;
    c.bucket_keys = 0;
  }
}

__global__ void k_init_single(Ctl* g, SegDesc* segs, uint64_t n, uint32_t p, uint32_t m, uint32_t stride,
                              uint64_t seed, uint32_t tile) {
  if (threadIdx.x == 0) init_single(g, segs, n, p, m, stride, seed, tile);
}

__global__ void k_init_ctl(Ctl* g) {
  if (threadIdx.x == 0) *g = Ctl{};
}

// Size classes of the segmented sort below one work-group's capacity:
// segments of up to WAVE keys are sorted by one wave each (many per
// work-group, no LDS), up to MID_CAP keys by a work-group with a small LDS
// footprint (several per CU), the rest by a work-group with the full LDS.
constexpr uint32_t MID_K = 4;
constexpr uint32_t MID_CAP = NT * MID_K;

// Segmented input: segments longer than C go to the top level's list, the
// others to the tiny, mid or small list by length.  A segment that ends
// before it starts, leaves [0, total) or is longer than maxlen (the bound
// the plan was made for) is skipped and flagged.
__global__ void k_seg_init(Ctl* g, const int64_t* off, uint32_t nseg, uint32_t C, SegDesc* top, uint32_t top_cap,
                           SmallEnt* small, SmallEnt* tiny, SmallEnt* mid, uint64_t seed, uint64_t total,
                           uint64_t maxlen) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += gridDim.x * blockDim.x) {
    int64_t b = off[i], e = off[i + 1];
    if (e < b || b < 0 || (uint64_t)e > total || (uint64_t)(e - b) > maxlen) {
      atomicOr(&g->status, ST_BAD_OFFSETS);
      continue;
    }
    uint64_t len = (uint64_t)(e - b);
    if (len == 0) continue;
    if (len <= WAVE) {
      uint32_t s = atomicAdd(&g->ntiny, 1u);
      tiny[s] = SmallEnt{(uint64_t)b, (uint32_t)len, 0};
    } else if (len <= MID_CAP) {
      uint32_t s = atomicAdd(&g->nmid, 1u);
      mid[s] = SmallEnt{(uint64_t)b, (uint32_t)len, 0};
    } else if (len <= C) {
      uint32_t s = atomicAdd(&g->nsmall, 1u);
      small[s] = SmallEnt{(uint64_t)b, (uint32_t)len, 0};
    } else {
      uint32_t s = atomicAdd(&g->lv[0].nsegs, 1u);
      if (s >= top_cap) { atomicOr(&g->status, ST_LIST_FULL); continue; }
      SegDesc d = {};
      d.beg = (uint64_t)b;
      d.len = (uint32_t)len;
      d.p = 0;
      d.seed = derive_seed(seed, 0, i);
      d.depth = 0;
      top[s] = d;
    }
  }
}

template <int KW, int VW>
__global__ void __launch_bounds__(NT) k_sort_small_list(Ctl* g, const SmallEnt* list, const void* src,
                                                        const void* vsrc, void* out, void* vout, int kind,
                                                        int iota, int fb) {
  using KT = typename KeyOf<KW>::T;
  // (fb: the list of segments the stable slot sort handed on)
  if (blockIdx.x >= (fb ? g->nsmall_fb : g->nsmall)) return;
  SmallEnt e = list[blockIdx.x];
  if constexpr (VW == 0) {
    // keys only: the slot sort first (its LDS shares the radix sort's); a
    // crowded segment, or one past its capacity, takes the radix sort
    __shared__ union {
      SmallLds<KW, VW, SmallCap<KW, VW>::KMAX> r;
      SlotLds<KW> q;
    } u;
    if (e.len <= (uint32_t)SlotLds<KW>::C &&
        slot_sort<KW, NT, SlotCap<KW>::C>((const KT*)src, (KT*)out, e.beg, e.len, kind, kind, u.q))
      return;
    __syncthreads();
    sort_small<KW, VW>((const KT*)src, nullptr, (KT*)out, vout, e.beg, e.len, 0, kind, kind, u.r);
  } else {
    __shared__ SmallLds<KW, VW, SmallCap<KW, VW>::KMAX> sm;
    // an iota payload is the index inside the segment (0-based from e.beg)
    sort_small<KW, VW>((const KT*)src, iota ? nullptr : vsrc, (KT*)out, vout, e.beg, e.len, 0, kind, kind, sm);
  }
}

// Segments of WAVE < len <= MID_CAP keys: the same LDS radix sort with
// MID_K keys per thread, whose small LDS lets several work-groups share a CU.
template <int KW, int VW>
__global__ void __launch_bounds__(NT) k_sort_mid_list(Ctl* g, const SmallEnt* list, const void* src,
                                                      const void* vsrc, void* out, void* vout, int kind, int iota) {
  using KT = typename KeyOf<KW>::T;
  __shared__ SmallLds<KW, VW, MID_K> sm;
  const uint32_t nm = g->nmid;
  for (uint32_t li = blockIdx.x; li < nm; li += gridDim.x) {
    const SmallEnt e = list[li];
    if (e.len <= (uint32_t)NT)
      sort_small_k<KW, VW, 1, MID_K>((const KT*)src, iota ? nullptr : vsrc, (KT*)out, vout, e.beg, e.len, 0, kind,
                                     kind, sm);
    else
      sort_small_k<KW, VW, MID_K, MID_K>((const KT*)src, iota ? nullptr : vsrc, (KT*)out, vout, e.beg, e.len, 0,
                                         kind, kind, sm);
  }
}

// Segments of at most WAVE keys: one wave per segment, one item per lane.
// A lane's rank is the number of items whose (key, index) is smaller, read
// lane by lane from the wave (scalar broadcasts, no LDS); every lane then
// writes its key (and payload) at its rank, which is the stable order.
template <int KW, int VW>
__global__ void __launch_bounds__(NT) k_sort_tiny_list(Ctl* g, const SmallEnt* list, const void* src,
                                                       const void* vsrc, void* out, void* vout, int kind, int iota) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  const uint32_t nt = g->ntiny;
  const int l = lane_id();
  for (uint32_t w = blockIdx.x * (NT / WAVE) + wave_id(); w < nt; w += gridDim.x * (NT / WAVE)) {
    const SmallEnt e = list[w];
    const uint32_t len = e.len;
    const bool in = (uint32_t)l < len;
    const KT key = in ? ((const KT*)src)[e.beg + l] : KT(0);
    const KT o = in ? to_ord(key, kind) : ~KT(0);
    uint32_t rank = 0;
#pragma unroll
    for (int j = 0; j < WAVE; j++) {
      if ((uint32_t)j >= len) break;   // (uniform across the wave)
      KT oj;
      if constexpr (KW == 4) {
        oj = (KT)__builtin_amdgcn_readlane((int)o, j);
      } else {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)o, j);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(o >> 32), j);
        oj = ((KT)hi << 32) | lo;
      }
      rank += (oj < o || (oj == o && j < l)) ? 1u : 0u;
    }
    if (in) {
      ((KT*)out)[e.beg + rank] = key;
      if constexpr (VW != 0) {
        const VT v = (iota || !vsrc) ? (VT)l : ((const VT*)vsrc)[e.beg + l];
        ((VT*)vout)[e.beg + rank] = v;
      }
    }
  }
}

template <int KW, int VW>
__global__ void __launch_bounds__(NT) k_sort_direct(const void* src, const void* vsrc, void* out, void* vout,
                                                    uint64_t beg, uint32_t len, int kind) {
  using KT = typename KeyOf<KW>::T;
  __shared__ SmallLds<KW, VW, SmallCap<KW, VW>::KMAX> sm;
  sort_small<KW, VW>((const KT*)src, vsrc, (KT*)out, vout, beg, len, 0, kind, kind, sm);
}

// One work-group sorts the whole array (used only when no p >= 2 meets the
// preconditions and the array exceeds one work-group).
template <int KW, int VW>
__global__ void __launch_bounds__(NT) k_sort_whole(const void* src, const void* vsrc, void* out, void* vout,
                                                   void* tmp, void* vtmp, uint64_t n, int kind) {
  using KT = typename KeyOf<KW>::T;
  __shared__ SmallLds<KW, VW, SmallCap<KW, VW>::KMAX> sm;
  sort_big_wg<KW, VW>((const KT*)src, vsrc, (KT*)out, vout, (KT*)tmp, vtmp, 0, n, 0, kind, kind, sm);
}

// Block bounds of regular sampling: block k = [floor(k n/p), floor((k+1) n/p)).
__global__ void k_block_offsets(int64_t* off, uint64_t n, uint32_t p) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k <= p; k += gridDim.x * blockDim.x)
    off[k] = (int64_t)(((uint64_t)k * n) / p);
}

// Backward of a row-wise sort: grad_x[r, perm[r, j]] = grad_y[r, j].
// Work-group w handles GRAD_V * 256 consecutive elements of one row: the
// grid is rows x chunks tiles, numbered row-major and mapped to work-groups
// so that each XCD takes a contiguous range of tiles (whole rows), which
// keeps every row's scattered writes in one XCD's L2, where they fill whole
// lines before they are written back.  Each thread loads GRAD_V gradients
// and GRAD_V indices with vector loads.  An index outside [0, cols) is not
// written and raises the library's gradient status flag (the rest of the
// row is still scattered).
constexpr int GRAD_V = 4;
constexpr int GRAD_NT = 256;

template <typename T>
__global__ void __launch_bounds__(GRAD_NT) k_scatter_grad(const T* gy, const int64_t* perm, T* gx, uint32_t rows,
                                                          uint32_t cols, uint32_t chunks, uint32_t* status) {
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint32_t r = tile / chunks, ch = tile - r * chunks;
  if (r >= rows) return;
  const uint32_t j0 = ch * (GRAD_V * GRAD_NT) + threadIdx.x * GRAD_V;
  if (j0 >= cols) return;
  const uint64_t base = (uint64_t)r * cols;
  const T* g = gy + base;
  const int64_t* pr = perm + base;
  T* out = gx + base;
  T v[GRAD_V];
  int64_t q[GRAD_V];
  // (a row of cols % GRAD_V != 0 ends unaligned: scalar loads at its end)
  if (j0 + GRAD_V <= cols && (cols % GRAD_V) == 0) {
    // GRAD_V gradients: 8, 16 or 32 bytes, aligned to their size (the row
    // length is a multiple of GRAD_V and grad_y is 16-byte aligned)
    if constexpr (sizeof(T) * GRAD_V == 8) {
      const uint2 w = *(const uint2*)(g + j0);
      __builtin_memcpy(v, &w, sizeof v);
    } else {
      constexpr int NV = sizeof(T) * GRAD_V / 16;
      uint4 w[NV];
#pragma unroll
      for (int k = 0; k < NV; k++) w[k] = ((const uint4*)(g + j0))[k];
      __builtin_memcpy(v, w, sizeof v);
    }
    const uint4* pv = (const uint4*)(pr + j0);
    uint4 pp[GRAD_V / 2];
#pragma unroll
    for (int k = 0; k < GRAD_V / 2; k++) pp[k] = pv[k];
    __builtin_memcpy(q, pp, sizeof q);
#pragma unroll
    for (int k = 0; k < GRAD_V; k++) {
      if ((uint64_t)q[k] < cols) out[q[k]] = v[k];
      else atomicOr(status, 1u);
    }
  } else {
    for (uint32_t j = j0; j < min(j0 + GRAD_V, cols); j++) {
      const int64_t pj = pr[j];
      if ((uint64_t)pj < cols) out[pj] = g[j];
      else atomicOr(status, 1u);
    }
  }
}

}  // namespace ss
