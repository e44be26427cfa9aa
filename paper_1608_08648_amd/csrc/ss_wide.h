// Wide split: keys-only sort of 4-byte keys with many buckets (p >= 1024).
//
// One sample, its p-1 splitters and the (key, position) classification of
// step 4 (ties between equal keys broken by the input position, Section
// 2.2), exactly as in the level kernels.  What differs is how the keys move:
// writing every tile straight into p buckets would leave runs of a few keys
// per bucket, so the keys travel in two passes of long runs instead:
//
//   k_wide_table    sorted splitter keys and a cell table over their range
//   k_wide_count    per tile: the fine bucket of every key (cell table and a
//                   short binary search), non-tie counts per (bucket, tile),
//                   tie counts per bucket; one byte per key for the first
//                   pass: its coarse region, or 0xFF for a tie key
//   k_scan_*        exclusive scans of both count arrays
//   k_wide_split_a  per tile: non-tie keys to P1 = 64 coarse regions (a
//                   coarse bucket is P2 = p / 64 consecutive fine buckets),
//                   read from the classification's bytes
//   k_wide_split_b  per piece of a coarse region: keys to their fine buckets
//                   (walk of the region's own subtree on the key alone)
//   k_wide_bucket   per fine bucket: fill the tie runs, sort the rest in LDS
//
// A tie key is a key equal to the key of one of its bucket's two splitters.
// Every other key differs from all p-1 splitter keys (the splitters are
// sorted, so any splitter key equal to it would bound its bucket), so for it
// the comparison with a splitter is decided by the key alone and the second
// pass needs no position.  Tie keys are never moved: a key equal to the
// lower splitter's key is no larger than any other key of its bucket, one
// equal to the upper splitter's key no smaller, so the bucket sort writes
// them as runs of that key at the bucket's two ends.  Bucket contents, and
// hence the output, are those of the one-pass split.
//
// Layout of the fine counts: bucket b owns R = W + 2 entries,
//   [b*R]          keys equal to the lower splitter's key (tie-low)
//   [b*R + 1 + w]  non-tie keys of input tile w
//   [b*R + W + 1]  keys equal to the upper splitter's key (tie-high)
// plus one last entry (0) so that, scanned, it holds n.  After the scan
// every entry is a final output position: bucket b starts at [b*R], its
// non-tie keys from tile w go to [b*R + 1 + w] onwards.
#pragma once
#include "ss_kernels.h"

namespace ss {

constexpr int WIDE_LG1 = 6;
constexpr uint32_t WIDE_P1 = 1u << WIDE_LG1;   // coarse buckets
constexpr int WIDE_PMAX = 4096;
constexpr int WIDE_U = 16;                     // keys per thread per chunk
constexpr int WIDE_CH = WIDE_U * NT;
constexpr int WIDE_UA = 8;                      // keys per thread per chunk of the second pass (LDS)
constexpr uint32_t WIDE_TILE = 7 * WIDE_U * 512; // keys per input tile (< 2^16: 16-bit tie counters)
constexpr uint32_t WIDE_TB = 24576;            // nominal keys per piece of the second pass (small pieces: the
                                               // work-groups finish together)
// bucket sort of the wide split: 1024 threads, 30720 keys per round in LDS
// (one work-group per CU), buckets of up to 65535 keys
constexpr int WIDE_BNT = 1024;
constexpr int WIDE_BCAP = 30720;
// The bucket sorts of the wide split and of sort-first come in two LDS
// layouts: 30720 keys a round over 2^14 slots (one work-group per CU), or
// 16000 keys a round over 2^13 slots (two work-groups share a CU, under 80 KB
// of LDS each).  The second is faster while the buckets take one or two
// rounds; each further round re-reads the whole bucket, so large or uneven
// buckets take the first: the second is chosen for a mean bucket of up to
// 32K keys with an oversampling ratio s >= 16, or up to 16K keys with s >= 8
// (the largest buckets grow with the mean and shrink with s).
constexpr int WIDE_SCAP = 16000;
constexpr int WIDE_SLG = 13;
inline bool wide_small_rounds(uint64_t n, uint32_t p, uint32_t s) {
  return (s >= 16 && n <= 32768ull * p) || (s >= 8 && n <= 16384ull * p);
}
constexpr uint32_t WIDE_BMAX = 65535;          // largest bucket the round-based slot sort takes
// expected largest bucket up to which the wide split sorts every bucket in
// rounds; above it a level below takes the buckets past WIDE_BMAX (on 2^26
// int32 keys with p = 1024 the rounds win at an estimate of 2^17 keys and
// lose at 1.2 * 2^17 and more)
constexpr uint32_t WIDE_LEVEL_MIN = 1u << 17;

struct WideHdr { uint32_t kmin, kmax, sh, ncell; };

struct WideArgs {
  const uint64_t* tree;   // Eytzinger tree, slot k in [1, p): (ord << 32) | tag
  uint32_t* hf;           // fine counts, p * (W + 2) + 1 entries, scanned in place
  uint32_t* ha;           // coarse non-tie counts, P1 * W + 1 entries (c-major), scanned in place
  const void* src;        // the caller's keys
  uint32_t* stage;        // coarse regions (ord images)
  uint32_t* fine;         // fine buckets (ord images)
  void* out;              // output (caller's key type)
  uint32_t* skeys;        // sorted splitter keys, rank 1..p-1 (entry 0 unused)
  uint32_t* stags;        // their tags
  uint32_t* cells;        // cell table
  WideHdr* hdr;
  uint8_t* cb;            // per key: its coarse region, 0xFF for a tie key (not moved)
  uint32_t n, p, lgp, W, tile;
  int kin, kout;
};

// Classification without a tree walk.  The sorted splitter keys are cut
// into cells of equal key range: cell j of the range [kmin, kmax] of the
// splitter keys covers keys kmin + [j << sh, (j + 1) << sh), and cells[j]
// packs L_j | U_j << 16 with L_j = #{splitters whose key < the cell's first
// key} and U_j = L_{j+1}.  A key in cell j has between L_j and U_j
// splitters below it; a binary search over those few candidates (about p
// / cells of them for evenly spread keys) finds the count.
constexpr int WIDE_CELL_BITS = 13;
constexpr int WIDE_CELLS = 1 << WIDE_CELL_BITS;   // (plus one sentinel cell past the range)
constexpr int WIDE_TABLE_WG = 8;                 // work-groups building the table

// One work-group: the sorted splitters (rank r in [1, p): key and tag) from
// the Eytzinger tree, and the cell table.
// (every work-group of the launch builds the sorted keys in LDS and takes
// its share of the tie entries and the cells; work-group 0 writes the rest)
__global__ void __launch_bounds__(NT) k_wide_table(WideArgs w) {
  __shared__ uint32_t sk[WIDE_PMAX];
  __shared__ uint16_t Ls[WIDE_CELLS + 2];
  const uint32_t p = w.p;
  const uint32_t g0 = blockIdx.x * NT + threadIdx.x, gs = gridDim.x * NT;
  // tie entries and the trailing totals of both count arrays start at zero
  // (the count kernel adds to them; it writes every other entry)
  {
    const uint32_t R = w.W + 2;
    for (uint32_t b = g0; b < p; b += gs) {
      w.hf[(uint64_t)b * R] = 0;
      w.hf[(uint64_t)b * R + R - 1] = 0;
    }
    if (g0 == 0) {
      w.hf[(uint64_t)p * R] = 0;
      w.ha[(uint64_t)WIDE_P1 * w.W] = 0;
    }
  }
  {
    // splitter of rank r from its tree slot (every load issued first)
    constexpr int R = WIDE_PMAX / NT;
    uint64_t nd[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
      const uint32_t r = q * NT + threadIdx.x + 1;
      uint32_t k = 1;
      if (r < p) {
        const uint32_t z = __builtin_ctz(r);
        k = (1u << (w.lgp - 1 - z)) + (r >> (z + 1));
      }
      nd[q] = r < p ? w.tree[k] : 0ull;
    }
#pragma unroll
    for (int q = 0; q < R; q++) {
      const uint32_t r = q * NT + threadIdx.x + 1;
      if (r < p) {
        sk[r] = (uint32_t)(nd[q] >> 32);
        if (blockIdx.x == 0) {
          w.skeys[r] = (uint32_t)(nd[q] >> 32);
          w.stags[r] = (uint32_t)nd[q];
        }
      }
    }
  }
  __syncthreads();
  const uint32_t kmin = sk[1], kmax = sk[p - 1];
  const int bw = bit_width<uint32_t>(kmax - kmin);
  const uint32_t sh = bw > WIDE_CELL_BITS ? (uint32_t)(bw - WIDE_CELL_BITS) : 0u;
  const uint32_t ncell = ((kmax - kmin) >> sh) + 1;
  // L(j) = #{r : sk[r] < kmin + (j << sh)} = #{r : cell(r) < j}, cell(r) =
  // (sk[r] - kmin) >> sh non-decreasing in r: splitter r sets L(j) = r - 1
  // on the cells (cell(r-1), cell(r)] (cell(0) = -1; r = p covers the rest
  // up to ncell + 1).  Cell ncell, past kmax, is the sentinel: every
  // splitter below.
  auto cell_of = [&](uint32_t r) -> int64_t {
    if (r == 0) return -1;
    if (r >= p) return (int64_t)ncell + 1;
    return (int64_t)((sk[r] - kmin) >> sh);
  };
  for (uint32_t r = threadIdx.x + 1; r <= p; r += NT) {
    const int64_t c0 = cell_of(r - 1), c1 = cell_of(r);
    for (int64_t j = c0 + 1; j <= c1; j++) Ls[j] = (uint16_t)(r - 1);
  }
  __syncthreads();
  for (uint32_t j = g0; j <= ncell; j += gs) w.cells[j] = (uint32_t)Ls[j] | ((uint32_t)Ls[j + 1] << 16);
  if (g0 == 0) *w.hdr = WideHdr{kmin, kmax, sh, ncell};
}

// Search of one key among the candidates of its cell, on the key alone:
// lo - 1 = #{splitters whose key < key}; tie = some splitter has this key
// (then it is splitter lo: the first with key >= key is always compared).
__device__ __forceinline__ uint32_t wide_lower(const uint32_t* sk, const uint32_t* cells, const WideHdr& h,
                                               uint32_t p, uint32_t key, bool& tie) {
  tie = false;
  if (key < h.kmin) return 1;
  if (key > h.kmax) return p;
  const uint32_t cell = cells[(key - h.kmin) >> h.sh];
  uint32_t lo = (cell & 0xFFFFu) + 1, len = (cell >> 16) - (cell & 0xFFFFu);
  if (len > 4) {
    // many candidates (runs of equal splitter keys): the first one settles
    // keys below all of them and keys equal to it at once
    const uint32_t v0 = sk[lo];
    if (v0 >= key) {
      tie = v0 == key;
      return lo;
    }
    lo++;
    len--;
  }
  uint32_t hk = ~key;
  while (len) {
    const uint32_t half = len >> 1, m = lo + half, v = sk[m];
    if (v < key) {
      lo = m + 1;
      len -= half + 1;
    } else {
      len = half;
      hk = v;
    }
  }
  tie = hk == key;
  return lo;
}

// Full classification of step 4 for a tie key (splitter lo has its key):
// b = (lo - 1) + #{r >= lo : (sk[r], st[r]) < (key, tag)}; tie-low when
// splitter b has the key, else tie-high (splitter b + 1 = lo has it).
__device__ __forceinline__ uint32_t wide_tie_bucket(const uint32_t* sk, const uint32_t* st, uint32_t p, uint32_t lo,
                                                    uint32_t up, uint32_t key, uint32_t tag, uint32_t& kind) {
  uint32_t a = lo, z = up + 1;              // first r in [lo, up + 1) with (sk, st)[r] >= (key, tag)
  (void)p;
  while (a < z) {
    const uint32_t m = (a + z) / 2;
    if (sk[m] == key && st[m] < tag) a = m + 1;
    else z = m;
  }
  kind = a > lo ? 1u : 2u;
  return a - 1;
}

// keys of one chunk, issued ahead of their use (prefetch into registers);
// streaming loads: each key is read once per pass, so they need not stay in
// L2, where the pass's tables and counts live
template <int U, int NTH = NT>
__device__ __forceinline__ void wide_load(uint32_t (&k)[U], const uint32_t* src, uint32_t i0, uint32_t end) {
  const int t = threadIdx.x;
  if (i0 + U * NTH <= end) {
#pragma unroll
    for (int u = 0; u < U; u++) k[u] = __builtin_nontemporal_load(&src[i0 + u * NTH + t]);
  } else {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t i = i0 + u * NTH + t;
      k[u] = i < end ? __builtin_nontemporal_load(&src[i]) : 0u;
    }
  }
}

// The coarse-region bytes of a chunk of 8 x 1024 keys: thread t's eight
// keys (chunk positions u * 1024 + t) have theirs in one 8-byte word, the
// chunk's word t, byte u (0xFF: a tie key, or past the end).  The
// classification and the first split pass share that key-to-thread map.
constexpr int CB_U = 8, CB_NT = 1024;
__device__ __forceinline__ uint64_t wide_cb_word(const uint8_t* cb, uint32_t i0) {
  return ((const uint64_t*)cb)[(i0 >> 3) + threadIdx.x];
}

struct WideCountLds {
  uint32_t sk[WIDE_PMAX + 2];    // sorted splitter keys (rank 1..p-1), then two all-ones sentinels
  uint32_t cells[WIDE_CELLS + 1];
  uint32_t cnt[WIDE_PMAX / 2];   // non-tie keys per fine bucket, two 16-bit counts per word
  uint32_t ties[WIDE_PMAX];      // tie-low | tie-high << 16 (a tile holds < 2^16 keys)
  uint32_t csum[WIDE_P1];
};

// Per tile: classify every key (step 4) and count.
//
// The common case is branch-free: a cell holds at most two splitter keys
// for nearly every key (2^13 cells over the splitters' range), so the
// key's count of splitters below it is L + [c1 < key] + [c2 < key] with
// c1, c2 the next two splitter keys after the cell's first L.  Reading them
// past the cell's last candidate is harmless: the next splitter's key lies
// in a later cell, so above the key, and two all-ones sentinels follow the
// last splitter.  The LDS reads of a thread's WIDE_U keys are issued
// together.  Keys of crowded cells (more than two candidates) and tie keys
// (equal to a splitter's key, which need the position) take the slower
// exact paths, entered once per row of a wave that holds any.  (Two
// work-groups per CU: 74 KB of LDS each.)
// (1024 threads, eight keys each per chunk, at most 64 VGPRs: eight waves
// per SIMD with two work-groups per CU)
constexpr int CNT_NT = 1024, CNT_U = 8, CNT_CH = CNT_NT * CNT_U;
static_assert(CNT_CH * 7 == (int)WIDE_TILE, "a tile is seven chunks");
template <int KIND>
__global__ void __launch_bounds__(CNT_NT, 8) k_wide_count(WideArgs w) {
  __shared__ WideCountLds sm;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= w.W) return;
  const int t = threadIdx.x;
  const uint32_t p = w.p, lg2 = w.lgp - WIDE_LG1;
  const uint32_t t0 = tile * w.tile, t1 = min(t0 + w.tile, w.n);
  const uint32_t* src = (const uint32_t*)w.src;
  uint32_t nk[CNT_U];
  wide_load<CNT_U, CNT_NT>(nk, src, t0, t1);
  const uint32_t* stg = w.stags;   // tags: only tie keys read them (from L2)
  // the splitter keys and the cell table: every load issued before the
  // first LDS store (one round trip, not one per loop step)
  {
    constexpr int RS = WIDE_PMAX / CNT_NT, RC = (WIDE_CELLS + 1 + CNT_NT - 1) / CNT_NT;
    const WideHdr h0 = *w.hdr;
    uint32_t vs[RS], vc[RC];
#pragma unroll
    for (int r = 0; r < RS; r++) {
      const uint32_t k = r * CNT_NT + t;
      vs[r] = k < p ? w.skeys[k] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RC; r++) {
      const uint32_t j = r * CNT_NT + t;
      vc[r] = j <= h0.ncell ? w.cells[j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RS; r++) {
      const uint32_t k = r * CNT_NT + t;
      if (k < p) {
        sm.sk[k] = vs[r];
        sm.ties[k] = 0;
      }
      if (k < p / 2) sm.cnt[k] = 0;
    }
#pragma unroll
    for (int r = 0; r < RC; r++) {
      const uint32_t j = r * CNT_NT + t;
      if (j <= h0.ncell) sm.cells[j] = vc[r];
    }
  }
  if (t < 2) sm.sk[p + t] = ~0u;
  const WideHdr h = *w.hdr;
  if (t < (int)WIDE_P1) sm.csum[t] = 0;
  __syncthreads();
  uint32_t hint = ~0u;               // bucket of this thread's previous tie key
  const uint64_t all = __ballot(1);
  static_assert(CNT_U == CB_U && CNT_NT == CB_NT, "the coarse-byte word layout");
  for (uint32_t i0 = t0; i0 < t1; i0 += CNT_CH) {
    uint32_t key[CNT_U], cv[CNT_U], c1[CNT_U], c2[CNT_U];
    uint64_t cbw = 0;                // this thread's coarse-region bytes of the chunk
#pragma unroll
    for (int u = 0; u < CNT_U; u++) key[u] = to_ord(nk[u], KIND);
    if (i0 + CNT_CH < t1) wide_load<CNT_U, CNT_NT>(nk, src, i0 + CNT_CH, t1);
    // cell of every key (below the range: cell 0; above it: the sentinel
    // cell, whose first count is p - 1)
#pragma unroll
    for (int u = 0; u < CNT_U; u++) {
      const uint32_t d = max(key[u], h.kmin) - h.kmin;
      cv[u] = sm.cells[min(d >> h.sh, h.ncell)];
    }
#pragma unroll
    for (int u = 0; u < CNT_U; u++) {
      const uint32_t L = cv[u] & 0xFFFFu;
      c1[u] = sm.sk[L + 1];
      c2[u] = sm.sk[L + 2];
    }
#pragma unroll
    for (int u = 0; u < CNT_U; u++) {
      const uint32_t i = i0 + u * CNT_NT + t;
      const bool valid = i < t1;
      const uint32_t k = key[u];
      const uint32_t L = cv[u] & 0xFFFFu, len = (cv[u] >> 16) - L;
      uint32_t b = L + (c1[u] < k ? 1u : 0u) + (c2[u] < k ? 1u : 0u);   // splitters below the key
      bool tie = (c1[u] == k && len >= 1) || (c2[u] == k && len >= 2);
      if (__ballot(valid && len > 2)) {
        if (valid && len > 2) b = wide_lower(sm.sk, sm.cells, h, p, k, tie) - 1;
      }
      uint32_t kind = 0;
      if (__ballot(valid && tie)) {
        if (valid && tie) {
          // equal keys in input order mostly share a bucket: try the last one
          const uint32_t lo = b + 1;   // the first splitter with key >= k (it has key k)
          const uint32_t hb = hint;
          bool hit = false;
          if (hb != ~0u && hb + 1 >= lo) {
            const bool above = hb == 0 || sm.sk[hb] < k || (sm.sk[hb] == k && stg[hb] < i);
            const bool below = hb + 1 == p || k < sm.sk[hb + 1] || (k == sm.sk[hb + 1] && i < stg[hb + 1]);
            hit = above && below;
          }
          if (hit) {
            b = hb;
            kind = (hb > 0 && sm.sk[hb] == k) ? 1u : 2u;
          } else {
            // every splitter with this key lies in the key's cell: [lo, up]
            const uint32_t up = sm.cells[(k - h.kmin) >> h.sh] >> 16;
            b = wide_tie_bucket(sm.sk, stg, p, lo, up, k, i, kind);
          }
          hint = b;
        }
      }
      cbw |= (uint64_t)((valid && !tie) ? (b >> lg2) : 0xFFu) << (8 * u);
      // count: one atomic for a row of one (kind, bucket) (sorted or
      // constant input), else one per key
      const uint32_t idx = (kind << 16) | b;
      const uint32_t f = __builtin_amdgcn_readfirstlane(idx);
      if (__ballot(valid && idx == f) == all) {
        if (t % WAVE == 0) {
          const uint32_t run = (uint32_t)__popcll(all);
          if (kind == 0) atomicAdd(&sm.cnt[b >> 1], run << (16 * (b & 1)));
          else atomicAdd(&sm.ties[b], kind == 1 ? run : run << 16);
        }
      } else if (valid) {
        if (kind == 0) atomicAdd(&sm.cnt[b >> 1], 1u << (16 * (b & 1)));
        else atomicAdd(&sm.ties[b], kind == 1 ? 1u : 1u << 16);
      }
    }
    ((uint64_t*)w.cb)[(i0 >> 3) + t] = cbw;
  }
  __syncthreads();
  const uint32_t R = w.W + 2;
  for (uint32_t b = t; b < p; b += CNT_NT) {
    w.hf[(uint64_t)b * R + 1 + tile] = (sm.cnt[b >> 1] >> (16 * (b & 1))) & 0xFFFFu;
    const uint32_t tl = sm.ties[b] & 0xFFFFu, th = sm.ties[b] >> 16;
    if (tl) atomicAdd(&w.hf[(uint64_t)b * R], tl);
    if (th) atomicAdd(&w.hf[(uint64_t)b * R + R - 1], th);
  }
  // non-tie keys per coarse bucket: each thread sums p / CNT_NT consecutive
  // fine counts (all inside one coarse bucket, as p / CNT_NT <= p / P1)
  {
    const uint32_t K = p / CNT_NT, P2 = p >> WIDE_LG1;
    uint32_t s = 0;
    for (uint32_t j = 0; j < K; j++) {
      const uint32_t b = t * K + j;
      s += (sm.cnt[b >> 1] >> (16 * (b & 1))) & 0xFFFFu;
    }
    if (s) atomicAdd(&sm.csum[(t * K) / P2], s);
  }
  __syncthreads();
  if (t < (int)WIDE_P1) w.ha[(uint64_t)t * w.W + tile] = sm.csum[t];
}

// Grouping of one chunk by bucket in LDS, then contiguous run writes:
// shared by both passes (NB buckets; bucket ~0u = key not moved).
template <int NB, int U = WIDE_U, int NTH = NT>
struct WideSplitLds {
  uint32_t gofs[NB];       // before the first chunk: output position of each bucket's run;
                           // then output position - chunk position of the current chunk's run
  uint32_t cur[2][NB];     // chunk counts, then cursors (alternating chunks)
  uint32_t ctot[2];        // keys of the chunk that move
  uint32_t sk[U * NTH];
  uint8_t sb[U * NTH];
};

template <int NB, int U, int NTH>
__device__ __forceinline__ void wide_group_write(WideSplitLds<NB, U, NTH>& sm, const uint32_t (&key)[U],
                                                 const uint32_t (&bk)[U], uint32_t* dst, int x, bool first) {
  const int t = threadIdx.x;
  // sorted or constant input puts a wave's row of 64 keys into one bucket:
  // then (tested on the first row) each row claims its slots with one
  // atomic instead of 64 on one address
  const bool rows = __ballot(bk[0] == __builtin_amdgcn_readfirstlane(bk[0])) == __ballot(1);
  if (rows) {
#pragma unroll
    for (int u = 0; u < U; u++)
      if (bk[u] != ~0u) lds_count(sm.cur[x], bk[u]);
  } else {
#pragma unroll
    for (int u = 0; u < U; u++)
      if (bk[u] != ~0u) atomicAdd(&sm.cur[x][bk[u]], 1u);
  }
  __syncthreads();
  // close the previous chunk's bookkeeping, then chunk starts of this one
  // (NB <= 64: one wave)
  if (t < NB) {
    const int o = x ^ 1;
    uint32_t g = sm.gofs[t];               // output position of the bucket's next run
    if (!first) {
      g += sm.cur[o][t];                   // (previous delta + previous chunk's end of the run)
      sm.cur[o][t] = 0;
    }
    const uint32_t v = sm.cur[x][t];
    const uint32_t inc = wave_incl_scan(v);
    sm.cur[x][t] = inc - v;
    sm.gofs[t] = g - (inc - v);
    if (t == NB - 1) sm.ctot[x] = inc;
  }
  __syncthreads();
  if (rows) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (bk[u] != ~0u) {
        const uint32_t pos = lds_claim(sm.cur[x], bk[u]);
        sm.sk[pos] = key[u];
        sm.sb[pos] = (uint8_t)bk[u];
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (bk[u] != ~0u) {
        const uint32_t pos = atomicAdd(&sm.cur[x][bk[u]], 1u);
        sm.sk[pos] = key[u];
        sm.sb[pos] = (uint8_t)bk[u];
      }
    }
  }
  __syncthreads();
  const uint32_t tot = sm.ctot[x];
#pragma unroll 4
  for (uint32_t j = t; j < tot; j += NTH) dst[sm.gofs[sm.sb[j]] + j] = sm.sk[j];
}

// (the first pass: 1024 threads, eight keys each per chunk, at most 64
// VGPRs: eight waves per SIMD with two work-groups per CU)
constexpr int SA_NT = 1024, SA_U = 8;
struct WideALds {
  WideSplitLds<WIDE_P1, SA_U, SA_NT> g;
};

// First pass, per input tile: non-tie keys to their coarse region, in runs.
// The region comes from the classification's byte per key (the fine bucket's
// top bits; 0xFF: a tie key, which stays where it is), so the keys are not
// searched again.
__global__ void __launch_bounds__(SA_NT, 8) k_wide_split_a(WideArgs w) {
  __shared__ WideALds sm;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= w.W) return;
  const int t = threadIdx.x;
  const uint32_t t0 = tile * w.tile, t1 = min(t0 + w.tile, w.n);
  const uint32_t* src = (const uint32_t*)w.src;
  static_assert(SA_U == CB_U && SA_NT == CB_NT, "the coarse-byte word layout");
  uint32_t nk[SA_U];
  wide_load<SA_U, SA_NT>(nk, src, t0, t1);
  uint64_t nbw = wide_cb_word(w.cb, t0);
  if (t < (int)WIDE_P1) {
    sm.g.gofs[t] = w.ha[(uint64_t)t * w.W + tile];
    sm.g.cur[0][t] = 0;
    sm.g.cur[1][t] = 0;
  }
  __syncthreads();
  int x = 0;
  for (uint32_t i0 = t0; i0 < t1; i0 += SA_U * SA_NT, x ^= 1) {
    uint32_t key[SA_U], c[SA_U];
#pragma unroll
    for (int u = 0; u < SA_U; u++) key[u] = to_ord(nk[u], w.kin);
#pragma unroll
    for (int u = 0; u < SA_U; u++) {
      const uint32_t nb = (uint32_t)(nbw >> (8 * u)) & 0xFFu;
      c[u] = (i0 + u * SA_NT + t < t1 && nb != 0xFFu) ? nb : ~0u;
    }
    if (i0 + SA_U * SA_NT < t1) {
      wide_load<SA_U, SA_NT>(nk, src, i0 + SA_U * SA_NT, t1);
      nbw = wide_cb_word(w.cb, i0 + SA_U * SA_NT);
    }
    wide_group_write(sm.g, key, c, w.stage, x, i0 == t0);
  }
}

struct WideBLds {
  uint32_t sub[64];        // the coarse bucket's subtree (keys), local Eytzinger slots [1, P2)
  uint32_t info[4];
  WideSplitLds<64, WIDE_UA> g;
};

// Second pass.  Coarse region c is cut into pieces at input-tile
// boundaries: piece j holds the runs of the input tiles whose run starts in
// [j*TB, (j+1)*TB) of the region, so its keys of fine bucket b go to the
// scanned position of (b, first tile of the piece) onwards.
__global__ void __launch_bounds__(NT) k_wide_split_b(WideArgs w) {
  __shared__ WideBLds sm;
  const int t = threadIdx.x;
  const uint32_t W = w.W, lg2 = w.lgp - WIDE_LG1, P2 = 1u << lg2;
  if (t < WAVE) {
    // which region and piece: lane c counts the pieces of region c
    const uint32_t c = t;
    uint32_t pieces = 0, rb = 0, re = 0;
    if (c < WIDE_P1) {
      rb = w.ha[(uint64_t)c * W];
      re = w.ha[(uint64_t)(c + 1) * W];          // c = P1-1: the trailing total
      pieces = (re - rb + WIDE_TB - 1) / WIDE_TB;
    }
    const uint32_t inc = wave_incl_scan(pieces);
    const uint32_t bid = blockIdx.x;
    const bool mine = c < WIDE_P1 && bid >= inc - pieces && bid < inc;
    const uint64_t m = __ballot(mine);
    if (t == 0) sm.info[0] = m ? (uint32_t)__builtin_ctzll(m) : ~0u;
    if (mine) {
      sm.info[1] = bid - (inc - pieces);
      sm.info[2] = rb;
      sm.info[3] = re;
    }
  }
  __syncthreads();
  const uint32_t c = sm.info[0];
  if (c == ~0u) return;
  const uint32_t j = sm.info[1], rb = sm.info[2], re = sm.info[3];
  // input tiles whose run starts inside the piece: [wl, wh)
  auto first_at = [&](uint32_t lim) {             // first w with run start - rb >= lim
    uint32_t a = 0, z = W;
    while (a < z) {
      uint32_t mid = (a + z) / 2;
      if (w.ha[(uint64_t)c * W + mid] - rb < lim) a = mid + 1;
      else z = mid;
    }
    return a;
  };
  const uint32_t wl = first_at(j * WIDE_TB);
  const uint32_t wh = first_at((j + 1) * WIDE_TB);
  if (wl >= wh) return;                           // no run starts here (uniform across the group)
  const uint32_t r0 = w.ha[(uint64_t)c * W + wl];
  const uint32_t r1 = (wh < W) ? w.ha[(uint64_t)c * W + wh] : re;
  uint32_t nk[WIDE_UA];
  wide_load(nk, w.stage, r0, r1);
  const uint32_t R = W + 2;
  if (t < 64) {                                   // P2 <= 64 fine buckets; the rest stay empty
    const uint32_t l = t;
    if (l > 0 && l < P2) {
      const uint32_t d = 31 - __clz(l);
      const uint32_t k = ((WIDE_P1 + c) << d) + (l - (1u << d));
      sm.sub[l] = (uint32_t)(w.tree[k] >> 32);
    }
    sm.g.gofs[l] = l < P2 ? w.hf[(uint64_t)(c * P2 + l) * R + 1 + wl] : 0u;
    sm.g.cur[0][l] = 0;
    sm.g.cur[1][l] = 0;
  }
  __syncthreads();
  // the subtree's top three levels (nodes 1..7, the same for every key of
  // the group) from registers: three selects instead of three dependent
  // LDS reads per key
  const bool top3 = lg2 >= 3;
  uint32_t n[8];
#pragma unroll
  for (int l = 1; l < 8; l++) n[l] = top3 ? __builtin_amdgcn_readfirstlane(sm.sub[l]) : 0u;
  int x = 0;
  for (uint32_t i0 = r0; i0 < r1; i0 += WIDE_UA * NT, x ^= 1) {
    uint32_t key[WIDE_UA], f[WIDE_UA];
#pragma unroll
    for (int u = 0; u < WIDE_UA; u++) {
      key[u] = nk[u];
      f[u] = 1;
    }
    if (i0 + WIDE_UA * NT < r1) wide_load(nk, w.stage, i0 + WIDE_UA * NT, r1);
    uint32_t l = 0;
    if (top3) {
#pragma unroll
      for (int u = 0; u < WIDE_UA; u++) {
        const uint32_t k = key[u];
        const uint32_t a = n[1] < k ? 1u : 0u;
        const uint32_t b = (a ? n[3] : n[2]) < k ? 1u : 0u;
        const uint32_t m = a ? (b ? n[7] : n[6]) : (b ? n[5] : n[4]);
        f[u] = 8 + 4 * a + 2 * b + (m < k ? 1u : 0u);
      }
      l = 3;
    }
    for (; l < lg2; l++) {
#pragma unroll
      for (int u = 0; u < WIDE_UA; u++) f[u] = 2 * f[u] + (sm.sub[f[u]] < key[u] ? 1u : 0u);
    }
#pragma unroll
    for (int u = 0; u < WIDE_UA; u++) f[u] = (i0 + u * NT + t < r1) ? f[u] - P2 : ~0u;
    wide_group_write(sm.g, key, f, w.fine, x, i0 == r0);
  }
}

// Slot sort of up to 65535 keys in rounds (4-byte ord keys).  As the slot
// sort of the level kernels: slot(key) = (key - lo) >> sh over S = 2^LG2
// slots, count, scan, place, then order each slot's few keys.  A bucket
// larger than the LDS is handled in rounds: round r places the keys of the
// slots whose start lies in [r*C', (r+1)*C'), C' = CAP - ROUNDS_MAX_FILL, so
// a round never holds more than CAP keys.  Each round re-reads the bucket
// (from L2).  Returns false (having written nothing) when a slot is too
// crowded or the bucket too large.
constexpr int ROUNDS_LOG2 = 14;   // default S = 16384 slots (one work-group per CU: 156 KB of LDS)
constexpr uint32_t ROUNDS_MAX = 64;     // rounds the LDS bookkeeping has room for

template <int CAP, int LG2 = ROUNDS_LOG2>
struct SlotRoundsLds {
  uint32_t placed[CAP];
  uint32_t cnt[(1 << LG2) / 2];   // 16-bit slot counts, then starts, then cursors / ends, two per word
  alignas(8) uint64_t red[64];
  uint32_t flag;
  uint32_t rslot[ROUNDS_MAX + 1], rbase[ROUNDS_MAX + 1];   // first slot and first position of each round
};

// (crowded: a slot of more than ROUNDS_MAX_FILL keys, whose ranking would
// cost that many steps per key)
constexpr uint32_t ROUNDS_MAX_FILL = 256;

// C16: 16-bit counters over 2^LG2 slots (buckets up to 65535 keys);
// otherwise 32-bit counters over half as many slots in the same LDS
// (buckets of any size, in more rounds).
template <int NTH, int CAP, bool C16 = true, int LG2 = ROUNDS_LOG2>
__device__ __forceinline__ bool slot_sort_rounds(const uint32_t* in, uint32_t* out, uint32_t len, int kout,
                                                 SlotRoundsLds<CAP, LG2>& sm, bool lo_known, uint32_t lo, bool hi_known,
                                                 uint32_t hi) {
  constexpr int LG = C16 ? LG2 : LG2 - 1;
  constexpr int S = 1 << LG;
  constexpr int W = C16 ? S / 2 : S;       // counter words
  constexpr uint32_t CR = CAP - ROUNDS_MAX_FILL;
  const int t = threadIdx.x;
  if (C16 && len > 65535u) return false;   // (16-bit counters and positions)
  // a round re-reads the input after earlier rounds wrote the output, so
  // more than one round needs them apart
  if ((const void*)in == (const void*)out && len > CR) return false;
  if ((len + (CAP - ROUNDS_MAX_FILL) - 1) / (CAP - ROUNDS_MAX_FILL) > ROUNDS_MAX) return false;
  // every key of the bucket to fn, eight per thread per step: whole steps
  // load without bounds tests, the last one clamps its index into the bucket
  auto each_key = [&](auto&& fn) {
    uint32_t i0 = 0;
    for (; i0 + 8 * NTH <= len; i0 += 8 * NTH) {
      uint32_t k[8];
#pragma unroll
      for (int u = 0; u < 8; u++) k[u] = in[i0 + u * NTH + t];
#pragma unroll
      for (int u = 0; u < 8; u++) fn(k[u]);
    }
    if (i0 < len) {
      uint32_t k[8] = {};
#pragma unroll
      for (int u = 0; u < 8; u++)   // (rows wholly past the end load nothing)
        if (i0 + u * NTH < len) k[u] = in[min(i0 + u * NTH + t, len - 1)];
#pragma unroll
      for (int u = 0; u < 8; u++)
        if (i0 + u * NTH + t < len) fn(k[u]);
    }
  };
  uint32_t mn = ~0u, mx = 0;
  if (!(lo_known && hi_known))
    each_key([&](uint32_t k) {
      mn = k < mn ? k : mn;
      mx = k > mx ? k : mx;
    });
  for (int q = t; q < W; q += NTH) sm.cnt[q] = 0;
  if (!(lo_known && hi_known)) block_minmax<NTH>(mn, mx, (uint32_t*)sm.red);   // (ends with a barrier)
  else __syncthreads();
  if (lo_known) mn = lo;
  if (hi_known) mx = hi;
  if (mn == mx) {                          // one key value: already sorted
    for (uint32_t i = t; i < len; i += NTH) out[i] = from_ord(mn, kout);
    return true;
  }
  const int bw = bit_width<uint32_t>(mx - mn);
  const int sh = bw > LG ? bw - LG : 0;
  auto slot = [&](uint32_t k) { return (k - mn) >> sh; };
  auto get = [&](uint32_t q) -> uint32_t {   // (16-bit counter q is half q & 1 of word q >> 1)
    if constexpr (C16) return ((const u16_alias*)sm.cnt)[q];
    else return sm.cnt[q];
  };
  // old value of slot q's counter, then += 1
  auto inc = [&](uint32_t q) -> uint32_t {
    if constexpr (C16) {
      const uint32_t sft = 16 * (q & 1);
      return (atomicAdd(&sm.cnt[q >> 1], 1u << sft) >> sft) & 0xFFFFu;
    } else {
      return atomicAdd(&sm.cnt[q], 1u);
    }
  };
  each_key([&](uint32_t k) {
    const uint32_t q = slot(k);
    if constexpr (C16) atomicAdd(&sm.cnt[q >> 1], 1u << (16 * (q & 1)));
    else atomicAdd(&sm.cnt[q], 1u);
  });
  __syncthreads();
  // exclusive scan of the slot counts, and the fullest slot
  {
    constexpr int PER = W / NTH;
    uint32_t v[PER], sum = 0, mxc = 0;
#pragma unroll
    for (int j = 0; j < PER; j++) {
      v[j] = sm.cnt[t * PER + j];
      if constexpr (C16) {
        const uint32_t a0 = v[j] & 0xFFFFu, a1 = v[j] >> 16;
        sum += a0 + a1;
        mxc = max(mxc, max(a0, a1));
      } else {
        sum += v[j];
        mxc = max(mxc, v[j]);
      }
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<NTH>(sum, (uint32_t*)sm.red, &tot);
    uint32_t wm = wave_max(mxc);
    if (t == 0) sm.flag = 0;
    __syncthreads();
    if (lane_id() == 0 && wm > ROUNDS_MAX_FILL) atomicOr(&sm.flag, 1u);
#pragma unroll
    for (int j = 0; j < PER; j++) {
      if constexpr (C16) {
        const uint32_t a0 = v[j] & 0xFFFFu;
        sm.cnt[t * PER + j] = run | ((run + a0) << 16);   // starts of slots 2w and 2w+1
        run += a0 + (v[j] >> 16);
      } else {
        sm.cnt[t * PER + j] = run;
        run += v[j];
      }
    }
  }
  __syncthreads();
  const bool crowded = sm.flag != 0;
  __syncthreads();
  if (crowded) return false;
  // first slot whose start is >= x (slot starts are non-decreasing; S if none)
  auto first_slot = [&](uint32_t x) {
    uint32_t a = 0, z = S;
    while (a < z) {
      uint32_t m = (a + z) / 2;
      if (get(m) < x) a = m + 1;
      else z = m;
    }
    return a;
  };
  // round boundaries, taken while the counters still hold the slot starts
  const uint32_t rounds = (len + CR - 1) / CR;
  for (uint32_t t2 = t; t2 <= rounds; t2 += NTH) {
    const int t = (int)t2;
    const uint32_t b = (t == 0) ? 0u : ((uint32_t)t < rounds ? first_slot(t * CR) : (uint32_t)S);
    sm.rslot[t] = b;
    sm.rbase[t] = b < (uint32_t)S ? get(b) : len;
  }
  __syncthreads();
  for (uint32_t r = 0; r < rounds; r++) {
    // slots [qa, qb) of this round; slots below qa already hold their ends
    const uint32_t qa = sm.rslot[r], qb = sm.rslot[r + 1], base = sm.rbase[r];
    auto place = [&](uint32_t k) {
      const uint32_t q = slot(k);
      if (rounds == 1 || (q >= qa && q < qb)) sm.placed[inc(q) - base] = k;
    };
    each_key(place);
    __syncthreads();
    // order each slot (the counter of slot q < qb now holds its end)
    const uint32_t top = (qb < (uint32_t)S ? get(qb - 1) : len) - base;
    slot_rank_write<4, NTH>(sm.placed, top, out + base, kout, [&](uint32_t k, uint32_t& s0, uint32_t& s1) {
      const uint32_t q = slot(k);
      const uint32_t e0 = get(q ? q - 1 : 0u);
      s0 = (q ? e0 : 0u) - base;
      s1 = get(q) - base;
    });
    __syncthreads();
  }
  return true;
}

// One fine bucket per work-group: write its tie runs, slot-sort its other
// keys (or hand them to the leftover list).
template <int CAP, int LG2>
__global__ void __launch_bounds__(WIDE_BNT) k_wide_bucket(LevelArgs a, WideArgs w, int export_stages) {
  __shared__ SlotRoundsLds<CAP, LG2> sm;
  const uint32_t b = blockIdx.x;
  if (b >= w.p) return;
  const int t = threadIdx.x;
  const uint32_t R = w.W + 2;
  const uint32_t beg = w.hf[(uint64_t)b * R], nt0 = w.hf[(uint64_t)b * R + 1];
  const uint32_t nt1 = w.hf[(uint64_t)b * R + R - 1], end = w.hf[(uint64_t)(b + 1) * R];
  if (export_stages && t == 0) a.exp_counts[b] = end - beg;
  auto spl_key = [&](uint32_t r) -> uint32_t {   // key of splitter of rank r (1-based)
    const uint32_t z = __builtin_ctz(r);
    const uint32_t k = (1u << (w.lgp - 1 - z)) + (r >> (z + 1));
    return (uint32_t)(w.tree[k] >> 32);
  };
  const bool lo_k = b >= 1, hi_k = b + 1 < w.p;
  const uint32_t lo = lo_k ? spl_key(b) : 0u;
  const uint32_t hi = hi_k ? spl_key(b + 1) : 0u;
  uint32_t* out = (uint32_t*)w.out;
  if (nt0 > beg) {
    const uint32_t v = from_ord(lo, w.kout);
    for (uint32_t i = beg + t; i < nt0; i += WIDE_BNT) __builtin_nontemporal_store(v, &out[i]);
  }
  if (end > nt1) {
    const uint32_t v = from_ord(hi, w.kout);
    for (uint32_t i = nt1 + t; i < end; i += WIDE_BNT) __builtin_nontemporal_store(v, &out[i]);
  }
  const uint32_t sz = nt1 - nt0;
  if (sz > WIDE_BMAX && a.next_segs) {
    // larger than one work-group sorts: the next level splits the keys
    // between the tie runs again (they are in the workspace copy, where it
    // reads)
    if (t == 0) {
      atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)(end - beg - sz));
      const uint32_t slot = atomicAdd(&a.next_ctl->nsegs, 1u);
      if (slot < a.next_cap) {
        SegDesc nd = {};
        nd.beg = nt0;
        nd.len = sz;
        nd.seed = derive_seed(a.segs[0].seed, 1, b);
        nd.depth = 1;
        nd.parent_bkt = b;
        a.next_segs[slot] = nd;
      } else {
        atomicOr(&a.gctl->status, ST_LIST_FULL);
        const uint32_t k = atomicAdd(a.nleft, 1u);
        a.left[k] = SmallEnt{nt0, sz, b};
      }
    }
    return;
  }
  bool done = sz == 0;
  if (!done && sz <= WIDE_BMAX)
    done = slot_sort_rounds<WIDE_BNT, CAP, true, LG2>(w.fine + nt0, out + nt0, sz, w.kout, sm, lo_k, lo, hi_k, hi);
  else if (!done)
    done = slot_sort_rounds<WIDE_BNT, CAP, false, LG2>(w.fine + nt0, out + nt0, sz, w.kout, sm, lo_k, lo, hi_k, hi);
  if (t == 0) {
    if (done) {
      atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)(end - beg));
    } else {
      atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)(end - beg - sz));
      const uint32_t k = atomicAdd(a.nleft, 1u);
      a.left[k] = SmallEnt{nt0, sz, b};
    }
  }
}

// Keys only, 4-byte keys: buckets the slot sort of a level handed on (too
// large for it, or crowded) get the round-based slot sort; what that cannot
// take goes on to the radix sort's list.
__global__ void __launch_bounds__(WIDE_BNT) k_bucket_rounds_keys(LevelArgs a) {
  __shared__ SlotRoundsLds<WIDE_BCAP> sm;
  const uint32_t nl = *a.nleft;
  for (uint32_t li = blockIdx.x; li < nl; li += gridDim.x) {
    const SmallEnt e = a.left[li];
    const uint32_t* src = (const uint32_t*)a.dst + e.beg;
    uint32_t* dst = (uint32_t*)a.out + e.beg;
    if ((const void*)src == (const void*)dst && e.len > WIDE_BCAP - ROUNDS_MAX_FILL) {
      // the level wrote its buckets into the output (odd levels): a bucket
      // sorted in several rounds reads a copy in tmp, whose range of the
      // bucket the level's split has already consumed
      uint32_t* cp = (uint32_t*)a.tmp + e.beg;
      for (uint32_t i = threadIdx.x; i < e.len; i += WIDE_BNT) cp[i] = src[i];
      __threadfence();
      __syncthreads();
      src = cp;
    }
    const bool done = e.len <= WIDE_BMAX
                          ? slot_sort_rounds<WIDE_BNT, WIDE_BCAP>(src, dst, e.len, a.kout, sm, false, 0u, false, 0u)
                          : slot_sort_rounds<WIDE_BNT, WIDE_BCAP, false>(src, dst, e.len, a.kout, sm, false, 0u,
                                                                         false, 0u);
    if (threadIdx.x == 0) {
      if (done) {
        atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)e.len);
      } else {
        const uint32_t k = atomicAdd(a.nleft2, 1u);
        a.left2[k] = e;
      }
    }
    __syncthreads();
  }
}

}  // namespace ss
