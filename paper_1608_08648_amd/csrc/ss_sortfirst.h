// Sort-first organisation of the method, as Alg. 1 and Alg. 2 state it:
//   step 1  the p blocks [floor(k n / p), floor((k+1) n / p)) are sorted by
//           (key, in-block index) (the segmented path, index as payload);
//   steps 2-3 the sample (regular: from the sorted blocks, Alg. 1; random:
//           from the input, Alg. 2) and its p - 1 splitters, as in the
//           split-first path;
//   step 4  every splitter is placed in every sorted block by binary search
//           (the alternative the analysis of step 4 gives to merging), which
//           cuts block k into the runs X_{k,j};
//   step 5  bucket j is formed from its p runs X_{0,j} .. X_{p-1,j}: merged
//           pairwise (k_sf_merge, SS_F_SF_MERGE: the merging the paper
//           states), or gathered in block order and sorted in LDS with the
//           round-based slot sort (the default); the concatenation of the
//           buckets is the output.  Those two forms of step 5 take 4-byte
//           keys without payload; 8-byte keys and every payload are gathered
//           with their payloads (k_sf_gather_any) and the p buckets sorted
//           as segments by the segmented path.
// Keys compare as (ord(key), global index), the same total order as the
// split-first classification, so bucket j holds exactly the keys that
// classification puts in bucket j.
#pragma once
#include "ss_wide.h"

namespace ss {

constexpr int SF_NT = 1024;                // threads of the search kernel
constexpr uint32_t SF_LDS_BYTES = 65536;   // sorted block keys the search holds in LDS (at most 64 KB)
constexpr uint32_t SF_PMAX = 4096;         // largest p: the gather kernel's run table (32 KB)
constexpr int SF_GNT = 512;                // threads of the gather kernel

struct SfArgs {
  const uint32_t* bkeys;   // step 1: the sorted blocks (keys as given; 8-byte keys: two words each)
  const uint32_t* bidx;    // in-block index of each sorted key
  const uint64_t* tree;    // Eytzinger tree of the splitters, slot k in [1, p): (ord << 32) | tag for
                           // 4-byte keys; the ord for 8-byte keys, whose tags are in tree_tag
  const uint32_t* tree_tag;
  uint32_t* pos;           // p rows of p + 1: pos[k (p+1) + j] = start of X_{k,j} in sorted block k
  uint2* bkt;              // per bucket: (output start, size)
  uint32_t* stage;         // step 5: the gathered buckets, as ord keys
  uint64_t n;
  uint32_t p, lgp;
  int kind;                // key kind (to_ord / from_ord)
  uint32_t lds_keys;       // search: the longest block when it fits SF_LDS_KEYS (the LDS launched), else 0
};

__device__ __forceinline__ uint64_t sf_block_start(uint64_t n, uint32_t p, uint32_t k) {
  return ((uint64_t)k * n) / p;
}

// splitter of rank r (1 <= r < p) from the Eytzinger tree
__device__ __forceinline__ uint64_t sf_splitter(const uint64_t* tree, uint32_t lgp, uint32_t r) {
  const uint32_t z = __builtin_ctz(r);
  return tree[(1u << (lgp - 1 - z)) + (r >> (z + 1))];
}

// Step 4: one work-group per sorted block k writes pos[k][0..p]: the number
// of the block's keys not above each splitter in (key, index) order (a key
// belongs to the bucket of the first splitter not below it, so a sampled
// key equal to splitter j stays in bucket j - 1, as the classification
// #{splitters < (key, index)} has it).
template <int KW>
__global__ void __launch_bounds__(SF_NT) k_sf_search(SfArgs f) {
  using KT = typename KeyOf<KW>::T;
  extern __shared__ uint64_t sk_raw[];   // f.lds_keys keys
  KT* sk = (KT*)sk_raw;
  const KT* bkeys = (const KT*)f.bkeys;
  const uint32_t k = blockIdx.x;
  if (k >= f.p) return;
  const uint64_t bs = sf_block_start(f.n, f.p, k);
  const uint32_t len = (uint32_t)(sf_block_start(f.n, f.p, k + 1) - bs);
  const bool lds = len <= f.lds_keys;
  if (lds)
    for (uint32_t i = threadIdx.x; i < len; i += SF_NT) sk[i] = to_ord(bkeys[bs + i], f.kind);
  __syncthreads();
  uint32_t* row = f.pos + (uint64_t)k * (f.p + 1);
  // each thread takes consecutive splitters: the first by binary search, each
  // later one by a galloping search from the previous one's place (the
  // splitters are sorted, so their places are too)
  const uint32_t per = (f.p + SF_NT) / SF_NT;   // (p + 1 entries)
  const uint32_t r0 = threadIdx.x * per, r1 = min(f.p + 1, r0 + per);
  uint32_t prev = 0;
  for (uint32_t r = r0; r < r1; r++) {
    uint32_t res = len;
    if (r == 0) {
      res = 0;
    } else if (r < f.p) {
      KT skey;
      uint64_t stag;
      if constexpr (KW == 4) {
        const uint64_t sp = sf_splitter(f.tree, f.lgp, r);
        skey = (KT)(sp >> 32);
        stag = (uint32_t)sp;
      } else {
        const uint32_t z = __builtin_ctz(r);
        const uint32_t slot = (1u << (f.lgp - 1 - z)) + (r >> (z + 1));
        skey = f.tree[slot];
        stag = f.tree_tag[slot];
      }
      // upto(m): the block's key m is not above the splitter; the answer is
      // the first m in [prev, len) where it fails
      auto upto = [&](uint32_t m) {
        const KT km = lds ? sk[m] : to_ord(bkeys[bs + m], f.kind);
        return km < skey || (km == skey && bs + f.bidx[bs + m] <= stag);
      };
      uint32_t a = prev, z = len;
      if (r > r0) {   // gallop: widen [a, a + step) until it holds the answer
        uint32_t step = 1;
        while (a + step <= len && upto(a + step - 1)) {
          a += step;
          step *= 2;
        }
        z = min(len, a + step);
      }
      while (a < z) {
        const uint32_t m = (a + z) >> 1;
        if (upto(m)) a = m + 1;
        else z = m;
      }
      res = a;
    }
    prev = res;
    row[r] = res;
  }
}

// Step 5 for any key and payload width: bucket j gathers its runs (block
// order) with their payloads -- the caller's payload of each key, found
// through its in-block index, or for an index payload that index -- into
// the stage, and the buckets are then sorted as segments (stable, so equal
// keys keep the gathered order, which is input order).  off[j] = start of
// bucket j, off[p] = n.
template <int KW, int VW>
__global__ void __launch_bounds__(SF_GNT) k_sf_gather_any(SfArgs f, void* kstage, void* vstage, const void* vin,
                                                          int iota, int64_t* off, uint64_t* exp_counts) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  __shared__ uint32_t offs[SF_PMAX + 1];   // start of run k in the bucket
  __shared__ uint32_t src[SF_PMAX];        // start of run k in the sorted blocks
  __shared__ uint32_t red[2 * (SF_GNT / WAVE)];
  const uint32_t j = xcd_tile(blockIdx.x, gridDim.x), p = f.p;   // (consecutive buckets on one XCD)
  if (j >= p) return;
  const int t = threadIdx.x;
  const uint32_t per = (p + SF_GNT - 1) / SF_GNT;
  const uint32_t k0 = min(p, (uint32_t)t * per), k1 = min(p, k0 + per);
  uint32_t cnt = 0, below = 0;
  for (uint32_t k = k0; k < k1; k++) {
    const uint32_t* row = f.pos + (uint64_t)k * (p + 1);
    const uint32_t a = row[j], b = row[j + 1];
    src[k] = (uint32_t)sf_block_start(f.n, p, k) + a;
    offs[k] = b - a;
    cnt += b - a;
    below += a;
  }
  uint32_t tot;
  uint32_t run = block_excl_scan<SF_GNT>(cnt, red, &tot);
  __syncthreads();
  for (uint32_t k = k0; k < k1; k++) {
    const uint32_t l = offs[k];
    offs[k] = run;
    run += l;
  }
  if (t == 0) offs[p] = tot;
  uint32_t start;
  block_excl_scan<SF_GNT>(below, red, &start);
  __syncthreads();
  const KT* bkeys = (const KT*)f.bkeys;
  for (uint32_t e = t; e < tot; e += SF_GNT) {
    uint32_t a = 0, z = p;   // last run whose start is <= e
    while (z - a > 1) {
      const uint32_t m = (a + z) >> 1;
      if (offs[m] <= e) a = m;
      else z = m;
    }
    const uint32_t q = src[a] + (e - offs[a]);            // position in the sorted blocks
    ((KT*)kstage)[start + e] = bkeys[q];
    if constexpr (VW != 0) {
      const uint64_t gi = sf_block_start(f.n, p, a) + f.bidx[q];   // input index of the key
      ((VT*)vstage)[start + e] = iota ? (VT)gi : ((const VT*)vin)[gi];
    }
  }
  if (t == 0) {
    off[j] = start;
    if (j == p - 1) off[p] = (int64_t)f.n;
    f.bkt[j] = make_uint2(start, tot);
    if (exp_counts) exp_counts[j] = tot;
  }
}

// Step 5, first half: one work-group per bucket j finds its runs X_{k,j},
// their places in the bucket (a scan over k) and the bucket's output start
// (the keys of all blocks up to splitter j), and copies the runs, in block
// order, to stage[start ..] as ord keys.  Each wave copies a contiguous
// range, one key per lane and step; a bitmap of the positions where a
// non-empty run starts gives each lane its run: the wave's count of run
// starts so far plus those among the lanes up to it (a bucket past the
// bitmap finds each key's run by binary search instead).
constexpr uint32_t SF_GMAP = 65536;        // bucket positions the run-start bitmap covers (8 KB)

__global__ void __launch_bounds__(SF_GNT) k_sf_gather(SfArgs f, uint64_t* exp_counts) {
  __shared__ uint32_t off[SF_PMAX + 1];    // start of run k in the bucket
  __shared__ uint32_t src[SF_PMAX];        // start of run k in the sorted blocks
  __shared__ uint32_t red[2 * (SF_GNT / WAVE)];
  __shared__ uint16_t nz[SF_PMAX];         // k of the i-th non-empty run
  __shared__ uint32_t bits[SF_GMAP / 32];  // bit e: a non-empty run starts at bucket position e
  // consecutive buckets on one XCD: bucket j + 1's run of block k starts where
  // bucket j's ends, so the cache lines of one bucket's runs serve the next
  // from that XCD's L2
  const uint32_t j = xcd_tile(blockIdx.x, gridDim.x), p = f.p;
  if (j >= p) return;
  const int t = threadIdx.x;
  const uint32_t per = (p + SF_GNT - 1) / SF_GNT;   // consecutive runs per thread
  const uint32_t k0 = min(p, (uint32_t)t * per), k1 = min(p, k0 + per);
  uint32_t cnt = 0, below = 0, cnz = 0;
  for (uint32_t k = k0; k < k1; k++) {
    const uint32_t* row = f.pos + (uint64_t)k * (p + 1);
    const uint32_t a = row[j], b = row[j + 1];
    src[k] = (uint32_t)sf_block_start(f.n, p, k) + a;
    off[k] = b - a;            // (length until the scan)
    cnt += b - a;
    cnz += b > a ? 1u : 0u;
    below += a;
  }
  uint32_t tot;
  uint32_t run = block_excl_scan<SF_GNT>(cnt, red, &tot);
  __syncthreads();
  uint32_t nnz;
  uint32_t zi = block_excl_scan<SF_GNT>(cnz, red, &nnz);
  const bool mapped = tot <= SF_GMAP;
  if (mapped)
    for (uint32_t q = t; q < (tot + 31) / 32; q += SF_GNT) bits[q] = 0;
  __syncthreads();
  for (uint32_t k = k0; k < k1; k++) {
    const uint32_t l = off[k];
    off[k] = run;
    if (l) {
      nz[zi++] = (uint16_t)k;
      if (mapped) atomicOr(&bits[run >> 5], 1u << (run & 31));
    }
    run += l;
  }
  if (t == 0) off[p] = tot;
  uint32_t start;
  block_excl_scan<SF_GNT>(below, red, &start);   // (total of the keys up to splitter j)
  __syncthreads();
  if (mapped) {
    constexpr uint32_t NW = SF_GNT / WAVE;
    const uint32_t w = (uint32_t)t / WAVE, lane = (uint32_t)t % WAVE;
    const uint64_t upto = lane == WAVE - 1 ? ~0ull : ((1ull << (lane + 1)) - 1);   // lanes <= this one
    const uint32_t chunk = ((tot + NW - 1) / NW + WAVE - 1) / WAVE * WAVE;
    const uint32_t e0 = min(tot, w * chunk), e1 = min(tot, e0 + chunk);
    // runs that start before e0: the first i with off[nz[i]] >= e0
    uint32_t lo = 0, hi = nnz;
    while (lo < hi) {
      const uint32_t m = (lo + hi) >> 1;
      if (off[nz[m]] < e0) lo = m + 1;
      else hi = m;
    }
    int base = (int)lo - 1;    // nz index of the run holding position e0 - 1
    for (uint32_t e = e0 + lane; e - lane < e1; e += WAVE) {
      const bool in = e < e1;
      const bool st = in && ((bits[e >> 5] >> (e & 31)) & 1u);
      const uint64_t m = __ballot(st);
      if (in) {
        const uint32_t a = nz[base + __popcll(m & upto)];   // the run holding position e
        f.stage[start + e] = to_ord(f.bkeys[src[a] + (e - off[a])], f.kind);
      }
      base += __popcll(m);
    }
  } else {
    for (uint32_t e = t; e < tot; e += SF_GNT) {
      uint32_t a = 0, z = p;   // last run whose start is <= e
      while (z - a > 1) {
        const uint32_t m = (a + z) >> 1;
        if (off[m] <= e) a = m;
        else z = m;
      }
      f.stage[start + e] = to_ord(f.bkeys[src[a] + (e - off[a])], f.kind);
    }
  }
  if (t == 0) {
    f.bkt[j] = make_uint2(start, tot);
    if (exp_counts) exp_counts[j] = tot;
  }
}

// Step 5, second half: one work-group per bucket sorts its gathered keys
// (they lie between the keys of splitters j and j + 1, both included) with
// the round-based slot sort; crowded buckets go to the radix sort's list.
template <int CAP, int LG2>
__global__ void __launch_bounds__(WIDE_BNT) k_sf_bucket(LevelArgs a, SfArgs f) {
  __shared__ SlotRoundsLds<CAP, LG2> sm;
  const uint32_t j = blockIdx.x;
  if (j >= f.p) return;
  const uint2 e = f.bkt[j];
  const bool lo_k = j >= 1, hi_k = j + 1 < f.p;
  const uint32_t lo = lo_k ? (uint32_t)(sf_splitter(f.tree, f.lgp, j) >> 32) : 0u;
  const uint32_t hi = hi_k ? (uint32_t)(sf_splitter(f.tree, f.lgp, j + 1) >> 32) : 0u;
  uint32_t* out = (uint32_t*)a.out + e.x;
  bool done = e.y == 0;
  if (!done && e.y <= WIDE_BMAX)
    done = slot_sort_rounds<WIDE_BNT, CAP, true, LG2>(f.stage + e.x, out, e.y, f.kind, sm, lo_k, lo, hi_k, hi);
  else if (!done)
    done = slot_sort_rounds<WIDE_BNT, CAP, false, LG2>(f.stage + e.x, out, e.y, f.kind, sm, lo_k, lo, hi_k, hi);
  if (threadIdx.x == 0) {
    if (done) {
      atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)e.y);
    } else {
      const uint32_t k = atomicAdd(a.nleft, 1u);
      a.left[k] = SmallEnt{e.x, e.y, j};
    }
  }
}

// Step 5 as the paper states it: bucket j is the merge of its p runs
// X_{0,j} .. X_{p-1,j}.  One work-group per bucket merges neighbouring
// groups of runs pairwise, lg p rounds: in round r groups of 2^r runs
// become groups of 2^(r+1).  Buckets of up to SFM_CAP keys are merged in
// LDS; larger ones between the stage and the output (both in global
// memory, ping-pong), the last round writing the output.  In a round each
// thread produces consecutive outputs: it finds the pair its first output
// falls in, splits that pair's merge path at its output (a binary search
// on the diagonal, the first group winning ties) and merges sequentially
// from there, moving on to the next pair when one ends.
constexpr int SFM_NT = 1024;
constexpr uint32_t SFM_CAP = 16384;            // keys a bucket may have to be merged in LDS

struct SfMergeLds {
  uint32_t buf[2][SFM_CAP];      // (buf[1] holds the runs' block starts until the first round)
  uint32_t off[SF_PMAX + 1];     // start of run k in the bucket (off[p] = bucket size)
  uint32_t red[2 * (SFM_NT / WAVE)];
};
static_assert(SF_PMAX <= SFM_CAP, "run starts fit the second buffer");

// One merge round over the bucket: groups of w runs in `in` -> groups of 2w
// in `out` (outputs [e0, e1) of this thread); `last` converts to key bits.
__device__ __forceinline__ void sf_merge_round(const uint32_t* in, uint32_t* out, const uint32_t* off, uint32_t p,
                                               uint32_t w, uint32_t e0, uint32_t e1, bool last, int kind) {
  auto run_of = [&](uint32_t e) {                // last run whose start is <= e
    uint32_t lo = 0, hi = p;
    while (hi - lo > 1) {
      const uint32_t m = (lo + hi) >> 1;
      if (off[m] <= e) lo = m;
      else hi = m;
    }
    return lo;
  };
  uint32_t e = e0;
  while (e < e1) {
    const uint32_t q = run_of(e) / (2 * w);
    const uint32_t ra = 2 * q * w, rm = min(p, ra + w), rz = min(p, ra + 2 * w);
    const uint32_t pa = off[ra], pm = off[rm], pz = off[rz];
    const uint32_t la = pm - pa, lb = pz - pm, d = e - pa;
    // merge path: i elements from the first group, d - i from the second
    uint32_t lo = d > lb ? d - lb : 0, hi = min(d, la);
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (in[pa + mid] <= in[pm + d - 1 - mid]) lo = mid + 1;   // (the first group wins ties)
      else hi = mid;
    }
    uint32_t i = lo, k = d - lo;
    const uint32_t stop = min(e1, pz);
    for (; e < stop; e++) {
      const bool takeA = k >= lb || (i < la && in[pa + i] <= in[pm + k]);
      const uint32_t v = takeA ? in[pa + i] : in[pm + k];
      out[e] = last ? from_ord(v, kind) : v;
      if (takeA) i++;
      else k++;
    }
  }
}

__global__ void __launch_bounds__(SFM_NT) k_sf_merge(LevelArgs a, SfArgs f, uint64_t* exp_counts) {
  __shared__ SfMergeLds sm;
  const uint32_t j = xcd_tile(blockIdx.x, gridDim.x), p = f.p;   // (consecutive buckets on one XCD)
  if (j >= p) return;
  const int t = threadIdx.x;
  uint32_t* src = sm.buf[1];     // start of run k in the sorted blocks
  // run table (as in the gather): lengths, their scan, the bucket's start
  const uint32_t per = (p + SFM_NT - 1) / SFM_NT;
  const uint32_t k0 = min(p, (uint32_t)t * per), k1 = min(p, k0 + per);
  uint32_t cnt = 0, below = 0;
  for (uint32_t k = k0; k < k1; k++) {
    const uint32_t* row = f.pos + (uint64_t)k * (p + 1);
    const uint32_t ra = row[j], rb = row[j + 1];
    src[k] = (uint32_t)sf_block_start(f.n, p, k) + ra;
    sm.off[k] = rb - ra;
    cnt += rb - ra;
    below += ra;
  }
  uint32_t tot;
  uint32_t run = block_excl_scan<SFM_NT>(cnt, sm.red, &tot);
  __syncthreads();
  for (uint32_t k = k0; k < k1; k++) {
    const uint32_t l = sm.off[k];
    sm.off[k] = run;
    run += l;
  }
  if (t == 0) sm.off[p] = tot;
  uint32_t start;
  block_excl_scan<SFM_NT>(below, sm.red, &start);
  __syncthreads();
  if (t == 0) {
    f.bkt[j] = make_uint2(start, tot);
    if (exp_counts) exp_counts[j] = tot;
  }
  auto run_of = [&](uint32_t e) {
    uint32_t lo = 0, hi = p;
    while (hi - lo > 1) {
      const uint32_t m = (lo + hi) >> 1;
      if (sm.off[m] <= e) lo = m;
      else hi = m;
    }
    return lo;
  };
  uint32_t rounds = 0;
  while ((1u << rounds) < p) rounds++;
  const bool lds = tot <= SFM_CAP;
  // the runs, in block order, as ord keys: in LDS, or in global memory
  // where an odd number of rounds then ends in the output
  uint32_t* g0 = (rounds & 1) ? f.stage + start : (uint32_t*)a.out + start;
  uint32_t* g1 = (rounds & 1) ? (uint32_t*)a.out + start : f.stage + start;
  uint32_t* b0 = lds ? sm.buf[0] : g0;
  for (uint32_t e = t; e < tot; e += SFM_NT) {
    const uint32_t r = run_of(e);
    b0[e] = to_ord(f.bkeys[src[r] + (e - sm.off[r])], f.kind);
  }
  __syncthreads();
  const uint32_t K = (tot + SFM_NT - 1) / SFM_NT;
  const uint32_t e0 = min(tot, (uint32_t)t * K), e1 = min(tot, e0 + K);
  uint32_t* bufs[2] = {b0, lds ? sm.buf[1] : g1};
  for (uint32_t r = 0; r < rounds; r++) {
    const bool last = !lds && r + 1 == rounds;
    sf_merge_round(bufs[r & 1], bufs[(r + 1) & 1], sm.off, p, 1u << r, e0, e1, last, f.kind);
    __syncthreads();
  }
  if (lds) {
    const uint32_t* res = bufs[rounds & 1];
    uint32_t* out = (uint32_t*)a.out + start;
    for (uint32_t e = t; e < tot; e += SFM_NT) out[e] = from_ord(res[e], f.kind);
  } else if (rounds == 0) {
    uint32_t* out = (uint32_t*)a.out + start;   // (p = 1 does not occur: one run is the bucket)
    for (uint32_t e = t; e < tot; e += SFM_NT) out[e] = from_ord(b0[e], f.kind);
  }
  if (t == 0) atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)tot);
}

}  // namespace ss
