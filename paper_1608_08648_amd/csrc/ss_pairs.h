// Stable bucket sort for (key, payload) pairs.
//
// The stable split (step 4) leaves every bucket in input order, so the
// position of an element inside its bucket is its input order among equal
// keys.  The slot sort of the keys-only path orders a bucket by counting its
// keys into value slots and ranking each key inside its slot; here every
// placed element also carries its position in the bucket, and the rank
// inside a slot compares (key, position): equal keys keep input order, so
// the result is the stable order (Section 1) without a radix pass per digit.
#pragma once
#include "ss_wide.h"

namespace ss {

// Elements per bucket in LDS (key, payload, 16-bit position): about 143 KB
// next to the slot counters, for one 1024-thread work-group per CU.
template <int KW, int VW> struct StableSlotCap {
  static constexpr int C = (KW + VW <= 8) ? 14336 : ((KW + VW <= 12) ? 10240 : 7680);
};
constexpr uint32_t STABLE_MAX_FILL = 64;   // crowded-slot limit

// IOTA: the payload is the position inside the bucket (an in-segment
// index), which the placed 16-bit position already holds: no payload array,
// so 16384 4-byte keys fit (112 KB).
template <int KW, int VW, bool IOTA = false>
struct SlotStableLds {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  static constexpr int C = IOTA ? (KW == 4 ? 16384 : 8192) : StableSlotCap<KW, VW>::C;
  KT pk[C];
  VT pv[IOTA ? 1 : C];
  uint16_t pi[C];
  uint32_t scnt[(1 << SLOT_LOG2) / 2];   // two 16-bit slot counters per word
  alignas(8) uint64_t red[64];
  uint32_t flag;
};

// Sorts in[0, len) (key map kin: ord images by default) with payloads
// vin[0, len) into out / vout (caller's key type), stable; IOTA: the payload
// is the index in [0, len) and vin is not read.  Returns false (having
// written nothing) when the bucket is larger than the LDS or a slot is
// crowded.
template <int KW, int VW, int NTH, bool IOTA = false>
__device__ __forceinline__ bool slot_sort_stable(const typename KeyOf<KW>::T* in, const typename ValOf<VW>::T* vin,
                                                 typename KeyOf<KW>::T* out, typename ValOf<VW>::T* vout,
                                                 uint32_t len, int kout, SlotStableLds<KW, VW, IOTA>& sm,
                                                 bool lo_known, typename KeyOf<KW>::T lo, bool hi_known,
                                                 typename KeyOf<KW>::T hi, int kin = 0) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  constexpr int S = 1 << SLOT_LOG2;
  constexpr int W = S / 2;
  const int t = threadIdx.x;
  if (len > (uint32_t)SlotStableLds<KW, VW, IOTA>::C) return false;
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
  if (mn == mx) {                          // one key value: the bucket is in input order already
    for (uint32_t i = t; i < len; i += NTH) {
      out[i] = from_ord(mn, kout);
      vout[i] = IOTA ? (VT)i : vin[i];
    }
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
      const uint32_t a0 = v[j] & 0xFFFFu, a1 = v[j] >> 16;
      sum += a0 + a1;
      mxc = max(mxc, max(a0, a1));
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<NTH>(sum, (uint32_t*)sm.red, &tot);
    const uint32_t wm = wave_max(mxc);
    if (t == 0) sm.flag = 0;
    __syncthreads();
    if (lane_id() == 0 && wm > STABLE_MAX_FILL) atomicOr(&sm.flag, 1u);
#pragma unroll
    for (int j = 0; j < PER; j++) {
      const uint32_t a0 = v[j] & 0xFFFFu;
      sm.scnt[t * PER + j] = run | ((run + a0) << 16);   // starts of slots 2w and 2w+1
      run += a0 + (v[j] >> 16);
    }
  }
  __syncthreads();
  const bool crowded = sm.flag != 0;
  __syncthreads();
  if (crowded) return false;
  // place (key, payload, position); afterwards each slot's counter holds its end
  // (the last read of the bucket: streaming loads; the output, written once,
  // leaves with streaming stores)
  for (uint32_t i0 = 0; i0 < len; i0 += 4 * NTH) {
    KT k[4];
    VT v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      k[u] = KT(0);
      v[u] = VT(0);
      if (i0 + u * NTH < len) {   // (rows wholly past the end load nothing)
        const uint32_t i = min(i0 + u * NTH + t, len - 1);
        k[u] = to_ord(__builtin_nontemporal_load(&in[i]), kin);
        if constexpr (!IOTA) v[u] = __builtin_nontemporal_load(&vin[i]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint32_t i = i0 + u * NTH + t;
      if (i < len) {
        const uint32_t q = slot(k[u]);
        const uint32_t sft = 16 * (q & 1);
        const uint32_t pos = (atomicAdd(&sm.scnt[q >> 1], 1u << sft) >> sft) & 0xFFFFu;
        sm.pk[pos] = k[u];
        if constexpr (!IOTA) sm.pv[pos] = v[u];
        sm.pi[pos] = (uint16_t)i;
      }
    }
  }
  __syncthreads();
  // rank inside the slot by (key, position)
  auto slot_end = [&](uint32_t q) -> uint32_t { return ((const u16_alias*)sm.scnt)[q]; };
  for (uint32_t j = t; j < len; j += NTH) {
    const KT k = sm.pk[j];
    const uint32_t ip = sm.pi[j];
    const uint32_t q = slot(k);
    const uint32_t e0 = slot_end(q ? q - 1 : 0u);
    const uint32_t s0 = q ? e0 : 0u, s1 = slot_end(q);
    uint32_t rank = 0;
    if constexpr (KW == 4) {
      // (key, input position) as one 64-bit number: one compare per key
      const uint64_t me = ((uint64_t)k << 32) | ip;
      for (uint32_t o = s0; o < s1; o++) rank += (((uint64_t)sm.pk[o] << 32) | sm.pi[o]) < me ? 1u : 0u;
    } else {
      for (uint32_t o = s0; o < s1; o++) {
        const KT ko = sm.pk[o];
        rank += (ko < k || (ko == k && sm.pi[o] < ip)) ? 1u : 0u;
      }
    }
    __builtin_nontemporal_store(from_ord(k, kout), &out[s0 + rank]);
    __builtin_nontemporal_store(IOTA ? (VT)ip : sm.pv[j], &vout[s0 + rank]);
  }
  __syncthreads();
  return true;
}

// Segments of the small class whose payload is their in-segment index
// (4-byte keys; the blocks of the sort-first organisation and of regular
// sampling, the row sort's short rows): the stable slot sort, whose placed
// positions are that payload, with 1024 threads; a segment past its LDS or
// with a crowded slot goes to the list `fb`, which the radix sort of the
// small class takes next.
template <int KW, int VW>
__global__ void __launch_bounds__(WIDE_BNT) k_sort_small_list_iota(Ctl* g, const SmallEnt* list, SmallEnt* fb,
                                                                   const void* src, void* out, void* vout, int kind) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  static_assert(KW == 4 && VW == 4, "4-byte keys with a 32-bit index");
  __shared__ SlotStableLds<KW, VW, true> sm;
  if (blockIdx.x >= g->nsmall) return;
  const SmallEnt e = list[blockIdx.x];
  if (!slot_sort_stable<KW, VW, WIDE_BNT, true>((const KT*)src + e.beg, nullptr, (KT*)out + e.beg,
                                                (VT*)vout + e.beg, e.len, kind, sm, false, KT(0), false, KT(0), kind) &&
      threadIdx.x == 0)
    fb[atomicAdd(&g->nsmall_fb, 1u)] = e;
}

// Buckets of a split level (pairs): stable slot sort in LDS; buckets too
// large or crowded go to the list of the radix / next-level kernel.
template <int KW, int VW>
__global__ void __launch_bounds__(WIDE_BNT) k_bucket_sort_pairs(LevelArgs a, int export_stages) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  __shared__ SlotStableLds<KW, VW> sm;
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
  auto spl_key = [&](uint32_t r) -> KT {
    const uint32_t z = __builtin_ctz(r);
    const uint32_t k = (1u << (d.lgp - 1 - z)) + (r >> (z + 1));
    const uint64_t node = ((const uint64_t*)a.tree)[d.tree_off + k];
    if constexpr (KW == 4) return (KT)(node >> 32);
    else return (KT)node;
  };
  const bool lo_k = b >= 1, hi_k = b + 1 < d.p;
  const KT lo = lo_k ? spl_key(b) : KT(0);
  const KT hi = hi_k ? spl_key(b + 1) : KT(0);
  const bool done = slot_sort_stable<KW, VW, WIDE_BNT>((const KT*)a.dst + gb, (const VT*)a.vdst + gb,
                                                        (KT*)a.out + gb, (VT*)a.vout + gb, sz, a.kout, sm, lo_k, lo,
                                                        hi_k, hi);
  if (threadIdx.x == 0) {
    if (done) {
      atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)sz);
    } else {
      const uint32_t k = atomicAdd(a.nleft, 1u);
      a.left[k] = SmallEnt{gb, sz, x};
    }
  }
}

// Pairs: buckets handed on -- stable radix sort in LDS, or the next level /
// fallback when larger than one work-group.
template <int KW, int VW>
__global__ void __launch_bounds__(NT) k_bucket_leftover_pairs(LevelArgs a) {
  using KT = typename KeyOf<KW>::T;
  constexpr uint32_t C = SmallCap<KW, VW>::C;
  __shared__ SmallLds<KW, VW, SmallCap<KW, VW>::KMAX> sm;
  const uint32_t nl = *a.nleft;
  for (uint32_t li = blockIdx.x; li < nl; li += gridDim.x) {
    const SmallEnt e = a.left[li];
    if (e.len <= C) {
      sort_small<KW, VW>((const KT*)a.dst, a.vdst, (KT*)a.out, a.vout, e.beg, e.len, 0, 0, a.kout, sm);
      if (threadIdx.x == 0) atomicAdd((unsigned long long*)&a.ctl->bucket_keys, (unsigned long long)e.len);
      continue;
    }
    const LevelCtl c = *a.ctl;
    const uint32_t si = find_seg(a.segs, c.nsegs, e.pad, [](const SegDesc& d) { return (uint64_t)d.bkt_off; });
    const SegDesc d = a.segs[si];
    bucket_overflow<KW, VW>(a, d, e.pad - d.bkt_off, e.beg, e.len, sm);
    __syncthreads();
  }
}

// ---------------------------------------------------- stable split

// Stable split (step 4) of pairs into at most 256 buckets without a sort of
// the chunk: wave w takes the contiguous keys [w*R*64, (w+1)*R*64) of the
// chunk as R rows of 64.  Inside a row, the lanes with the same bucket are
// found with one ballot per bucket bit, so a key's rank among them is the
// number of such lanes before it; a per-wave counter per bucket, advanced
// row by row, adds the earlier rows.  The waves' counts then give each
// wave's offset inside each bucket's run, so every key's position follows
// input order (stability); the chunk is grouped by bucket in LDS and every
// bucket's run is written contiguously.
// rows per wave in a chunk: 6 for 8-byte keys (3072 pairs, whose LDS then
// allows three work-groups per CU), 8 for 4-byte keys (measured faster)
template <int KW> struct PairsChunk {
  static constexpr int R = KW == 8 ? 6 : 8;
  static constexpr int CH = R * NT;          // keys per chunk
  static constexpr int WPE = KW == 8 ? 6 : 1;   // waves per SIMD the kernel is built for (1: no bound)
};
constexpr int PAIRS_WAVES = NT / WAVE;

template <int KW, int VW>
struct ScatterPairsLds {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  TreeLds<KW, 256> tr;
  uint32_t wcnt[PAIRS_WAVES][256];           // per-wave running counts, then the waves' offsets
  uint32_t gofs[256];                        // before the first chunk: in-segment position of each
                                             // bucket's run; then that position - chunk position
  uint32_t tot[256];                         // keys of each bucket in the chunk
  KT sk[PairsChunk<KW>::CH];
  VT sv[PairsChunk<KW>::CH];
  uint8_t sb[PairsChunk<KW>::CH];
  alignas(8) uint32_t red[32];
};

// (8-byte keys: six waves per SIMD, three work-groups per CU with a 4-byte
// payload, whose chunk takes 53 KB of LDS)
template <int KW, int VW>
__global__ void __launch_bounds__(NT, PairsChunk<KW>::WPE) k_scatter_pairs(LevelArgs a) {
  using KT = typename KeyOf<KW>::T;
  using VT = typename ValOf<VW>::T;
  constexpr int R = PairsChunk<KW>::R;
  constexpr int PAIRS_CH = PairsChunk<KW>::CH;
  __shared__ ScatterPairsLds<KW, VW> sm;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const LevelCtl c = *a.ctl;
  if (tile >= c.total_tiles) return;
  const uint32_t si = find_seg(a.segs, c.nsegs, tile, [](const SegDesc& d) { return (uint64_t)d.tile_off; });
  const SegDesc d = a.segs[si];
  const uint32_t tw = tile - d.tile_off;
  const int t = threadIdx.x, w = wave_id(), ln = lane_id();
  sm.tr.load(a.tree, a.tree_tag, d.tree_off, d.p);
  const uint32_t base = a.hist[d.hist_off];
  for (uint32_t b = t; b < 256; b += NT) {
    sm.gofs[b] = b < d.p ? a.hist[d.hist_off + (uint64_t)b * d.ntiles + tw] - base : 0u;
    for (int v = 0; v < PAIRS_WAVES; v++) sm.wcnt[v][b] = 0;
  }
  __syncthreads();
  const uint32_t t0 = tw * a.tile;
  const uint32_t t1 = min(t0 + a.tile, d.len);
  const KT* src = (const KT*)a.src + d.beg;
  const VT* vsrc = (const VT*)a.vsrc;
  KT* dst = (KT*)a.dst + d.beg;
  VT* vdst = (VT*)a.vdst + d.beg;
  const uint32_t nbits = d.lgp + 1;          // bucket p marks keys past the end of the tile
  for (uint32_t c0 = t0; c0 < t1; c0 += PAIRS_CH) {
    const uint32_t cn = min((uint32_t)PAIRS_CH, t1 - c0);
    KT key[R];
    VT val[R];
    uint32_t tag[R], bk[R], off[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const uint32_t i = (uint32_t)(w * R + r) * WAVE + ln;   // chunk position: wave, row, lane
      tag[r] = c0 + i;
      key[r] = 0;
      val[r] = 0;
      if (i < cn) {
        key[r] = to_ord(src[c0 + i], a.kin);
        val[r] = a.iota ? (VT)(c0 + i) : vsrc[d.beg + c0 + i];
      }
    }
    sm.tr.template classify_many<R>(key, tag, d.lgp, d.p, bk);
    // rank among the lanes of the row with the same bucket, plus the wave's
    // earlier rows of that bucket
#pragma unroll
    for (int r = 0; r < R; r++) {
      const uint32_t i = (uint32_t)(w * R + r) * WAVE + ln;
      const uint32_t b = i < cn ? bk[r] : d.p;
      uint64_t peers = ~0ull;
      for (uint32_t bit = 0; bit < nbits; bit++) {
        const bool on = (b >> bit) & 1u;
        const uint64_t m = __ballot(on);
        peers &= on ? m : ~m;
      }
      const uint32_t rank = lane_rank(peers);
      uint32_t o = 0;
      if (b < d.p) {
        o = sm.wcnt[w][b];
        if (rank == 0) sm.wcnt[w][b] = o + (uint32_t)__popcll(peers);
      }
      off[r] = o + rank;
      bk[r] = b;
    }
    __syncthreads();
    // per bucket: the waves' offsets, the chunk total, then chunk starts
    {
      constexpr int PER = (256 + NT - 1) / NT;
      uint32_t v[PER], sum = 0;
#pragma unroll
      for (int j = 0; j < PER; j++) {
        const uint32_t b = t * PER + j;
        uint32_t run = 0;
        if (b < 256) {
          for (int ww = 0; ww < PAIRS_WAVES; ww++) {
            const uint32_t x = sm.wcnt[ww][b];
            sm.wcnt[ww][b] = run;
            run += x;
          }
        }
        v[j] = run;
        sum += run;
      }
      uint32_t total;
      uint32_t cs = block_excl_scan<NT>(sum, sm.red, &total);
#pragma unroll
      for (int j = 0; j < PER; j++) {
        const uint32_t b = t * PER + j;
        if (b < 256) {
          sm.tot[b] = cs;                    // chunk start of the bucket
          sm.gofs[b] -= cs;                  // output position - chunk position
        }
        cs += v[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++) {
      const uint32_t b = bk[r];
      if (b < d.p) {
        const uint32_t pos = sm.tot[b] + sm.wcnt[w][b] + off[r];
        sm.sk[pos] = key[r];
        sm.sv[pos] = val[r];
        sm.sb[pos] = (uint8_t)b;
      }
    }
    __syncthreads();
    for (uint32_t j = t; j < cn; j += NT) {
      const uint32_t g = sm.gofs[sm.sb[j]] + j;
      dst[g] = sm.sk[j];
      vdst[g] = sm.sv[j];
    }
    __syncthreads();
    // next chunk: each bucket's run continues after this chunk's keys
    // (chunk start + total = next bucket's chunk start), counters from zero
    for (uint32_t b = t; b < 256; b += NT) {
      const uint32_t nx = (b + 1 < 256) ? sm.tot[b + 1] : cn;
      sm.gofs[b] += nx;
      for (int v = 0; v < PAIRS_WAVES; v++) sm.wcnt[v][b] = 0;
    }
    __syncthreads();
  }
}

}  // namespace ss
