// Host side of the sample sort: argument checks, the plan (effective p,
// sample size, split levels, workspace layout) and the launch sequence.
// Every entry point only enqueues kernels on the caller's stream; nothing
// here allocates device memory or waits for the GPU (except ss_status).
#include "../../include/samplesort.h"
#include "ss_kernels.h"
#include "ss_wide.h"
#include "ss_pairs.h"
#include "ss_sortfirst.h"
#include "ss_tuned.h"
#include "ss_strings.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

using namespace ss;

namespace {

thread_local char g_err[512];

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(x)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) return fail(SS_EHIP, "%s: %s", #x, hipGetErrorString(e_));    \
  } while (0)
#define LAUNCH_CHECK()                                                                  \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess) return fail(SS_EHIP, "launch: %s", hipGetErrorString(e_));    \
  } while (0)

// ---------------------------------------------------------------- profiling
enum ProfKind {
  PK_INIT, PK_PLAN, PK_SAMPLE, PK_SAMPLE_SORT, PK_SAMPLE_MERGE, PK_TREE, PK_CLASSIFY, PK_SCAN, PK_SCATTER,
  PK_BUCKET_SORT, PK_BUCKET_LEFT, PK_SMALL_SORT, PK_BLOCK_SORT_REGULAR, PK_GRAD, PK_SPLIT_COARSE, PK_SPLIT_FINE,
  PK_SF_SEARCH, PK_SF_GATHER, PK_WIDEN, PK_COUNT
};
const char* const PROF_NAMES[PK_COUNT] = {
    "init", "plan", "sample", "sample_sort", "sample_merge", "tree", "classify", "scan", "scatter",
    "bucket_sort", "bucket_leftover", "small_sort", "regular_blocks", "scatter_grad", "split_coarse",
    "split_fine", "sf_search", "sf_gather", "widen"};

// The profiling state is shared by every host thread: `on` is read without
// the lock on each launch (so sorts cost nothing extra while profiling is
// off); everything else is touched under `mu`.
struct Prof {
  std::atomic<bool> on{false};
  std::mutex mu;
  uint32_t mask = ~0u;              // kinds that get events
  int cap = 0, used = 0;
  std::vector<hipEvent_t> ev;       // 2 per launch
  std::vector<int> kind;
  double total[PK_COUNT] = {};
  uint64_t count[PK_COUNT] = {};
  void reset() {
    mask = ~0u;
    cap = used = 0;
    ev.clear();
    kind.clear();
    for (int i = 0; i < PK_COUNT; i++) total[i] = 0.0, count[i] = 0;
  }
};
Prof g_prof;
// kind every launch of this thread counts as (a nested sort's launches), or -1
thread_local int g_prof_force = -1;

// bracket one launch with events (no-op unless profiling is on)
struct ProfScope {
  int slot = -1;
  hipStream_t st;
  ProfScope(int k, hipStream_t s) : st(s) {
    if (!g_prof.on.load(std::memory_order_acquire)) return;
    if (g_prof_force >= 0) k = g_prof_force;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.on.load(std::memory_order_relaxed) || !((g_prof.mask >> k) & 1u) || g_prof.used >= g_prof.cap)
      return;
    slot = g_prof.used++;
    g_prof.kind[slot] = k;
    (void)hipEventRecord(g_prof.ev[2 * slot], st);
  }
  ~ProfScope() {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (slot < (int)g_prof.kind.size()) (void)hipEventRecord(g_prof.ev[2 * slot + 1], st);
  }
};
#define LAUNCH(kind, ...)                 \
  do {                                    \
    ProfScope prof_scope_((kind), st);    \
    hipLaunchKernelGGL(__VA_ARGS__);      \
  } while (0)

struct Types {
  int kt = 0, vt = 0;
  int KW = 4, VW = 0;
  int kind = 0;     // 0 unsigned, 1 signed, 2 float
  bool iota = false;
};

int parse_types(int kt, int vt, Types* ty) {
  if (kt < SS_U32 || kt > SS_F64) return fail(SS_EINVAL, "unknown key_type %d", kt);
  ty->kt = kt;
  ty->vt = vt;
  ty->KW = kt <= SS_F32 ? 4 : 8;
  ty->kind = (kt == SS_U32 || kt == SS_U64) ? 0 : ((kt == SS_I32 || kt == SS_I64) ? 1 : 2);
  switch (vt) {
    case SS_V_NONE: ty->VW = 0; ty->iota = false; break;
    case SS_V_B32: ty->VW = 4; ty->iota = false; break;
    case SS_V_B64: ty->VW = 8; ty->iota = false; break;
    case SS_V_IOTA32: ty->VW = 4; ty->iota = true; break;
    case SS_V_IOTA64: ty->VW = 8; ty->iota = true; break;
    default: return fail(SS_EINVAL, "unknown val_type %d", vt);
  }
  return SS_OK;
}

uint32_t small_cap(int KW, int VW) {
  int s = KW + VW;
  return (uint32_t)NT * (s <= 4 ? 64 : (s <= 8 ? 32 : 16));
}
uint32_t sample_cap(int KW) { return (uint32_t)NT * (KW == 4 ? 32 : 16); }
uint32_t sample_chunk(int KW) { return KW == 4 ? (uint32_t)SampleChunk<4>::C : (uint32_t)SampleChunk<8>::C; }
// keys-only buckets up to this size are sorted by the slot sort
uint32_t slot_cap(int KW) { return KW == 4 ? (uint32_t)SlotCap<4>::C : (uint32_t)SlotCap<8>::C; }
uint32_t split_chunk(int KW, int VW) { return (uint32_t)NT * ((KW + VW <= 4) ? 8 : 4); }

constexpr size_t ALIGN = 256;
struct Layout {
  size_t cur = 0;
  size_t take(size_t bytes) {
    size_t o = (cur + ALIGN - 1) & ~(ALIGN - 1);
    cur = o + bytes;
    return o;
  }
};

uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Largest bucket of a random split relative to the mean, as a planning
// estimate (the levels below are sized from it; a larger bucket is still
// sorted correctly, by the next level or the one-work-group fallback).
double spread(uint32_t s) { return 1.0 + 4.0 / std::sqrt((double)std::max(1u, s)); }

// Effective bucket count: the largest power of two <= p with p <= n
// (Theorem 1) and p*s < n/2 (Claim 1, random) or 4*s*p^2 <= n (regular).
uint32_t p_effective(uint64_t n, uint32_t p, uint32_t s, int mode) {
  uint64_t q = 1;
  while (q * 2 <= p) q *= 2;
  for (; q >= 2; q /= 2) {
    if (q > n) continue;
    if (mode == SS_RANDOM) {
      if (2 * q * (uint64_t)s < n) return (uint32_t)q;
    } else {
      if (4 * (uint64_t)s * q * q <= n) return (uint32_t)q;
    }
  }
  return 1;
}

// Tiles are whole multiples of 8192 keys (the split chunk and id block of
// every key width).
constexpr uint32_t TILE_UNIT = 8192;
// capacity (LDS tree and counters) of the split kernels for a level whose
// segments take up to p buckets: the smallest instantiated bound >= p
uint32_t pmax_for(uint32_t p) { return p <= 256 ? 256 : (p <= 512 ? 512 : (p <= 1024 ? 1024 : 4096)); }

uint32_t default_tile(uint32_t p) {
  uint64_t t = std::max<uint64_t>(65536, 16ull * p);
  return (uint32_t)(cdiv(t, TILE_UNIT) * TILE_UNIT);
}

// ------------------------------------------------------- tuned parameters
//
// What a call with prm == NULL uses, per size class: class c holds lengths
// in (2^(c-1), 2^c] (c = ceil(lg n)), per form (single array, segmented),
// key width (4, 8) and payload width as sorted (0, 4, 8; a 64-bit index is
// sorted as a 4-byte one).  The paper chooses p for the machine after
// calibration (Section 2.1, Section 3); here the table holds what a tuning
// run on an MI355X measured fastest, and ss_set_tuning replaces it with a
// newer run's.  In the segmented table p = 0 means "sized from the
// segment's length" (buckets of about half what one work-group sorts).
struct TuneTab {
  uint16_t p[33], s[33];
  uint32_t tile[33];
};
TuneTab g_tune[2][2][3];   // [form][key width 4, 8][payload 0, 4, 8]
bool g_tune_ready = false;
std::mutex g_tune_mu;

int size_class(uint64_t n) {
  int c = 0;
  while (c < 32 && (1ull << c) < n) c++;
  return c;
}

// Built-in table: the measured entries of ss_tuned.h over a rule for the
// groups no run measured.  Rule: single arrays, keys only, buckets of ~16K
// 4-byte keys (p up to 4096), ~8K 8-byte keys (p up to 1024); with a
// payload p <= 256 (the stable ballot split); s = 16.  Segmented: p from
// the length, s = 8.
void tune_builtin(TuneTab (&t)[2][2][3]) {
  for (int kw = 0; kw < 2; kw++)
    for (int vw = 0; vw < 3; vw++)
      for (int c = 0; c <= 32; c++) {
        uint32_t p;
        if (vw == 0 && kw == 0) p = c > 15 ? (1u << std::min(c - 14, 12)) : 2u;
        else if (vw == 0) p = c > 14 ? (1u << std::min(c - 13, 10)) : 2u;
        else p = c > 14 ? (1u << std::min(c - 13, 8)) : 2u;
        t[0][kw][vw].p[c] = (uint16_t)std::max<uint32_t>(p, 2);
        t[0][kw][vw].s[c] = 16;
        t[0][kw][vw].tile[c] = 0;
        t[1][kw][vw].p[c] = 0;
        t[1][kw][vw].s[c] = 8;
        t[1][kw][vw].tile[c] = 0;
      }
  for (const auto& e : TUNED) {
    TuneTab& tt = t[e[0]][e[1] == 8][e[2] == 0 ? 0 : (e[2] == 4 ? 1 : 2)];
    tt.p[e[3]] = (uint16_t)e[4];
    tt.s[e[3]] = (uint16_t)e[5];
    tt.tile[e[3]] = e[6];
  }
}

const TuneTab& tune_for(int form, int KW, int VW) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_ready) {
    tune_builtin(g_tune);
    g_tune_ready = true;
  }
  return g_tune[form][KW == 8 ? 1 : 0][VW == 0 ? 0 : (VW == 4 ? 1 : 2)];
}

// payload width as sorted (a 64-bit index travels as a 32-bit one)
int sorted_vw(const Types& ty) { return (ty.iota && ty.VW == 8) ? 4 : ty.VW; }

struct LevelPlan {
  uint32_t tile = 0, seg_cap = 0, pmax = 256, p_cap = 256, target = 0, s = 1;
  uint64_t samp_cap = 0, tiles_cap = 0, hist_cap = 0, bkt_cap = 0;
  size_t o_segs = 0, o_sord = 0, o_stag = 0, o_tree = 0, o_ttag = 0, o_hist = 0, o_part = 0, o_left = 0, o_left2 = 0;
};

struct LevelsPlan {
  int nlev = 0;
  LevelPlan lv[MAX_LEVELS];
  bool big_sample = false;  // top level sample larger than one work-group (single segment only)
};

// Shapes of the split levels.  Level 0 either has one segment with given p0
// and sample size m0 (single sort) or up to seg_cap0 segments sized on the
// device (p0 == 0).  N = total elements, maxlen0 = longest top segment.
// Segments sized on the device take p and s from the tuning table `tab`
// (when given): the level's target bucket size is then the smallest that a
// tuned class asks for, so that the table's p never exceeds what the
// target rule would give (the capacities below are sized by that rule),
// and the expected largest bucket follows the table class by class.
uint32_t tab_target(const TuneTab& tab, uint32_t C, uint64_t maxlen, uint32_t target) {
  for (int c = size_class((uint64_t)C + 1); c <= size_class(maxlen); c++) {
    if (!tab.p[c]) continue;
    const uint64_t b = (c ? (1ull << (c - 1)) : 1ull) / tab.p[c];
    target = (uint32_t)std::min<uint64_t>(target, std::max<uint64_t>(b, 256));
  }
  return target;
}

void plan_levels(Layout& L, const Types& ty, uint64_t N, uint64_t seg_cap0, uint64_t maxlen0, uint32_t p0,
                 uint64_t m0, uint64_t est_max0, uint32_t s, uint32_t p_cap, uint32_t tile_req, bool recurse,
                 LevelsPlan* P, uint32_t cpush0 = 0, const TuneTab* tab = nullptr) {
  const uint32_t C = small_cap(ty.KW, ty.VW);
  // buckets larger than this go one level down when there is a level below
  // (keys only: beyond the slot sort's capacity)
  const uint32_t Cpush = ty.VW == 0 ? slot_cap(ty.KW) : C;
  const uint32_t Cs = sample_cap(ty.KW);
  double f = spread(s);
  // automatically sized buckets aim at about half of what the bucket sort
  // takes in one work-group (the slot sort for keys only)
  uint32_t target = ty.VW == 0 ? (uint32_t)(0.53 * slot_cap(ty.KW))
                               : (uint32_t)std::max(1024.0, (double)C / (1.2 * f));
  if (tab) {
    target = tab_target(*tab, C, maxlen0, target);
    for (int c = size_class((uint64_t)C + 1); c <= size_class(maxlen0); c++)
      f = std::max(f, spread(tab->s[c] ? tab->s[c] : s));
  }
  // expected largest bucket after splitting segments of up to `len` keys
  auto after = [&](uint64_t len) -> uint64_t {
    double b = std::max<double>(target, (double)len / p_cap);
    if (tab)
      for (int c = size_class((uint64_t)C + 1); c <= size_class(len); c++)
        if (tab->p[c]) b = std::max(b, std::min<double>((double)len, (double)(1ull << c)) / std::max<uint32_t>(tab->p[c], 2));
    return (uint64_t)(b * f);
  };
  P->nlev = 0;
  uint64_t est = 0;
  for (int l = 0; l < MAX_LEVELS; l++) {
    LevelPlan& lv = P->lv[l];
    lv.s = s;
    lv.target = target;
    if (l == 0 && p0) {
      lv.p_cap = p0;
      lv.pmax = pmax_for(p0);
      lv.tile = tile_req ? (uint32_t)(cdiv(tile_req, TILE_UNIT) * TILE_UNIT) : default_tile(p0);
      lv.seg_cap = 1;
      lv.samp_cap = m0;
      lv.tiles_cap = cdiv(N, lv.tile);
      lv.hist_cap = (uint64_t)p0 * lv.tiles_cap;
      lv.bkt_cap = p0;
      est = est_max0;
    } else {
      lv.p_cap = p_cap;
      lv.pmax = pmax_for(p_cap);
      lv.tile = tile_req ? (uint32_t)(cdiv(tile_req, TILE_UNIT) * TILE_UNIT) : default_tile(p_cap);
      uint64_t sc = (l == 0) ? seg_cap0 : std::min<uint64_t>(P->lv[l - 1].bkt_cap, N / (Cpush + 1) + 1);
      sc = std::min<uint64_t>(sc, N / (Cpush + 1) + 1);
      lv.seg_cap = (uint32_t)std::max<uint64_t>(sc, 1);
      lv.tiles_cap = N / lv.tile + lv.seg_cap + 1;
      lv.bkt_cap = std::min<uint64_t>((uint64_t)lv.seg_cap * p_cap, 2 * N / target + 2ull * lv.seg_cap + 2);
      lv.hist_cap = (uint64_t)p_cap * lv.tiles_cap;
      lv.samp_cap = std::min<uint64_t>((uint64_t)Cs * lv.seg_cap, (uint64_t)s * lv.bkt_cap);
      uint64_t len = (l == 0) ? maxlen0 : est;
      est = after(len);
    }
    lv.o_segs = L.take(sizeof(SegDesc) * lv.seg_cap);
    lv.o_sord = L.take((size_t)ty.KW * std::max<uint64_t>(lv.samp_cap, 1));
    lv.o_stag = L.take(4 * std::max<uint64_t>(lv.samp_cap, 1));
    lv.o_tree = L.take(8 * std::max<uint64_t>(lv.bkt_cap, 1));
    lv.o_ttag = (ty.KW == 8) ? L.take(4 * std::max<uint64_t>(lv.bkt_cap, 1)) : 0;
    lv.o_hist = L.take(4 * std::max<uint64_t>(lv.hist_cap, 1));
    lv.o_part = L.take(4 * (cdiv(std::max<uint64_t>(lv.hist_cap, 1), SCAN_BLOCK) + 1));
    lv.o_left = L.take(sizeof(SmallEnt) * std::max<uint64_t>(lv.bkt_cap, 1));
    lv.o_left2 = L.take(sizeof(SmallEnt) * std::max<uint64_t>(lv.bkt_cap, 1));
    if (l == 0 && p0 && m0 > Cs) P->big_sample = true;
    P->nlev = l + 1;
    // the top level of a single sort has a caller-chosen p, so its buckets
    // may well exceed the slot sort; deeper levels pick p for the target
    // size, and only a rare tail exceeds it: those take the radix sort
    // (cpush0: the top level's own bucket sort capacity, when it has one)
    if (!recurse || est <= ((l == 0 && p0) ? (cpush0 ? cpush0 : Cpush) : C)) break;
  }
}

// Full plan of one call.
struct Plan {
  Types ty;
  uint64_t n = 0;          // elements (single) / index range end (segmented)
  ss_params prm{};
  bool segmented = false;
  uint64_t nseg = 0, maxlen = 0;
  bool direct = false;     // n fits one work-group
  bool whole = false;      // no valid p: one work-group sorts everything
  uint32_t p_eff = 1, s = 1, stride = 1;
  uint64_t m = 0;
  bool regular = false;
  LevelsPlan lp;
  size_t o_ctl = 0, o_tmp = 0, o_vtmp = 0;
  size_t o_exp_so = 0, o_exp_st = 0, o_exp_po = 0, o_exp_pt = 0, o_exp_cnt = 0;
  bool exp = false;
  size_t o_small = 0, o_tiny = 0, o_mid = 0;   // segmented: lists of segments below one level
  size_t o_small_fb = 0;                       // small segments handed from the stable slot sort to the radix sort
  // regular sampling: sorted blocks and the nested segmented plan
  size_t o_regk = 0, o_regi = 0, o_regoff = 0, o_nested = 0;
  Plan* nested = nullptr;
  // wide split (keys only, 4-byte keys, p >= 1024): count arrays and their scan partials
  bool wide = false;
  uint32_t wide_W = 0;
  size_t o_whf = 0, o_whf_part = 0, o_wha = 0, o_wha_part = 0, o_wkeys = 0, o_wtags = 0, o_wcells = 0, o_whdr = 0;
  size_t o_wcb = 0;        // coarse region of every key
  size_t o_tmp2 = 0;       // wide split with input == output: a second copy
  // sort-first organisation: sorted blocks (o_regk, o_regi), the run table and the buckets
  bool sortfirst = false;
  size_t o_sfpos = 0, o_sfbkt = 0;
  // sort-first with 8-byte keys or a payload: the gathered buckets, sorted as segments
  Plan* nested_b = nullptr;
  size_t o_sfoff = 0, o_nested_b = 0;
  // a large sample of 4-byte keys: packed records and the nested sort that orders them
  Plan* nested_s = nullptr;
  size_t o_spack = 0, o_nested_s = 0;
  size_t o_scnt = 0;       // 4-byte big sample ranked by chunk pairs: the counts
  // segmented without user parameters: the tuning table's p and s per size class
  bool use_tab = false;
  TuneTab tab{};
  // a 64-bit index payload sorted as a 32-bit one, then widened
  bool widen = false;
  size_t o_widen = 0;
  size_t bytes = 0;
  ~Plan() {
    delete nested;
    delete nested_s;
    delete nested_b;
  }
};

int check_params(const ss_params* prm, ss_params* out, const Types& ty, uint64_t n, int form = 0) {
  ss_params d{};
  d.sampling = SS_RANDOM;
  d.stable = 1;
  d.seed = 0x5EEDull;
  {
    const TuneTab& t = tune_for(form, ty.KW, sorted_vw(ty));
    const int c = size_class(n);
    d.p = t.p[c] ? t.p[c] : 256;    // (segmented p = 0: sized on the device, at most 256)
    d.s = t.s[c];
    d.tile = t.tile[c];
  }
  if (prm) d = *prm;
  if (d.p < 2 || d.p > SS_P_MAX || (d.p & (d.p - 1))) return fail(SS_EINVAL, "p = %u: need a power of two in [2, %u]", d.p, SS_P_MAX);
  if (d.s < 1 || d.s > 4096) return fail(SS_EINVAL, "s = %u: need 1 <= s <= 4096", d.s);
  if (d.sampling != SS_RANDOM && d.sampling != SS_REGULAR) return fail(SS_EINVAL, "unknown sampling rule %d", d.sampling);
  *out = d;
  return SS_OK;
}

int plan_segmented(Plan* P, uint64_t total, uint64_t nseg, uint64_t maxlen, const Types& ty, const ss_params& prm,
                   bool user_params);

int plan_single(Plan* P, uint64_t n, const Types& ty, const ss_params& prm);

int plan_single_t(Plan* P, uint64_t n, const Types& ty, const ss_params& prm) {
  P->ty = ty;
  P->n = n;
  P->prm = prm;
  if (n >= (1ull << 32)) return fail(SS_EINVAL, "n = %llu: at most 2^32-1 keys per array", (unsigned long long)n);
  if ((prm.flags & SS_F_SF_MERGE) && (prm.flags & SS_F_SORT_FIRST) && !(ty.KW == 4 && ty.VW == 0))
    return fail(SS_EINVAL, "SS_F_SF_MERGE: 4-byte keys without payload only");
  const uint32_t C = small_cap(ty.KW, ty.VW);
  Layout L;
  P->o_ctl = L.take(sizeof(Ctl));
  P->regular = prm.sampling == SS_REGULAR;
  P->p_eff = p_effective(n, prm.p, prm.s, prm.sampling);
  P->direct = (n <= C && !(prm.flags & SS_F_FORCE_PIPELINE)) || n < 2;
  if (!P->direct && P->p_eff < 2) P->whole = true;
  if (P->direct || P->whole) {
    P->p_eff = 1;
    P->regular = false;
    if (P->whole) {
      P->o_tmp = L.take((size_t)ty.KW * n);
      P->o_vtmp = ty.VW ? L.take((size_t)ty.VW * n) : 0;
    }
    P->bytes = L.cur;
    return SS_OK;
  }
  const uint32_t p = P->p_eff;
  P->s = prm.s;
  P->sortfirst = (prm.flags & SS_F_SORT_FIRST) != 0;
  if (P->sortfirst && p > SF_PMAX) return fail(SS_EINVAL, "SS_F_SORT_FIRST: p = %u, at most %u", p, SF_PMAX);
  uint64_t est;
  if (P->regular) {
    P->m = (uint64_t)prm.s * p * p;
    P->stride = prm.s * p;
    // Lemma 1: no bucket exceeds (S + p) * x, S = s*p, x = ceil(ceil(n/p)/S)
    uint64_t S = (uint64_t)prm.s * p, x = cdiv(cdiv(n, p), S);
    est = (S + p) * x;
  } else {
    P->m = (uint64_t)p * prm.s - 1;
    P->stride = prm.s;
    est = (uint64_t)((double)n / p * spread(prm.s));
  }
  P->exp = (prm.flags & SS_F_EXPORT_STAGES) != 0;
  if (P->exp) {
    P->o_exp_so = L.take(8 * P->m);
    P->o_exp_st = L.take(8 * P->m);
    P->o_exp_po = L.take(8 * (p - 1));
    P->o_exp_pt = L.take(8 * (p - 1));
    P->o_exp_cnt = L.take(8 * p);
  }
  P->o_tmp = L.take((size_t)ty.KW * n);
  P->o_vtmp = ty.VW ? L.take((size_t)ty.VW * n) : 0;
  bool recurse = !(prm.flags & SS_F_NO_RECURSION) && !P->sortfirst;
  // wide split: many buckets of keys only; buckets beyond the round-based
  // slot sort's 65535 keys go one level down
  P->wide = ty.VW == 0 && ty.KW == 4 && p >= 1024 && p <= (uint32_t)WIDE_PMAX && !(prm.flags & SS_F_NO_WIDE) &&
            !P->sortfirst;
  if (P->wide) {
    const uint64_t W = cdiv(n, WIDE_TILE);
    P->wide_W = (uint32_t)W;
    const uint64_t nf = (uint64_t)p * (W + 2) + 1, na = (uint64_t)WIDE_P1 * W + 1;
    P->o_whf = L.take(4 * nf);
    P->o_whf_part = L.take(4 * (cdiv(nf, SCAN_BLOCK) + 1));
    P->o_wha = L.take(4 * na);
    P->o_wha_part = L.take(4 * (cdiv(na, SCAN_BLOCK) + 1));
    P->o_wkeys = L.take(4 * (size_t)p);
    P->o_wtags = L.take(4 * (size_t)p);
    P->o_wcells = L.take(4 * ((size_t)WIDE_CELLS + 1));
    P->o_whdr = L.take(sizeof(WideHdr));
    P->o_wcb = L.take(W * WIDE_TILE);   // (whole chunks: one 8-byte word per thread per chunk)
  }
  // (the wide split's bucket sort takes any size in rounds; a level below
  // pays once buckets would need many rounds)
  plan_levels(L, ty, n, 1, n, p, P->m, est, prm.s, 256, prm.tile, recurse, &P->lp, P->wide ? WIDE_LEVEL_MIN : 0);
  // with input == output the wide split's first pass needs a buffer of its
  // own: the stage, or the fine buckets (which a bucket sort of several
  // rounds re-reads while it writes the output)
  if (P->wide) P->o_tmp2 = L.take((size_t)ty.KW * n);
  if (ty.KW == 4 && P->lp.big_sample && P->m >= SAMPLE_NESTED_MIN) {
    // the sample's records (ord key, tag) become 64-bit keys ord << 32 | tag,
    // whose order is the records' order, and are sorted by a nested sort
    Types st;
    parse_types(SS_U64, SS_V_NONE, &st);
    ss_params sp = prm;
    sp.p = 256;
    sp.s = 16;
    sp.sampling = SS_RANDOM;
    sp.flags = 0;
    sp.tile = 0;
    sp.seed = prm.seed ^ 0x5A3C96E1D2B4F087ull;
    P->nested_s = new Plan();
    int rc = plan_single(P->nested_s, P->m, st, sp);
    if (rc) return rc;
    P->o_spack = L.take(8 * P->m);
    P->o_nested_s = L.take(P->nested_s->bytes);
  } else if (ty.KW == 4 && P->lp.big_sample) {
    // the sorted chunks' records also packed as ord << 32 | tag, for the rank
    // pass; up to SAMPLE_PAIR_MAXCH chunks, 16-bit counts per (chunk, record)
    P->o_spack = L.take(8 * P->m);
    const uint64_t nch = cdiv(P->m, sample_chunk(4));
    if (nch <= SAMPLE_PAIR_MAXCH) P->o_scnt = L.take(2 * nch * P->m);
  }
  if (P->sortfirst) {
    P->o_sfpos = L.take(4 * (size_t)p * (p + 1));
    P->o_sfbkt = L.take(8 * (size_t)p);
    if (!(ty.KW == 4 && ty.VW == 0)) {
      // step 5 gathers each bucket's runs with their payloads (an index
      // payload becomes a stored one), then sorts the p buckets as segments
      // of any length up to n
      Types gt = ty;
      gt.iota = false;
      gt.vt = ty.VW == 0 ? SS_V_NONE : (ty.VW == 4 ? SS_V_B32 : SS_V_B64);
      ss_params gp = prm;
      gp.sampling = SS_RANDOM;
      gp.flags &= SS_F_NO_RECURSION;
      P->nested_b = new Plan();
      int rc = plan_segmented(P->nested_b, n, p, n, gt, gp, false);
      if (rc) return rc;
      P->o_sfoff = L.take(8 * ((size_t)p + 1));
      P->o_nested_b = L.take(P->nested_b->bytes);
    }
  }
  if (P->regular || P->sortfirst) {
    // blocks sorted with their in-block index as payload (Alg. 1 step 1)
    P->o_regk = L.take((size_t)ty.KW * n);
    P->o_regi = L.take(4 * n);
    P->o_regoff = L.take(8 * (p + 1));
    Types bt = ty;
    bt.vt = SS_V_IOTA32;
    bt.VW = 4;
    bt.iota = true;
    P->nested = new Plan();
    ss_params bp = prm;
    bp.sampling = SS_RANDOM;
    bp.flags &= SS_F_NO_RECURSION;
    int rc = plan_segmented(P->nested, n, p, cdiv(n, p), bt, bp, false);
    if (rc) return rc;
    P->o_nested = L.take(P->nested->bytes);
  }
  P->bytes = L.cur;
  return SS_OK;
}

int plan_segmented_t(Plan* P, uint64_t total, uint64_t nseg, uint64_t maxlen, const Types& ty, const ss_params& prm,
                   bool user_params) {
  P->ty = ty;
  P->n = total;
  P->prm = prm;
  P->segmented = true;
  P->nseg = nseg;
  if (prm.flags & SS_F_SORT_FIRST) return fail(SS_EINVAL, "SS_F_SORT_FIRST: single arrays only");
  if (maxlen == 0 || maxlen > total) maxlen = total;
  P->maxlen = maxlen;
  if (maxlen >= (1ull << 32)) return fail(SS_EINVAL, "segments of 2^32 or more keys are not supported");
  if (nseg >= (1ull << 31)) return fail(SS_EINVAL, "too many segments");
  const uint32_t C = small_cap(ty.KW, ty.VW);
  Layout L;
  P->o_ctl = L.take(sizeof(Ctl));
  P->o_small = L.take(sizeof(SmallEnt) * std::max<uint64_t>(nseg, 1));
  P->o_small_fb = L.take(sizeof(SmallEnt) * std::max<uint64_t>(nseg, 1));
  P->o_tiny = L.take(sizeof(SmallEnt) * std::max<uint64_t>(nseg, 1));
  P->o_mid = L.take(sizeof(SmallEnt) * std::max<uint64_t>(nseg, 1));
  P->s = prm.s;
  // user parameters: prm->p caps every segment's buckets and prm->s
  // applies to all; otherwise p and s come from the tuning table per size
  // class of each segment
  uint32_t p_cap = std::min<uint32_t>(prm.p, 4096);
  const TuneTab* tab = nullptr;
  if (!user_params) {
    tab = &tune_for(1, ty.KW, ty.VW);
    p_cap = 2;
    for (int c = size_class((uint64_t)C + 1); c <= size_class(maxlen); c++)
      p_cap = std::max<uint32_t>(p_cap, tab->p[c] ? tab->p[c] : 256u);
    p_cap = std::min<uint32_t>(p_cap, 4096);
    P->tab = *tab;
    P->use_tab = true;
  }
  if (maxlen > C) {
    P->o_tmp = L.take((size_t)ty.KW * total);
    P->o_vtmp = ty.VW ? L.take((size_t)ty.VW * total) : 0;
    uint64_t seg_cap0 = std::min<uint64_t>(nseg, total / (C + 1) + 1);
    const bool recurse = !(prm.flags & SS_F_NO_RECURSION);
    plan_levels(L, ty, total, seg_cap0, maxlen, 0, 0, 0, prm.s, p_cap, prm.tile, recurse, &P->lp, 0, tab);
  }
  P->bytes = L.cur;
  return SS_OK;
}

template <int KW, int VW>
struct Launch;

// Bytes of an argument range, for overlap checks.
bool overlap_partial(const void* a, size_t an, const void* b, size_t bn) {
  if (!a || !b || !an || !bn) return false;
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  if (x == y && an == bn) return false;
  return x < y + bn && y < x + an;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// A 64-bit index payload (< 2^32 within an array or a segment) is sorted as
// a 32-bit one into the workspace and widened once at the end: every pass
// then moves 4 bytes less per element.
Types narrow_index(const Types& ty) {
  Types t = ty;
  t.VW = 4;
  t.vt = SS_V_IOTA32;
  return t;
}

void add_widen(Plan* P, uint64_t n) {
  Layout L;
  L.cur = P->bytes;
  P->o_widen = L.take(4 * std::max<uint64_t>(n, 1));
  P->bytes = L.cur;
  P->widen = true;
}

int plan_single(Plan* P, uint64_t n, const Types& ty, const ss_params& prm) {
  if (!(ty.iota && ty.VW == 8)) return plan_single_t(P, n, ty, prm);
  const int rc = plan_single_t(P, n, narrow_index(ty), prm);
  if (rc) return rc;
  add_widen(P, n);
  return SS_OK;
}

int plan_segmented(Plan* P, uint64_t total, uint64_t nseg, uint64_t maxlen, const Types& ty, const ss_params& prm,
                   bool user_params) {
  if (!(ty.iota && ty.VW == 8)) return plan_segmented_t(P, total, nseg, maxlen, ty, prm, user_params);
  const int rc = plan_segmented_t(P, total, nseg, maxlen, narrow_index(ty), prm, user_params);
  if (rc) return rc;
  add_widen(P, total);
  return SS_OK;
}

LevelArgs level_args(const Plan& P, char* ws, int l, const void* in, const void* vin, void* out, void* vout) {
  const LevelPlan& lv = P.lp.lv[l];
  LevelArgs a{};
  Ctl* g = (Ctl*)(ws + P.o_ctl);
  a.gctl = g;
  a.segs = (SegDesc*)(ws + lv.o_segs);
  a.ctl = &g->lv[l];
  a.seg_cap = lv.seg_cap;
  if (l + 1 < P.lp.nlev) {
    a.next_segs = (SegDesc*)(ws + P.lp.lv[l + 1].o_segs);
    a.next_ctl = &g->lv[l + 1];
    a.next_cap = P.lp.lv[l + 1].seg_cap;
  }
  void* tmp = ws + P.o_tmp;
  void* vtmp = P.ty.VW ? (void*)(ws + P.o_vtmp) : nullptr;
  // level 0 reads the input and writes tmp; deeper levels alternate tmp <-> out
  if (l == 0) {
    a.src = in;
    a.vsrc = P.ty.iota ? nullptr : vin;
    a.dst = tmp;
    a.vdst = vtmp;
  } else if (l % 2 == 1) {
    a.src = tmp;
    a.vsrc = vtmp;
    a.dst = out;
    a.vdst = vout;
  } else {
    a.src = out;
    a.vsrc = vout;
    a.dst = tmp;
    a.vdst = vtmp;
  }
  a.out = out;
  a.vout = vout;
  a.tmp = tmp;
  a.vtmp = vtmp;
  a.s_ord = ws + lv.o_sord;
  a.s_tag = (uint32_t*)(ws + lv.o_stag);
  a.s_pack = (l == 0 && P.ty.KW == 4 && P.lp.big_sample && !P.nested_s && P.o_spack)
                 ? (uint64_t*)(ws + P.o_spack) : nullptr;
  a.tree = ws + lv.o_tree;
  a.tree_tag = lv.o_ttag ? (uint32_t*)(ws + lv.o_ttag) : nullptr;
  a.hist = (uint32_t*)(ws + lv.o_hist);
  a.scan_part = (uint32_t*)(ws + lv.o_part);
  a.left = (SmallEnt*)(ws + lv.o_left);
  a.nleft = &g->nleft[l];
  a.left2 = (SmallEnt*)(ws + lv.o_left2);
  a.nleft2 = &g->nleft2[l];
  if (P.exp && l == 0) {
    a.exp_smp_ord = (uint64_t*)(ws + P.o_exp_so);
    a.exp_smp_tag = (uint64_t*)(ws + P.o_exp_st);
    a.exp_spl_ord = (uint64_t*)(ws + P.o_exp_po);
    a.exp_spl_tag = (uint64_t*)(ws + P.o_exp_pt);
    a.exp_counts = (uint64_t*)(ws + P.o_exp_cnt);
  }
  a.tile = lv.tile;
  a.s = lv.s;
  a.p_cap = lv.p_cap;
  a.target = lv.target;
  a.use_tab = P.use_tab ? 1u : 0u;
  if (P.use_tab)
    for (int c = 0; c <= 32; c++) {
      a.tab_p[c] = P.tab.p[c];
      a.tab_s[c] = P.tab.s[c];
    }
  a.kin = (l == 0) ? P.ty.kind : 0;   // the top level writes unsigned images for every deeper pass
  a.kout = P.ty.kind;
  a.iota = (l == 0 && P.ty.iota) ? 1 : 0;
  return a;
}

// scans of up to this many blocks per array skip the partials launch
constexpr uint32_t SCAN_SELF_MAX = 2048;

uint32_t grid_of(uint64_t work, uint32_t per, uint32_t cap) {
  uint64_t g = cdiv(std::max<uint64_t>(work, 1), per);
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(g, 1), cap);
}

// The wide split of a single keys-only sort (level 0 after its splitter
// tree): count, scans, two split passes, bucket sorts.  The keys travel
// input -> stage -> fine -> output.  With a level below, the fine buckets
// are always in the workspace copy tmp (where that level reads them);
// without one, input == output puts stage and fine buckets in the two
// workspace copies, so no pass reads what it writes.
int run_wide(const Plan& P, char* ws, LevelArgs a, const void* in, void* out, int exp, hipStream_t st) {
  WideArgs w{};
  const bool inplace = in == out;
  uint32_t* tmp = (uint32_t*)(ws + P.o_tmp);
  w.tree = (const uint64_t*)a.tree;
  w.hf = (uint32_t*)(ws + P.o_whf);
  w.ha = (uint32_t*)(ws + P.o_wha);
  w.src = in;
  if (P.lp.nlev > 1) {
    // the level below reads the fine buckets from tmp
    w.stage = inplace ? (uint32_t*)(ws + P.o_tmp2) : (uint32_t*)out;
    w.fine = tmp;
  } else {
    w.stage = inplace ? tmp : (uint32_t*)out;
    w.fine = inplace ? (uint32_t*)(ws + P.o_tmp2) : tmp;
  }
  w.out = out;
  w.n = (uint32_t)P.n;
  w.p = P.p_eff;
  w.lgp = 31 - __builtin_clz(P.p_eff);
  w.W = P.wide_W;
  w.tile = WIDE_TILE;
  w.skeys = (uint32_t*)(ws + P.o_wkeys);
  w.stags = (uint32_t*)(ws + P.o_wtags);
  w.cells = (uint32_t*)(ws + P.o_wcells);
  w.hdr = (WideHdr*)(ws + P.o_whdr);
  w.cb = (uint8_t*)(ws + P.o_wcb);
  w.kin = P.ty.kind;
  w.kout = P.ty.kind;
  // the leftover kernel sorts fine -> out (the stage is free scratch by then)
  a.dst = w.fine;
  a.out = out;
  a.tmp = w.stage;
  const uint64_t nf = (uint64_t)w.p * (w.W + 2) + 1, na = (uint64_t)WIDE_P1 * w.W + 1;
  uint32_t* pf = (uint32_t*)(ws + P.o_whf_part);
  uint32_t* pa = (uint32_t*)(ws + P.o_wha_part);
  LAUNCH(PK_TREE, k_wide_table, dim3(WIDE_TABLE_WG), dim3(NT), 0, st, w);
  switch (P.ty.kind) {
    case 0: LAUNCH(PK_CLASSIFY, k_wide_count<0>, dim3(w.W), dim3(CNT_NT), 0, st, w); break;
    case 1: LAUNCH(PK_CLASSIFY, k_wide_count<1>, dim3(w.W), dim3(CNT_NT), 0, st, w); break;
    default: LAUNCH(PK_CLASSIFY, k_wide_count<2>, dim3(w.W), dim3(CNT_NT), 0, st, w); break;
  }
  LAUNCH_CHECK();
  const uint32_t nbf = (uint32_t)cdiv(nf, SCAN_BLOCK), nba = (uint32_t)cdiv(na, SCAN_BLOCK);
  // both count arrays in one set of scan launches
  ScanPair q;
  q.h2 = w.ha;
  q.part2 = pa;
  q.total2 = na;
  q.nb1 = nbf;
  LAUNCH(PK_SCAN, k_scan_reduce, dim3(nbf + nba), dim3(NT), 0, st, w.hf, pf, nf, (const uint64_t*)nullptr, q);
  // (arrays of few blocks: each block adds up the block sums before it, no partials launch)
  const int self = (nbf <= SCAN_SELF_MAX && nba <= SCAN_SELF_MAX) ? 1 : 0;
  if (!self) LAUNCH(PK_SCAN, k_scan_partials, dim3(2), dim3(NT), 0, st, pf, nf, (const uint64_t*)nullptr, q);
  LAUNCH(PK_SCAN, k_scan_down, dim3(nbf + nba), dim3(NT), 0, st, w.hf, pf, nf, (const uint64_t*)nullptr, q, self);
  LAUNCH_CHECK();
  LAUNCH(PK_SPLIT_COARSE, k_wide_split_a, dim3(w.W), dim3(SA_NT), 0, st, w);
  LAUNCH_CHECK();
  // pieces of the second pass: at most one per WIDE_TB keys of each region, plus one per region
  const uint32_t pieces = (uint32_t)(cdiv(P.n, WIDE_TB) + WIDE_P1);
  LAUNCH(PK_SPLIT_FINE, k_wide_split_b, dim3(pieces), dim3(NT), 0, st, w);
  LAUNCH_CHECK();
  if (wide_small_rounds(P.n, w.p, P.s))
    LAUNCH(PK_BUCKET_SORT, (k_wide_bucket<WIDE_SCAP, WIDE_SLG>), dim3(w.p), dim3(WIDE_BNT), 0, st, a, w, exp);
  else
    LAUNCH(PK_BUCKET_SORT, (k_wide_bucket<WIDE_BCAP, ROUNDS_LOG2>), dim3(w.p), dim3(WIDE_BNT), 0, st, a, w, exp);
  LAUNCH_CHECK();
  LAUNCH(PK_BUCKET_LEFT, (k_bucket_leftover_keys<4>), dim3(std::min<uint32_t>(w.p, 512)), dim3(NT), 0, st, a, 0);
  LAUNCH_CHECK();
  return SS_OK;
}

int run_single_any(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout, hipStream_t st);

// Sort-first organisation (steps 4 and 5 of Alg. 1 / Alg. 2; step 1 ran
// before the sample, steps 2-3 built the splitter tree): place the splitters
// in the sorted blocks, gather each bucket's runs into tmp, sort each bucket
// into the output.
int run_sort_first(const Plan& P, char* ws, LevelArgs a, void* out, int exp, hipStream_t st) {
  SfArgs f{};
  f.bkeys = (const uint32_t*)(ws + P.o_regk);
  f.bidx = (const uint32_t*)(ws + P.o_regi);
  f.tree = (const uint64_t*)a.tree;
  f.pos = (uint32_t*)(ws + P.o_sfpos);
  f.bkt = (uint2*)(ws + P.o_sfbkt);
  f.stage = (uint32_t*)(ws + P.o_tmp);
  f.n = P.n;
  f.p = P.p_eff;
  f.lgp = 31 - __builtin_clz(P.p_eff);
  f.kind = P.ty.kind;
  const uint64_t bmax = cdiv(P.n, f.p);   // longest block
  f.lds_keys = bmax <= SF_LDS_BYTES / 4 ? (uint32_t)bmax : 0u;
  LAUNCH(PK_SF_SEARCH, k_sf_search<4>, dim3(f.p), dim3(SF_NT), 4 * (size_t)f.lds_keys, st, f);
  LAUNCH_CHECK();
  a.dst = f.stage;
  a.out = out;
  if (P.prm.flags & SS_F_SF_MERGE) {
    LAUNCH(PK_BUCKET_SORT, k_sf_merge, dim3(f.p), dim3(SFM_NT), 0, st, a, f, exp ? a.exp_counts : nullptr);
    LAUNCH_CHECK();
    return SS_OK;
  }
  LAUNCH(PK_SF_GATHER, k_sf_gather, dim3(f.p), dim3(SF_GNT), 0, st, f, exp ? a.exp_counts : nullptr);
  LAUNCH_CHECK();
  if (wide_small_rounds(P.n, f.p, P.s))
    LAUNCH(PK_BUCKET_SORT, (k_sf_bucket<WIDE_SCAP, WIDE_SLG>), dim3(f.p), dim3(WIDE_BNT), 0, st, a, f);
  else
    LAUNCH(PK_BUCKET_SORT, (k_sf_bucket<WIDE_BCAP, ROUNDS_LOG2>), dim3(f.p), dim3(WIDE_BNT), 0, st, a, f);
  LAUNCH_CHECK();
  LAUNCH(PK_BUCKET_LEFT, (k_bucket_leftover_keys<4>), dim3(std::min<uint32_t>(f.p, 512)), dim3(NT), 0, st, a, 0);
  LAUNCH_CHECK();
  return SS_OK;
}

template <int KW, int VW>
int run_segmented(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout,
                  const int64_t* off, hipStream_t st);

// The top level of a single sort with random sampling whose 4-byte sample
// is ranked by chunk pairs: init, draw and chunk sorts are one launch.
bool fused_top(const Plan& P) {
  return !P.segmented && !P.regular && P.ty.KW == 4 && P.lp.big_sample && !P.nested_s && P.o_scnt != 0;
}

// Sort-first organisation for 8-byte keys or with a payload: step 4 as
// above; step 5 gathers bucket j's runs (with the payload of each key) into
// the stage and sorts the p buckets as segments into the output.
template <int KW, int VW>
int run_sort_first_any(const Plan& P, char* ws, LevelArgs a, const void* vin, void* out, void* vout, int exp,
                       hipStream_t st) {
  SfArgs f{};
  f.bkeys = (const uint32_t*)(ws + P.o_regk);
  f.bidx = (const uint32_t*)(ws + P.o_regi);
  f.tree = (const uint64_t*)a.tree;
  f.tree_tag = a.tree_tag;
  f.pos = (uint32_t*)(ws + P.o_sfpos);
  f.bkt = (uint2*)(ws + P.o_sfbkt);
  f.n = P.n;
  f.p = P.p_eff;
  f.lgp = 31 - __builtin_clz(P.p_eff);
  f.kind = P.ty.kind;
  const uint64_t bmax = cdiv(P.n, f.p);
  f.lds_keys = bmax <= SF_LDS_BYTES / KW ? (uint32_t)bmax : 0u;
  LAUNCH(PK_SF_SEARCH, k_sf_search<KW>, dim3(f.p), dim3(SF_NT), (size_t)KW * f.lds_keys, st, f);
  LAUNCH_CHECK();
  void* kst = ws + P.o_tmp;
  void* vst = VW ? (void*)(ws + P.o_vtmp) : nullptr;
  int64_t* off = (int64_t*)(ws + P.o_sfoff);
  LAUNCH(PK_SF_GATHER, (k_sf_gather_any<KW, VW>), dim3(f.p), dim3(SF_GNT), 0, st, f, kst, vst, vin,
         P.ty.iota ? 1 : 0, off, exp ? a.exp_counts : nullptr);
  LAUNCH_CHECK();
  g_prof_force = PK_BUCKET_SORT;
  const int rc = run_segmented<KW, VW>(*P.nested_b, ws + P.o_nested_b, kst, vst, out, vout, off, st);
  g_prof_force = -1;
  return rc;
}

template <int KW, int VW>
int run_levels(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout, hipStream_t st) {
  const uint32_t Cs = sample_cap(KW);
  for (int l = 0; l < P.lp.nlev; l++) {
    const LevelPlan& lv = P.lp.lv[l];
    LevelArgs a = level_args(P, ws, l, in, vin, out, vout);
    const int exp = (P.exp && l == 0) ? 1 : 0;
    // (the top level of a single sort is planned by k_init_single)
    if (l > 0 || P.segmented) {
      LAUNCH(PK_PLAN, k_plan, dim3(1), dim3(NT), 0, st, a, Cs);
      LAUNCH_CHECK();
    }
    // sample
    if (l == 0 && fused_top(P)) {
      // init, draw and chunk sorts in one launch, then the pair ranks
      TopInit ti{P.n, P.prm.seed, P.p_eff, (uint32_t)P.m, P.stride, P.lp.lv[0].tile};
      LAUNCH(PK_SAMPLE_SORT, k_sample_draw_sort, dim3((uint32_t)cdiv(P.m, sample_chunk(4))), dim3(NT), 0, st, a,
             (Ctl*)(ws + P.o_ctl), (SegDesc*)(ws + P.lp.lv[0].o_segs), ti);
      LAUNCH_CHECK();
    } else if (l == 0 && P.regular) {
      const uint32_t S = P.s * P.p_eff;
      LAUNCH(PK_SAMPLE, k_sample_regular<KW>, dim3(grid_of(P.m, 256, 4096)), dim3(256), 0, st, a,
                         (const void*)(ws + P.o_regk), (const uint32_t*)(ws + P.o_regi), (uint64_t)P.n, P.p_eff, S);
    } else {
      LAUNCH(PK_SAMPLE, k_sample_random<KW>, dim3(grid_of(lv.samp_cap, 256, 4096)), dim3(256), 0, st, a);
    }
    LAUNCH_CHECK();
    // sample sort and splitter tree
    bool sample_done = false;
    if constexpr (KW == 4) {
      if (l == 0 && P.nested_s) {
        uint64_t* pk = (uint64_t*)(ws + P.o_spack);
        LAUNCH(PK_SAMPLE_SORT, k_pack_sample, dim3(grid_of(P.m, 256, 4096)), dim3(256), 0, st,
               (const uint32_t*)a.s_ord, (const uint32_t*)a.s_tag, pk, (uint64_t)P.m);
        LAUNCH_CHECK();
        g_prof_force = PK_SAMPLE_SORT;
        const int rc = run_single_any(*P.nested_s, ws + P.o_nested_s, pk, nullptr, pk, nullptr, st);
        g_prof_force = -1;
        if (rc) return rc;
        LAUNCH(PK_SAMPLE_SORT, k_unpack_sample, dim3(grid_of(P.m, 256, 4096)), dim3(256), 0, st,
               (const uint64_t*)pk, (uint32_t*)a.s_ord, a.s_tag, (uint64_t)P.m);
        LAUNCH_CHECK();
        LAUNCH(PK_TREE, k_build_tree<KW>, dim3(grid_of(std::max<uint64_t>(P.m, P.p_eff), 256, 1024)), dim3(256), 0,
               st, a, (const void*)a.s_ord, (const uint32_t*)a.s_tag, exp);
        sample_done = true;
      }
    }
    if (sample_done) {
    } else if (l == 0 && P.lp.big_sample) {
      // sorted chunks, then every record's rank among all of them: the
      // splitters go straight to the tree
      const uint32_t ch = sample_chunk(KW);
      if (!fused_top(P)) {
        LAUNCH(PK_SAMPLE_SORT, k_sample_chunk_sort<KW>, dim3((uint32_t)cdiv(P.m, ch)), dim3(NT), 0, st, a);
        LAUNCH_CHECK();
      }
      const uint64_t nch = cdiv(P.m, ch);
      if (KW == 4 && P.o_scnt) {
        uint16_t* cnt = (uint16_t*)(ws + P.o_scnt);
        LAUNCH(PK_SAMPLE_MERGE, k_sample_pair_count, dim3((uint32_t)(nch * nch)), dim3(NT), 0, st, a, cnt);
        LAUNCH_CHECK();
        LAUNCH(PK_SAMPLE_MERGE, k_sample_rank_sum, dim3((uint32_t)cdiv(P.m, 256)), dim3(256), 0, st, a,
               (const uint16_t*)cnt, exp);
      } else {
        // lanes per record: the chunk count rounded up to a power of two, at most a wave
        uint32_t lgL = 0;
        while ((1ull << lgL) < nch && lgL < 6) lgL++;
        LAUNCH(PK_SAMPLE_MERGE, k_sample_rank<KW>, dim3((uint32_t)cdiv(P.m << lgL, 256)), dim3(256), 0, st, a,
               exp, lgL);
      }
    } else {
      LAUNCH(PK_SAMPLE_SORT, k_sample_sort_wg<KW>, dim3(lv.seg_cap), dim3(NT), 0, st, a, exp);
    }
    LAUNCH_CHECK();
    if (l == 0 && P.sortfirst) {
      if constexpr (KW == 4 && VW == 0) return run_sort_first(P, ws, a, out, exp, st);
      else return run_sort_first_any<KW, VW>(P, ws, a, vin, out, vout, exp, st);
    }
    if constexpr (KW == 4 && VW == 0) {
      if (l == 0 && P.wide) {
        int rc = run_wide(P, ws, a, in, out, exp, st);
        if (rc) return rc;
        continue;
      }
    }
    const uint32_t tiles = (uint32_t)lv.tiles_cap;
    switch (lv.pmax) {
      case 256: LAUNCH(PK_CLASSIFY, (k_classify<KW, 256>), dim3(tiles), dim3(NT), 0, st, a); break;
      case 512: LAUNCH(PK_CLASSIFY, (k_classify<KW, 512>), dim3(tiles), dim3(NT), 0, st, a); break;
      case 1024: LAUNCH(PK_CLASSIFY, (k_classify<KW, 1024>), dim3(tiles), dim3(NT), 0, st, a); break;
      default: LAUNCH(PK_CLASSIFY, (k_classify<KW, 4096>), dim3(tiles), dim3(NT), 0, st, a); break;
    }
    LAUNCH_CHECK();
    const uint32_t nb = (uint32_t)cdiv(std::max<uint64_t>(lv.hist_cap, 1), SCAN_BLOCK);
    const uint64_t* tot_dev = &a.ctl->total_hist;
    LAUNCH(PK_SCAN, k_scan_reduce, dim3(nb), dim3(NT), 0, st, a.hist, a.scan_part, (uint64_t)0, tot_dev,
           ScanPair{});
    const int self = nb <= SCAN_SELF_MAX ? 1 : 0;
    if (!self)
      LAUNCH(PK_SCAN, k_scan_partials, dim3(1), dim3(NT), 0, st, a.scan_part, (uint64_t)0, tot_dev, ScanPair{});
    LAUNCH(PK_SCAN, k_scan_down, dim3(nb), dim3(NT), 0, st, a.hist, a.scan_part, (uint64_t)0, tot_dev, ScanPair{},
           self);
    LAUNCH_CHECK();
    if constexpr (VW == 0) {
      // keys only: equal keys are bit-identical, so placement order inside a bucket is free
      switch (lv.pmax) {
        case 256: LAUNCH(PK_SCATTER, (k_scatter_keys<KW, 256>), dim3(tiles), dim3(NT), 0, st, a); break;
        case 512: LAUNCH(PK_SCATTER, (k_scatter_keys<KW, 512>), dim3(tiles), dim3(NT), 0, st, a); break;
        case 1024: LAUNCH(PK_SCATTER, (k_scatter_keys<KW, 1024>), dim3(tiles), dim3(NT), 0, st, a); break;
        default: LAUNCH(PK_SCATTER, (k_scatter_keys<KW, 4096>), dim3(tiles), dim3(NT), 0, st, a); break;
      }
      LAUNCH_CHECK();
      LAUNCH(PK_BUCKET_SORT, (k_bucket_sort_keys<KW>), dim3((uint32_t)lv.bkt_cap), dim3(NT), 0, st, a, exp);
      LAUNCH_CHECK();
      // few buckets are handed on: small grids walk the lists (4-byte keys
      // first try the round-based slot sort)
      const uint32_t gl = (uint32_t)std::min<uint64_t>(lv.bkt_cap, 512);
      if constexpr (KW == 4) {
        LAUNCH(PK_BUCKET_LEFT, k_bucket_rounds_keys, dim3(std::min<uint32_t>(gl, 256)), dim3(WIDE_BNT), 0, st, a);
        LAUNCH_CHECK();
      }
      LAUNCH(PK_BUCKET_LEFT, (k_bucket_leftover_keys<KW>), dim3(gl), dim3(NT), 0, st, a, KW == 4 ? 1 : 0);
    } else {
      switch (lv.pmax) {
        case 256: LAUNCH(PK_SCATTER, (k_scatter_pairs<KW, VW>), dim3(tiles), dim3(NT), 0, st, a); break;
        case 512: LAUNCH(PK_SCATTER, (k_scatter<KW, VW, 512>), dim3(tiles), dim3(NT), 0, st, a); break;
        case 1024: LAUNCH(PK_SCATTER, (k_scatter<KW, VW, 1024>), dim3(tiles), dim3(NT), 0, st, a); break;
        default: LAUNCH(PK_SCATTER, (k_scatter<KW, VW, 4096>), dim3(tiles), dim3(NT), 0, st, a); break;
      }
      LAUNCH_CHECK();
      // stable slot sort; buckets too large or crowded go on to the radix /
      // next-level kernel
      LAUNCH(PK_BUCKET_SORT, (k_bucket_sort_pairs<KW, VW>), dim3((uint32_t)lv.bkt_cap), dim3(WIDE_BNT), 0, st, a,
             exp);
      LAUNCH_CHECK();
      LAUNCH(PK_BUCKET_LEFT, (k_bucket_leftover_pairs<KW, VW>), dim3((uint32_t)std::min<uint64_t>(lv.bkt_cap, 512)),
             dim3(NT), 0, st, a);
    }
    LAUNCH_CHECK();
  }
  return SS_OK;
}

template <int KW, int VW>
int run_segmented(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout,
                  const int64_t* off, hipStream_t st) {
  Ctl* g = (Ctl*)(ws + P.o_ctl);
  const uint32_t C = small_cap(KW, VW);
  LAUNCH(PK_INIT, k_init_ctl, dim3(1), dim3(64), 0, st, g);
  LAUNCH_CHECK();
  SegDesc* top = P.lp.nlev ? (SegDesc*)(ws + P.lp.lv[0].o_segs) : nullptr;
  uint32_t top_cap = P.lp.nlev ? P.lp.lv[0].seg_cap : 0;
  LAUNCH(PK_INIT, k_seg_init, dim3(grid_of(P.nseg, 256, 1024)), dim3(256), 0, st, g, off, (uint32_t)P.nseg,
                     P.lp.nlev ? C : 0xFFFFFFFFu, top, top_cap, (SmallEnt*)(ws + P.o_small),
                     (SmallEnt*)(ws + P.o_tiny), (SmallEnt*)(ws + P.o_mid), P.prm.seed, (uint64_t)P.n,
                     (uint64_t)P.maxlen);
  LAUNCH_CHECK();
  // the three classes below one split level, each launch sized for every
  // segment falling into it (the lists are filled on the device)
  const int iota = P.ty.iota ? 1 : 0;
  LAUNCH(PK_SMALL_SORT, (k_sort_tiny_list<KW, VW>), dim3(grid_of(P.nseg, NT / WAVE, 8192)), dim3(NT), 0, st, g,
         (const SmallEnt*)(ws + P.o_tiny), in, vin, out, vout, P.ty.kind, iota);
  LAUNCH_CHECK();
  if (P.maxlen > WAVE) {
    LAUNCH(PK_SMALL_SORT, (k_sort_mid_list<KW, VW>), dim3(grid_of(P.nseg, 1, 8192)), dim3(NT), 0, st, g,
           (const SmallEnt*)(ws + P.o_mid), in, vin, out, vout, P.ty.kind, iota);
    LAUNCH_CHECK();
  }
  if (P.maxlen > MID_CAP) {
    const dim3 gs((uint32_t)std::max<uint64_t>(P.nseg, 1));
    if constexpr (KW == 4 && VW == 4) {
      if (iota) {
        LAUNCH(PK_SMALL_SORT, (k_sort_small_list_iota<KW, VW>), gs, dim3(WIDE_BNT), 0, st, g,
               (const SmallEnt*)(ws + P.o_small), (SmallEnt*)(ws + P.o_small_fb), in, out, vout, P.ty.kind);
        LAUNCH_CHECK();
        LAUNCH(PK_SMALL_SORT, (k_sort_small_list<KW, VW>), gs, dim3(NT), 0, st, g,
               (const SmallEnt*)(ws + P.o_small_fb), in, vin, out, vout, P.ty.kind, iota, 1);
      } else {
        LAUNCH(PK_SMALL_SORT, (k_sort_small_list<KW, VW>), gs, dim3(NT), 0, st, g, (const SmallEnt*)(ws + P.o_small),
               in, vin, out, vout, P.ty.kind, iota, 0);
      }
    } else {
      LAUNCH(PK_SMALL_SORT, (k_sort_small_list<KW, VW>), gs, dim3(NT), 0, st, g, (const SmallEnt*)(ws + P.o_small),
             in, vin, out, vout, P.ty.kind, iota, 0);
    }
    LAUNCH_CHECK();
  }
  return run_levels<KW, VW>(P, ws, in, vin, out, vout, st);
}

template <int KW, int VW>
int run_single(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout, hipStream_t st) {
  if (P.n == 0) return SS_OK;
  Ctl* g = (Ctl*)(ws + P.o_ctl);
  const void* vsrc = P.ty.iota ? nullptr : vin;
  if (P.direct) {
    LAUNCH(PK_INIT, k_init_ctl, dim3(1), dim3(64), 0, st, g);
    LAUNCH(PK_SMALL_SORT, (k_sort_direct<KW, VW>), dim3(1), dim3(NT), 0, st, in, vsrc, out, vout, (uint64_t)0,
                       (uint32_t)P.n, P.ty.kind);
    LAUNCH_CHECK();
    return SS_OK;
  }
  if (P.whole) {
    LAUNCH(PK_INIT, k_init_ctl, dim3(1), dim3(64), 0, st, g);
    LAUNCH(PK_SMALL_SORT, (k_sort_whole<KW, VW>), dim3(1), dim3(NT), 0, st, in, vsrc, out, vout,
                       (void*)(ws + P.o_tmp), P.ty.VW ? (void*)(ws + P.o_vtmp) : nullptr, (uint64_t)P.n, P.ty.kind);
    LAUNCH_CHECK();
    return SS_OK;
  }
  if (P.regular || P.sortfirst) {
    // Alg. 1 step 1: sort the p blocks (key, in-block index) with the segmented path
    int64_t* boff = (int64_t*)(ws + P.o_regoff);
    LAUNCH(PK_INIT, k_block_offsets, dim3(grid_of(P.p_eff + 1, 256, 64)), dim3(256), 0, st, boff, (uint64_t)P.n,
                       P.p_eff);
    LAUNCH_CHECK();
    int rc = run_segmented<KW, 4>(*P.nested, ws + P.o_nested, in, nullptr, ws + P.o_regk, ws + P.o_regi, boff, st);
    if (rc) return rc;
  }
  // (the fused sample kernel initialises the level itself)
  if (!fused_top(P)) {
    LAUNCH(PK_INIT, k_init_single, dim3(1), dim3(64), 0, st, g, (SegDesc*)(ws + P.lp.lv[0].o_segs), (uint64_t)P.n,
           P.p_eff, (uint32_t)P.m, P.stride, P.prm.seed, P.lp.lv[0].tile);
    LAUNCH_CHECK();
  }
  return run_levels<KW, VW>(P, ws, in, vin, out, vout, st);
}

template <int KW, int VW>
int dispatch_single(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout, hipStream_t st) {
  return run_single<KW, VW>(P, ws, in, vin, out, vout, st);
}

int run_single_t(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout, hipStream_t st) {
  const int KW = P.ty.KW, VW = P.ty.VW;
  if (KW == 4 && VW == 0) return dispatch_single<4, 0>(P, ws, in, vin, out, vout, st);
  if (KW == 4 && VW == 4) return dispatch_single<4, 4>(P, ws, in, vin, out, vout, st);
  if (KW == 4 && VW == 8) return dispatch_single<4, 8>(P, ws, in, vin, out, vout, st);
  if (KW == 8 && VW == 0) return dispatch_single<8, 0>(P, ws, in, vin, out, vout, st);
  if (KW == 8 && VW == 4) return dispatch_single<8, 4>(P, ws, in, vin, out, vout, st);
  return dispatch_single<8, 8>(P, ws, in, vin, out, vout, st);
}

int run_segmented_t(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout,
                    const int64_t* off, hipStream_t st) {
  const int KW = P.ty.KW, VW = P.ty.VW;
  if (KW == 4 && VW == 0) return run_segmented<4, 0>(P, ws, in, vin, out, vout, off, st);
  if (KW == 4 && VW == 4) return run_segmented<4, 4>(P, ws, in, vin, out, vout, off, st);
  if (KW == 4 && VW == 8) return run_segmented<4, 8>(P, ws, in, vin, out, vout, off, st);
  if (KW == 8 && VW == 0) return run_segmented<8, 0>(P, ws, in, vin, out, vout, off, st);
  if (KW == 8 && VW == 4) return run_segmented<8, 4>(P, ws, in, vin, out, vout, off, st);
  return run_segmented<8, 8>(P, ws, in, vin, out, vout, off, st);
}

int run_single_any(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout, hipStream_t st) {
  if (!P.widen) return run_single_t(P, ws, in, vin, out, vout, st);
  uint32_t* v32 = (uint32_t*)(ws + P.o_widen);
  const int rc = run_single_t(P, ws, in, vin, out, v32, st);
  if (rc) return rc;
  LAUNCH(PK_WIDEN, k_widen_index, dim3(grid_of(P.n, 256, 8192)), dim3(256), 0, st, (const uint32_t*)v32,
         (int64_t*)vout, (const int64_t*)nullptr, (uint64_t)0, (uint64_t)P.n);
  LAUNCH_CHECK();
  return SS_OK;
}

int run_segmented_any(const Plan& P, char* ws, const void* in, const void* vin, void* out, void* vout,
                      const int64_t* off, hipStream_t st) {
  if (!P.widen) return run_segmented_t(P, ws, in, vin, out, vout, off, st);
  uint32_t* v32 = (uint32_t*)(ws + P.o_widen);
  const int rc = run_segmented_t(P, ws, in, vin, out, v32, off, st);
  if (rc) return rc;
  // (only [off[0], off[nseg]) holds sorted segments)
  LAUNCH(PK_WIDEN, k_widen_index, dim3(grid_of(P.n, 256, 8192)), dim3(256), 0, st, (const uint32_t*)v32,
         (int64_t*)vout, off, (uint64_t)P.nseg, (uint64_t)P.n);
  LAUNCH_CHECK();
  return SS_OK;
}

int check_ws(const Plan& P, const void* ws, size_t ws_bytes) {
  if (P.bytes && !ws) return fail(SS_EWORKSPACE, "workspace is NULL (%zu bytes needed)", P.bytes);
  if (ws_bytes < P.bytes) return fail(SS_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, P.bytes);
  if (((uintptr_t)ws) % ALIGN) return fail(SS_EWORKSPACE, "workspace must be %zu-byte aligned", ALIGN);
  return SS_OK;
}

int sort_common(const void* keys_in, const void* vals_in, void* keys_out, void* vals_out, size_t n, int key_type,
                int val_type, const ss_params* prm, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  Types ty;
  int rc = parse_types(key_type, val_type, &ty);
  if (rc) return rc;
  ss_params p;
  rc = check_params(prm, &p, ty, n);
  if (rc) return rc;
  if (n == 0) return SS_OK;
  if (!keys_in || !keys_out) return fail(SS_EINVAL, "keys_in and keys_out must be device pointers");
  if (ty.VW) {
    if (!vals_out) return fail(SS_EINVAL, "vals_out must be a device pointer");
    if (ty.iota && vals_in) return fail(SS_EINVAL, "vals_in must be NULL for an IOTA payload");
    if (!ty.iota && !vals_in) return fail(SS_EINVAL, "vals_in must be a device pointer");
  }
  const size_t kb = (size_t)ty.KW * n, vb = (size_t)ty.VW * n;
  if (overlap_partial(keys_in, kb, keys_out, kb) || overlap_partial(vals_in, vb, vals_out, vb) ||
      overlap_partial(keys_in, kb, vals_out, vb) || overlap_partial(vals_in, vb, keys_out, kb) ||
      (keys_out == vals_out && ty.VW))
    return fail(SS_EINVAL, "inputs and outputs overlap partially");
  Plan P;
  rc = plan_single(&P, n, ty, p);
  if (rc) return rc;
  rc = check_ws(P, ws, ws_bytes);
  if (rc) return rc;
  return run_single_any(P, (char*)ws, keys_in, vals_in, keys_out, vals_out, as_stream(stream));
}

// ------------------------------------------------------- string keys
//
// Layout and plans of a string sort: the prefix words, the index, the
// round-0 pairs sort, the run flags and their scans, the gathered runs and
// the segmented sort that orders them.
struct StrPlan {
  uint64_t n = 0;
  uint32_t width = 0, W = 0;
  Plan pairs;            // round 0: (word 0, index) pairs
  Plan seg;              // later rounds: the runs as segments, planned for the largest case
  size_t o_w = 0, o_w2 = 0, o_perm = 0, o_b = 0, o_f = 0, o_g = 0, o_fp = 0, o_gp = 0;
  size_t o_kt = 0, o_vt = 0, o_pt = 0, o_ks = 0, o_vs = 0, o_off = 0, o_pairs = 0, o_seg = 0;
  size_t bytes = 0;
};

int plan_strings(StrPlan* S, uint64_t n, uint32_t width, const ss_params* prm) {
  if (width < 8 || width > 256 || width % 8) return fail(SS_EINVAL, "width = %u: a multiple of 8 in [8, 256]", width);
  if (n >= (1ull << 32) - 1) return fail(SS_EINVAL, "n = %llu: fewer than 2^32 - 1 strings", (unsigned long long)n);
  S->n = n;
  S->width = width;
  S->W = width / 8;
  Types kt, st;
  parse_types(SS_U64, SS_V_IOTA32, &kt);
  parse_types(SS_U64, SS_V_B32, &st);
  ss_params p0, p1;
  int rc = check_params(prm, &p0, kt, n);
  if (rc) return rc;
  rc = check_params(prm, &p1, st, n, 1);
  if (rc) return rc;
  rc = plan_single(&S->pairs, n, kt, p0);
  if (rc) return rc;
  const uint64_t nseg = std::max<uint64_t>(n / 2, 1);
  rc = plan_segmented(&S->seg, n, nseg, n, st, p1, prm != nullptr);
  if (rc) return rc;
  Layout L;
  const uint64_t m = std::max<uint64_t>(n, 1);
  S->o_w = L.take(8 * m);
  S->o_w2 = L.take(8 * m);
  S->o_perm = L.take(4 * m);
  S->o_b = L.take(m);
  S->o_f = L.take(4 * (m + 1));
  S->o_g = L.take(4 * (m + 1));
  S->o_fp = L.take(4 * (cdiv(m + 1, SCAN_BLOCK) + 1));
  S->o_gp = L.take(4 * (cdiv(m + 1, SCAN_BLOCK) + 1));
  S->o_kt = L.take(8 * m);
  S->o_vt = L.take(4 * m);
  S->o_pt = L.take(4 * m);
  S->o_ks = L.take(8 * m);
  S->o_vs = L.take(4 * m);
  S->o_off = L.take(8 * (nseg + 1));
  S->o_pairs = L.take(S->pairs.bytes);
  S->o_seg = L.take(S->seg.bytes);
  S->bytes = L.cur;
  return SS_OK;
}

int sort_strings(const void* recs, void* recs_out, int64_t* perm_out, size_t n, uint32_t width, const ss_params* prm,
                 void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  StrPlan S;
  int rc = plan_strings(&S, n, width, prm);
  if (rc) return rc;
  if (n == 0) return SS_OK;
  if (!recs || !perm_out) return fail(SS_EINVAL, "recs and perm_out must be device pointers");
  if (((uintptr_t)recs | (uintptr_t)recs_out) % 8) return fail(SS_EINVAL, "recs and recs_out must be 8-byte aligned");
  if (overlap_partial(recs, (size_t)n * width, recs_out, (size_t)n * width) || recs == recs_out)
    return fail(SS_EINVAL, "recs_out must not overlap recs");
  if (!ws || ws_bytes < S.bytes || ((uintptr_t)ws) % ALIGN)
    return fail(SS_EWORKSPACE, "workspace of %zu bytes (aligned to %zu) needed", S.bytes, ALIGN);
  hipStream_t st = as_stream(stream);
  char* b = (char*)ws;
  const uint8_t* R = (const uint8_t*)recs;
  uint64_t* w = (uint64_t*)(b + S.o_w);
  uint64_t* w2 = (uint64_t*)(b + S.o_w2);
  uint32_t* perm = (uint32_t*)(b + S.o_perm);
  uint8_t* bd = (uint8_t*)(b + S.o_b);
  uint32_t* f = (uint32_t*)(b + S.o_f);
  uint32_t* g = (uint32_t*)(b + S.o_g);
  const uint32_t grid = grid_of(n, 256, 8192);
  // round 0: word 0 with the index, stable pairs sort
  LAUNCH(PK_SAMPLE, k_str_word, dim3(grid), dim3(256), 0, st, R, width, 0u, (const uint32_t*)nullptr, w, (uint64_t)n);
  LAUNCH_CHECK();
  rc = run_single_any(S.pairs, b + S.o_pairs, w, nullptr, w2, perm, st);
  if (rc) return rc;
  uint64_t* cur = w2;
  for (uint32_t k = 1; k < S.W; k++) {
    LAUNCH(PK_CLASSIFY, k_str_flags, dim3(grid_of(n + 1, 256, 8192)), dim3(256), 0, st, (const uint64_t*)cur,
           k == 1 ? (const uint8_t*)nullptr : (const uint8_t*)bd, bd, f, g, (uint64_t)n);
    LAUNCH_CHECK();
    const uint64_t tot1 = n + 1;
    const uint32_t nb = (uint32_t)cdiv(tot1, SCAN_BLOCK);
    ScanPair q;
    q.h2 = g;
    q.part2 = (uint32_t*)(b + S.o_gp);
    q.total2 = tot1;
    q.nb1 = nb;
    uint32_t* fp = (uint32_t*)(b + S.o_fp);
    LAUNCH(PK_SCAN, k_scan_reduce, dim3(2 * nb), dim3(NT), 0, st, f, fp, tot1, (const uint64_t*)nullptr, q);
    const int self = nb <= SCAN_SELF_MAX ? 1 : 0;
    if (!self) LAUNCH(PK_SCAN, k_scan_partials, dim3(2), dim3(NT), 0, st, fp, tot1, (const uint64_t*)nullptr, q);
    LAUNCH(PK_SCAN, k_scan_down, dim3(2 * nb), dim3(NT), 0, st, f, fp, tot1, (const uint64_t*)nullptr, q, self);
    LAUNCH_CHECK();
    // how many strings sit in runs of equal prefixes, in how many runs
    uint32_t tot = 0, nruns = 0;
    HIP_TRY(hipMemcpyAsync(&tot, f + n, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&nruns, g + n, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (tot == 0) break;
    uint64_t* kt = (uint64_t*)(b + S.o_kt);
    uint32_t* vt = (uint32_t*)(b + S.o_vt);
    uint32_t* pt = (uint32_t*)(b + S.o_pt);
    uint64_t* ks = (uint64_t*)(b + S.o_ks);
    uint32_t* vs = (uint32_t*)(b + S.o_vs);
    int64_t* off = (int64_t*)(b + S.o_off);
    LAUNCH(PK_SCATTER, k_str_gather, dim3(grid_of(n + 1, 256, 8192)), dim3(256), 0, st, R, width, k,
           (const uint8_t*)bd, (const uint32_t*)f, (const uint32_t*)g, (const uint32_t*)perm, kt, vt, pt, off,
           (uint64_t)n);
    LAUNCH_CHECK();
    // the runs as segments (planned for this round's sizes, inside the
    // workspace planned for the largest case)
    Types sty;
    parse_types(SS_U64, SS_V_B32, &sty);
    ss_params p1;
    rc = check_params(prm, &p1, sty, tot, 1);
    if (rc) return rc;
    Plan P;
    rc = plan_segmented(&P, tot, nruns, tot, sty, p1, prm != nullptr);
    if (rc) return rc;
    if (P.bytes > S.seg.bytes) return fail(SS_EWORKSPACE, "string round plan exceeds its workspace");
    rc = run_segmented_any(P, b + S.o_seg, kt, vt, ks, vs, off, st);
    if (rc) return rc;
    LAUNCH(PK_SCATTER, k_str_scatter, dim3(grid_of(tot, 256, 8192)), dim3(256), 0, st, (const uint64_t*)ks,
           (const uint32_t*)vs, (const uint32_t*)pt, perm, cur, (const uint32_t*)f, (uint64_t)n);
    LAUNCH_CHECK();
  }
  LAUNCH(PK_WIDEN, k_widen_index, dim3(grid), dim3(256), 0, st, (const uint32_t*)perm, perm_out,
         (const int64_t*)nullptr, (uint64_t)0, (uint64_t)n);
  LAUNCH_CHECK();
  if (recs_out) {
    LAUNCH(PK_SCATTER, k_str_permute, dim3(grid_of((uint64_t)n * (width / 8), 256, 8192)), dim3(256), 0, st, R,
           (uint8_t*)recs_out, (const uint32_t*)perm, width, (uint64_t)n);
    LAUNCH_CHECK();
  }
  return SS_OK;
}

// -------------------------------------------------- no-allocation entry
//
// sample_sort_keys_noalloc runs the keys-only sort with its workspace in a
// static device array instead of a caller-provided buffer.  In host code
// `scratch` only names the symbol: its device address (one per GPU) comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int scratch_of_current_device(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(SS_EINVAL, "device %d: at most %d devices", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SS_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SS_OK;
}

int sort_noalloc(const void* keys_in, void* keys_out, size_t n, int key_type, const ss_params* prm, void* stream) {
  g_err[0] = 0;
  Types ty;
  int rc = parse_types(key_type, SS_V_NONE, &ty);
  if (rc) return rc;
  ss_params p;
  rc = check_params(prm, &p, ty, n);
  if (rc) return rc;
  if (n == 0) return SS_OK;
  if (!keys_in || !keys_out) return fail(SS_EINVAL, "keys_in and keys_out must be device pointers");
  const size_t kb = (size_t)ty.KW * n;
  if (overlap_partial(keys_in, kb, keys_out, kb)) return fail(SS_EINVAL, "inputs and outputs overlap partially");
  Plan P;
  rc = plan_single(&P, n, ty, p);
  if (rc) return rc;
  if (P.bytes > NOALLOC_SCRATCH_BYTES)
    return fail(SS_EWORKSPACE, "n = %zu needs %zu bytes of scratch; the static scratch array holds %zu", n, P.bytes,
                NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  return run_single_any(P, (char*)ws, keys_in, nullptr, keys_out, nullptr, as_stream(stream));
}

}  // namespace

extern "C" {

int sample_sort_keys_noalloc(const void* keys_in, void* keys_out, size_t n, int key_type, const ss_params* prm,
                             void* stream) {
  return sort_noalloc(keys_in, keys_out, n, key_type, prm, stream);
}

size_t ss_noalloc_capacity_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

int ss_strings_workspace_size(size_t n, uint32_t width, const ss_params* prm, size_t* bytes_out) {
  g_err[0] = 0;
  if (!bytes_out) return fail(SS_EINVAL, "bytes_out is NULL");
  StrPlan S;
  int rc = plan_strings(&S, n, width, prm);
  if (rc) return rc;
  *bytes_out = S.bytes;
  return SS_OK;
}

int sample_sort_strings(const void* recs, void* recs_out, int64_t* perm_out, size_t n, uint32_t width,
                        const ss_params* prm, void* ws, size_t ws_bytes, void* stream) {
  return sort_strings(recs, recs_out, perm_out, n, width, prm, ws, ws_bytes, stream);
}

const char* ss_last_error(void) { return g_err; }

int ss_workspace_size(size_t n, int key_type, int val_type, const ss_params* prm, size_t* bytes_out) {
  g_err[0] = 0;
  if (!bytes_out) return fail(SS_EINVAL, "bytes_out is NULL");
  Types ty;
  int rc = parse_types(key_type, val_type, &ty);
  if (rc) return rc;
  ss_params p;
  rc = check_params(prm, &p, ty, n);
  if (rc) return rc;
  Plan P;
  rc = plan_single(&P, n, ty, p);
  if (rc) return rc;
  *bytes_out = P.bytes;
  return SS_OK;
}

int ss_stage_layout(size_t n, int key_type, int val_type, const ss_params* prm, ss_stage_info* info) {
  g_err[0] = 0;
  if (!info) return fail(SS_EINVAL, "info is NULL");
  Types ty;
  int rc = parse_types(key_type, val_type, &ty);
  if (rc) return rc;
  ss_params p;
  rc = check_params(prm, &p, ty, n);
  if (rc) return rc;
  Plan P;
  rc = plan_single(&P, n, ty, p);
  if (rc) return rc;
  memset(info, 0, sizeof *info);
  info->p_eff = P.p_eff;
  info->stride = P.stride;
  info->m = P.m;
  info->direct = (P.direct || P.whole) ? 1u : 0u;
  info->levels = P.lp.nlev > 0 ? (uint32_t)(P.lp.nlev - 1) : 0u;
  if (P.exp) {
    info->sample_ord = P.o_exp_so;
    info->sample_tag = P.o_exp_st;
    info->spl_ord = P.o_exp_po;
    info->spl_tag = P.o_exp_pt;
    info->counts = P.o_exp_cnt;
  }
  return SS_OK;
}

int sample_sort_keys(const void* keys_in, void* keys_out, size_t n, int key_type, const ss_params* prm, void* ws,
                     size_t ws_bytes, void* stream) {
  return sort_common(keys_in, nullptr, keys_out, nullptr, n, key_type, SS_V_NONE, prm, ws, ws_bytes, stream);
}

int sample_sort_pairs(const void* keys_in, const void* vals_in, void* keys_out, void* vals_out, size_t n,
                      int key_type, int val_type, const ss_params* prm, void* ws, size_t ws_bytes, void* stream) {
  if (val_type == SS_V_NONE) {
    g_err[0] = 0;
    return fail(SS_EINVAL, "sample_sort_pairs needs a payload type");
  }
  return sort_common(keys_in, vals_in, keys_out, vals_out, n, key_type, val_type, prm, ws, ws_bytes, stream);
}

int ss_segmented_workspace_size(size_t total, size_t num_segments, size_t max_seg_len, int key_type, int val_type,
                                const ss_params* prm, size_t* bytes_out) {
  g_err[0] = 0;
  if (!bytes_out) return fail(SS_EINVAL, "bytes_out is NULL");
  Types ty;
  int rc = parse_types(key_type, val_type, &ty);
  if (rc) return rc;
  ss_params p;
  rc = check_params(prm, &p, ty, max_seg_len ? max_seg_len : total, 1);
  if (rc) return rc;
  Plan P;
  rc = plan_segmented(&P, total, num_segments, max_seg_len, ty, p, prm != nullptr);
  if (rc) return rc;
  *bytes_out = P.bytes;
  return SS_OK;
}

int segmented_sort(const void* keys_in, const void* vals_in, void* keys_out, void* vals_out, const int64_t* d_offsets,
                   size_t num_segments, size_t total, size_t max_seg_len, int key_type, int val_type,
                   const ss_params* prm, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  Types ty;
  int rc = parse_types(key_type, val_type, &ty);
  if (rc) return rc;
  ss_params p;
  rc = check_params(prm, &p, ty, max_seg_len ? max_seg_len : total, 1);
  if (rc) return rc;
  if (num_segments == 0 || total == 0) return SS_OK;
  if (!keys_in || !keys_out || !d_offsets) return fail(SS_EINVAL, "keys and offsets must be device pointers");
  if (ty.VW) {
    if (!vals_out) return fail(SS_EINVAL, "vals_out must be a device pointer");
    if (ty.iota && vals_in) return fail(SS_EINVAL, "vals_in must be NULL for an IOTA payload");
    if (!ty.iota && !vals_in) return fail(SS_EINVAL, "vals_in must be a device pointer");
  }
  const size_t kb = (size_t)ty.KW * total, vb = (size_t)ty.VW * total;
  if (overlap_partial(keys_in, kb, keys_out, kb) || overlap_partial(vals_in, vb, vals_out, vb) ||
      overlap_partial(keys_in, kb, vals_out, vb) || overlap_partial(vals_in, vb, keys_out, kb))
    return fail(SS_EINVAL, "inputs and outputs overlap partially");
  Plan P;
  rc = plan_segmented(&P, total, num_segments, max_seg_len, ty, p, prm != nullptr);
  if (rc) return rc;
  rc = check_ws(P, ws, ws_bytes);
  if (rc) return rc;
  return run_segmented_any(P, (char*)ws, keys_in, vals_in, keys_out, vals_out, d_offsets, as_stream(stream));
}

// Set by k_scatter_grad when an index falls outside its row; read and
// cleared by ss_grad_status.
__device__ uint32_t g_grad_status;

int ss_scatter_grad(const void* grad_y, const int64_t* perm, void* grad_x, size_t rows, size_t row_len,
                    int elem_bytes, void* stream) {
  g_err[0] = 0;
  if (rows == 0 || row_len == 0) return SS_OK;
  if (!grad_y || !perm || !grad_x) return fail(SS_EINVAL, "grad_y, perm and grad_x must be device pointers");
  if (grad_y == grad_x) return fail(SS_EINVAL, "grad_x must not alias grad_y");
  if (rows >= (1ull << 31) || row_len >= (1ull << 31))
    return fail(SS_EINVAL, "rows and row_len must be below 2^31");
  if (((uintptr_t)grad_y | (uintptr_t)perm) % 16)
    return fail(SS_EINVAL, "grad_y and perm must be 16-byte aligned");
  const uint32_t per = GRAD_V * GRAD_NT;
  const uint64_t chunks = cdiv(row_len, per);
  const uint64_t tiles = chunks * rows;
  if (tiles >= (1ull << 32)) return fail(SS_EINVAL, "too many elements");
  if (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8)
    return fail(SS_EINVAL, "elem_bytes = %d: need 2, 4 or 8", elem_bytes);
  uint32_t* status = nullptr;
  HIP_TRY(hipGetSymbolAddress((void**)&status, HIP_SYMBOL(g_grad_status)));
  hipStream_t st = as_stream(stream);
  switch (elem_bytes) {
    case 2:
      LAUNCH(PK_GRAD, k_scatter_grad<uint16_t>, dim3((uint32_t)tiles), dim3(GRAD_NT), 0, st, (const uint16_t*)grad_y,
             perm, (uint16_t*)grad_x, (uint32_t)rows, (uint32_t)row_len, (uint32_t)chunks, status);
      break;
    case 4:
      LAUNCH(PK_GRAD, k_scatter_grad<uint32_t>, dim3((uint32_t)tiles), dim3(GRAD_NT), 0, st, (const uint32_t*)grad_y,
             perm, (uint32_t*)grad_x, (uint32_t)rows, (uint32_t)row_len, (uint32_t)chunks, status);
      break;
    case 8:
      LAUNCH(PK_GRAD, k_scatter_grad<uint64_t>, dim3((uint32_t)tiles), dim3(GRAD_NT), 0, st, (const uint64_t*)grad_y,
             perm, (uint64_t*)grad_x, (uint32_t)rows, (uint32_t)row_len, (uint32_t)chunks, status);
      break;
    default:
      return fail(SS_EINVAL, "elem_bytes = %d: need 2, 4 or 8", elem_bytes);
  }
  LAUNCH_CHECK();
  return SS_OK;
}

int ss_grad_status(void* stream) {
  g_err[0] = 0;
  hipStream_t st = as_stream(stream);
  HIP_TRY(hipStreamSynchronize(st));
  uint32_t v = 0, zero = 0;
  HIP_TRY(hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_grad_status), sizeof v, 0, hipMemcpyDeviceToHost));
  if (!v) return SS_OK;
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(g_grad_status), &zero, sizeof zero, 0, hipMemcpyHostToDevice));
  return fail(SS_EDEVICE, "ss_scatter_grad: a permutation index was outside its row (those entries were not "
                          "written; the flag is now cleared)");
}

int ss_set_tuning(const ss_tune_entry* entries, size_t count) {
  g_err[0] = 0;
  if (count && !entries) return fail(SS_EINVAL, "entries is NULL");
  TuneTab t[2][2][3];
  tune_builtin(t);
  for (size_t i = 0; i < count; i++) {
    const ss_tune_entry& e = entries[i];
    if (e.form > 1 || (e.key_bytes != 4 && e.key_bytes != 8) ||
        (e.val_bytes != 0 && e.val_bytes != 4 && e.val_bytes != 8) || e.size_class > 32)
      return fail(SS_EINVAL, "tuning entry %zu: form %u, key_bytes %u, val_bytes %u, size_class %u", i, e.form,
                  e.key_bytes, e.val_bytes, e.size_class);
    const bool auto_p = e.form == 1 && e.p == 0;
    if ((!auto_p && (e.p < 2 || e.p > SS_P_MAX || (e.p & (e.p - 1)))) || e.s < 1 || e.s > 4096 ||
        e.tile > (1u << 24))
      return fail(SS_EINVAL, "tuning entry %zu: p = %u, s = %u, tile = %u", i, e.p, e.s, e.tile);
    TuneTab& tt = t[e.form][e.key_bytes == 8][e.val_bytes == 0 ? 0 : (e.val_bytes == 4 ? 1 : 2)];
    tt.p[e.size_class] = (uint16_t)e.p;
    tt.s[e.size_class] = (uint16_t)e.s;
    tt.tile[e.size_class] = e.tile;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int f = 0; f < 2; f++)
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 3; b++) g_tune[f][a][b] = t[f][a][b];
  g_tune_ready = true;
  return SS_OK;
}

int ss_get_tuning(int form, int key_type, int val_type, size_t n, ss_params* out) {
  g_err[0] = 0;
  if (!out) return fail(SS_EINVAL, "out is NULL");
  if (form != 0 && form != 1) return fail(SS_EINVAL, "form %d: 0 (single array) or 1 (segmented)", form);
  Types ty;
  int rc = parse_types(key_type, val_type, &ty);
  if (rc) return rc;
  return check_params(nullptr, out, ty, n, form);
}

int ss_profile_enable(int on, int max_launches) {
  g_err[0] = 0;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on.store(false, std::memory_order_release);
  for (hipEvent_t e : g_prof.ev) (void)hipEventDestroy(e);
  g_prof.reset();
  if (!on) return SS_OK;
  if (max_launches < 1 || max_launches > (1 << 20)) return fail(SS_EINVAL, "max_launches out of range");
  g_prof.ev.resize(2 * (size_t)max_launches);
  g_prof.kind.resize(max_launches);
  for (auto& e : g_prof.ev) HIP_TRY(hipEventCreate(&e));
  g_prof.cap = max_launches;
  g_prof.on.store(true, std::memory_order_release);
  return SS_OK;
}

int ss_profile_kinds(unsigned kind_mask) {
  g_err[0] = 0;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.mask = kind_mask;
  return SS_OK;
}

int ss_profile_collect(void) {
  g_err[0] = 0;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (int i = 0; i < g_prof.used; i++) {
    HIP_TRY(hipEventSynchronize(g_prof.ev[2 * i + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]));
    g_prof.total[g_prof.kind[i]] += ms;
    g_prof.count[g_prof.kind[i]] += 1;
  }
  g_prof.used = 0;
  return SS_OK;
}

int ss_profile_report(int kind, const char** name, double* total_ms, uint64_t* launches) {
  if (kind < 0 || kind >= PK_COUNT) return SS_EINVAL;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (name) *name = PROF_NAMES[kind];
  if (total_ms) *total_ms = g_prof.total[kind];
  if (launches) *launches = g_prof.count[kind];
  return SS_OK;
}

static_assert(MAX_LEVELS == SS_MAX_LEVELS, "level count of the ABI");

int ss_level_stats(const void* ws, int level, ss_level_info* info, void* stream) {
  g_err[0] = 0;
  if (!ws || !info) return fail(SS_EINVAL, "ws or info is NULL");
  if (level < 0 || level >= MAX_LEVELS) return fail(SS_EINVAL, "level %d outside [0, %d)", level, MAX_LEVELS);
  HIP_TRY(hipStreamSynchronize(as_stream(stream)));
  LevelCtl c;
  HIP_TRY(hipMemcpy(&c, (const char*)ws + offsetof(Ctl, lv) + sizeof(LevelCtl) * level, sizeof c,
                    hipMemcpyDeviceToHost));
  info->segments = c.nsegs;
  info->buckets = c.total_buckets;
  info->keys = c.keys;
  info->bucket_keys = c.bucket_keys;
  return SS_OK;
}

int ss_status(const void* ws, void* stream) {
  g_err[0] = 0;
  if (!ws) return fail(SS_EINVAL, "ws is NULL");
  HIP_TRY(hipStreamSynchronize(as_stream(stream)));
  uint32_t st = 0;
  HIP_TRY(hipMemcpy(&st, ws, sizeof st, hipMemcpyDeviceToHost));
  if (st & ST_BAD_OFFSETS)
    return fail(SS_EDEVICE, "segment offsets decrease, leave [0, total) or exceed max_seg_len; those segments "
                            "were skipped (status 0x%x)", st);
  if (st) snprintf(g_err, sizeof g_err, "note: status 0x%x%s%s", st,
                   (st & ST_FALLBACK) ? " (a bucket was sorted by the one-work-group fallback)" : "",
                   (st & ST_LIST_FULL) ? " (a split-level list was full)" : "");
  return SS_OK;
}

}  // extern "C"
