// Test infrastructure: runs the round-based slot sort (the bucket sort of the
// wide split and of handed-on level buckets) for one 1024-thread work-group
// on the host, through the HIP emulation in hip/hip_runtime.h, on generated
// buckets, and checks every sorted bucket against std::sort.  Built with
// AddressSanitizer by tests/test_emu_slot_sort.py; prints one summary line
// and exits non-zero on a wrong bucket.
#include "../../paper_1608_08648_amd/csrc/ss_wide.h"

#include <algorithm>
#include <thread>
#include <vector>

thread_local dim3 threadIdx;
thread_local dim3 blockIdx;
dim3 blockDim, gridDim;
EmuWave* g_emu_waves;
std::barrier<>* g_emu_block;

using namespace ss;

namespace {

struct Case {
  uint32_t len;
  bool lo_k, hi_k;
  uint32_t lo, hi;
  bool alias;            // input == output
  bool may_fall_back;    // crowded slots allowed to hand the bucket on
  std::vector<uint32_t> keys;
};

struct Rng {              // xorshift64*, test data only
  uint64_t s;
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 2685821657736338717ull;
  }
};

std::vector<Case> make_cases() {
  std::vector<Case> cs;
  Rng r{0x9E3779B97F4A7C15ull};
  const uint32_t sizes[] = {1, 2, 100, 5000, 16000, 30464, 30465, 45000, 65535, 70000, 130000};
  for (uint32_t len : sizes) {
    for (int kind = 0; kind < 4; kind++) {
      Case c{len, false, false, 0, 0, false, false, {}};
      c.keys.resize(len);
      for (uint32_t i = 0; i < len; i++) {
        const uint32_t u = (uint32_t)(r.next() >> 32);
        if (kind == 0) c.keys[i] = u;                                   // full range
        else if (kind == 1) c.keys[i] = 1000 + u % (3 * len + 1);       // dense range
        else if (kind == 2) c.keys[i] = u % (len / 40 + 1);             // ~40 per value
        else c.keys[i] = (i % 7 == 0) ? 99u : 12345u;                   // two values
      }
      c.may_fall_back = kind >= 2;
      if (kind == 1 && len > 2) {   // bucket bounds known (keys within them)
        c.lo_k = c.hi_k = true;
        c.lo = 999;
        c.hi = 1001 + 3 * len;
      }
      cs.push_back(std::move(c));
    }
  }
  // input == output with more than one round: must be refused untouched
  Case a{45000, false, false, 0, 0, true, true, {}};
  a.keys.resize(a.len);
  for (auto& k : a.keys) k = (uint32_t)(r.next() >> 32);
  cs.push_back(std::move(a));
  return cs;
}

}  // namespace

// one pass over all cases with the slot sort's LDS laid out for CAP keys a
// round over 2^LG2 slots; returns the number of wrong buckets
template <int CAP, int LG2>
size_t run_cases(const std::vector<Case>& cs, const char* name) {
  constexpr int NTH = WIDE_BNT;
  static SlotRoundsLds<CAP, LG2> sm;
  std::vector<uint32_t*> ins(cs.size()), outs(cs.size());
  std::vector<int> res(cs.size(), -1);
  for (size_t i = 0; i < cs.size(); i++) {
    ins[i] = new uint32_t[cs[i].len];   // exact sizes: AddressSanitizer sees any overrun
    std::copy(cs[i].keys.begin(), cs[i].keys.end(), ins[i]);
    outs[i] = cs[i].alias ? ins[i] : new uint32_t[cs[i].len];
  }
  std::vector<std::thread> th;
  for (int t = 0; t < NTH; t++)
    th.emplace_back([&, t] {
      threadIdx.x = t;
      for (size_t i = 0; i < cs.size(); i++) {
        const Case& c = cs[i];
        const bool ok = c.len <= WIDE_BMAX
                            ? slot_sort_rounds<NTH, CAP, true, LG2>(ins[i], outs[i], c.len, 0, sm, c.lo_k, c.lo,
                                                                    c.hi_k, c.hi)
                            : slot_sort_rounds<NTH, CAP, false, LG2>(ins[i], outs[i], c.len, 0, sm, c.lo_k, c.lo,
                                                                     c.hi_k, c.hi);
        if (t == 0) res[i] = ok ? 1 : 0;
        __syncthreads();
      }
    });
  for (auto& x : th) x.join();
  size_t wrong = 0, fell_back = 0;
  for (size_t i = 0; i < cs.size(); i++) {
    const Case& c = cs[i];
    if (c.alias) {   // refused, and the buffer left as it was
      if (res[i] != 0 || !std::equal(c.keys.begin(), c.keys.end(), ins[i])) {
        printf("%s: aliased case len %u: not refused untouched\n", name, c.len);
        wrong++;
      }
      continue;
    }
    if (res[i] == 0) {
      fell_back++;
      if (!c.may_fall_back) {
        printf("%s: case %zu len %u handed on unexpectedly\n", name, i, c.len);
        wrong++;
      }
      continue;
    }
    std::vector<uint32_t> w = c.keys;
    std::sort(w.begin(), w.end());
    if (!std::equal(w.begin(), w.end(), outs[i])) {
      printf("%s: case %zu len %u: wrong order\n", name, i, c.len);
      wrong++;
    }
  }
  for (size_t i = 0; i < cs.size(); i++) {
    if (outs[i] != ins[i]) delete[] outs[i];
    delete[] ins[i];
  }
  printf("%s: buckets %zu wrong %zu handed_on %zu\n", name, cs.size(), wrong, fell_back);
  return wrong;
}

int main() {
  std::vector<Case> cs = make_cases();
  g_emu_waves = new EmuWave[WIDE_BNT / 64];
  g_emu_block = new std::barrier<>(WIDE_BNT);
  size_t wrong = run_cases<WIDE_BCAP, ROUNDS_LOG2>(cs, "30720 keys, 2^14 slots");
  wrong += run_cases<WIDE_SCAP, WIDE_SLG>(cs, "16000 keys, 2^13 slots");
  printf("total wrong %zu \n", wrong);
  return wrong ? 1 : 0;
}
