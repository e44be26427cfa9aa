// Test infrastructure: a host emulation of the HIP device API that the
// kernel headers use, so that device functions can run on the CPU under
// AddressSanitizer.  One OS thread stands for one GPU thread of a single
// work-group: __syncthreads is a std::barrier over the work-group, and the
// cross-lane operations (ballot, shuffles, wave barrier) exchange values
// through a per-wave slot array between two barriers of the wave's 64
// threads.  Lanes of a wave are NOT in lockstep here, so code that relies
// on lockstep without a wave barrier shows up as a wrong result.  Nothing
// of the library includes this file.
#pragma once
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <barrier>
#include <cstdio>
#include <cstdlib>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__

struct dim3 {
  uint32_t x = 1, y = 1, z = 1;
};
extern thread_local dim3 threadIdx;
extern thread_local dim3 blockIdx;
extern dim3 blockDim, gridDim;

struct alignas(16) uint4 {
  uint32_t x, y, z, w;
};
struct alignas(8) uint2 {
  uint32_t x, y;
};
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return uint4{a, b, c, d}; }
inline uint2 make_uint2(uint32_t a, uint32_t b) { return uint2{a, b}; }

struct EmuWave {
  std::barrier<> bar{64};
  uint64_t v[64];
};
extern EmuWave* g_emu_waves;      // one per wave of the work-group
extern std::barrier<>* g_emu_block;

inline void __syncthreads() { g_emu_block->arrive_and_wait(); }
inline void __threadfence_block() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __builtin_amdgcn_wave_barrier() { g_emu_waves[threadIdx.x >> 6].bar.arrive_and_wait(); }
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
// streaming (non-temporal) accesses are ordinary ones on the host
#define __builtin_nontemporal_store(v, p) ((void)(*(p) = (v)))
#define __builtin_nontemporal_load(p) (*(p))

inline int emu_lane() { return threadIdx.x & 63; }

// every lane posts x, then reads lane src's value
template <class T>
inline T emu_xchg(T x, int src) {
  EmuWave& W = g_emu_waves[threadIdx.x >> 6];
  uint64_t b = 0;
  memcpy(&b, &x, sizeof(T));
  W.v[emu_lane()] = b;
  W.bar.arrive_and_wait();
  const uint64_t r = W.v[src & 63];
  W.bar.arrive_and_wait();
  T y;
  memcpy(&y, &r, sizeof(T));
  return y;
}

inline uint64_t __ballot(int pred) {
  EmuWave& W = g_emu_waves[threadIdx.x >> 6];
  W.v[emu_lane()] = pred ? 1 : 0;
  W.bar.arrive_and_wait();
  uint64_t m = 0;
  for (int i = 0; i < 64; i++) m |= W.v[i] ? (1ull << i) : 0ull;
  W.bar.arrive_and_wait();
  return m;
}
template <class T>
inline T __shfl(T x, int src, int width = 64) {
  const int l = emu_lane();
  return emu_xchg(x, (l & ~(width - 1)) + (src & (width - 1)));
}
template <class T>
inline T __shfl_xor(T x, int m, int width = 64) {
  (void)width;
  return emu_xchg(x, emu_lane() ^ m);
}
template <class T>
inline T __shfl_up(T x, unsigned d, int width = 64) {
  const int l = emu_lane();
  return emu_xchg(x, (int)((l & (width - 1)) >= (int)d ? l - (int)d : l));
}
template <class T>
inline T __builtin_amdgcn_readfirstlane(T x) {
  return emu_xchg(x, 0);
}
inline int __builtin_amdgcn_readlane(int x, int src) { return emu_xchg(x, src); }
inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t m, uint32_t acc) {
  const int l = emu_lane();
  return acc + __builtin_popcount(l >= 32 ? m : (m & ((1u << l) - 1u)));
}
inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t m, uint32_t acc) {
  const int l = emu_lane();
  return acc + __builtin_popcount(l <= 32 ? 0u : (m & ((1u << (l - 32)) - 1u)));
}

inline int __clz(int x) { return x ? __builtin_clz((unsigned)x) : 32; }
inline int __clzll(long long x) { return x ? __builtin_clzll((unsigned long long)x) : 64; }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __popc(unsigned x) { return __builtin_popcount(x); }
inline unsigned long long __umul64hi(unsigned long long a, unsigned long long b) {
  return (unsigned long long)(((unsigned __int128)a * b) >> 64);
}
inline unsigned __umulhi(unsigned a, unsigned b) { return (unsigned)(((uint64_t)a * b) >> 32); }

template <class T, class U>
inline T atomicAdd(T* p, U v) {
  return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST);
}
template <class T, class U>
inline T atomicOr(T* p, U v) {
  return __atomic_fetch_or(p, (T)v, __ATOMIC_SEQ_CST);
}
template <class T, class U>
inline T atomicMax(T* p, U v) {
  T o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (o < (T)v && !__atomic_compare_exchange_n(p, &o, (T)v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return o;
}

inline uint32_t min(uint32_t a, uint32_t b) { return a < b ? a : b; }
inline uint32_t max(uint32_t a, uint32_t b) { return a > b ? a : b; }
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline uint64_t min(uint64_t a, uint64_t b) { return a < b ? a : b; }
inline uint64_t max(uint64_t a, uint64_t b) { return a > b ? a : b; }

typedef int hipError_t;
typedef void* hipStream_t;
