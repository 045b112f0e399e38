// CPU emulation of the few HIP device features the contour engine uses, so
// that the unmodified device code can be compiled with g++ and run on the
// CPU for debugging and testing (test infrastructure only).  One wavefront
// is emulated by 64 std::threads in lockstep: every cross-lane operation
// (shuffle, ballot, barrier) is a rendezvous of all 64 threads.
#pragma once
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstring>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
// the CPU has one address space
#define TWK_GLOBAL_AS
#define TWK_LDS_AS
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))

namespace hip_emu {
constexpr int kLanes = 64;
struct Wave {
  std::barrier<> bar{kLanes};
  alignas(16) unsigned char buf[kLanes][8];
  uint64_t ballot_bits[kLanes];
};
inline Wave* g_wave = nullptr;
inline thread_local int t_lane = 0;
}  // namespace hip_emu

inline void __syncthreads() { hip_emu::g_wave->bar.arrive_and_wait(); }

template <class T>
inline T __hip_emu_exchange(T v, int src) {
  static_assert(sizeof(T) <= 8, "8-byte lanes");
  auto& W = *hip_emu::g_wave;
  std::memcpy(W.buf[hip_emu::t_lane], &v, sizeof(T));
  W.bar.arrive_and_wait();
  T r;
  std::memcpy(&r, W.buf[src & (hip_emu::kLanes - 1)], sizeof(T));
  W.bar.arrive_and_wait();
  return r;
}
template <class T>
inline T __shfl(T v, int src, int = 64) { return __hip_emu_exchange(v, src); }
template <class T>
inline T __shfl_up(T v, unsigned d, int = 64) {
  int s = hip_emu::t_lane - (int)d;
  T r = __hip_emu_exchange(v, s < 0 ? hip_emu::t_lane : s);
  return r;
}
template <class T>
inline T __shfl_xor(T v, int m, int = 64) { return __hip_emu_exchange(v, hip_emu::t_lane ^ m); }

inline unsigned long long __ballot(int pred) {
  auto& W = *hip_emu::g_wave;
  W.ballot_bits[hip_emu::t_lane] = pred ? 1ull : 0ull;
  W.bar.arrive_and_wait();
  unsigned long long m = 0;
  for (int i = 0; i < hip_emu::kLanes; ++i) m |= W.ballot_bits[i] << i;
  W.bar.arrive_and_wait();
  return m;
}
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
