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
#include <cstdio>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
// the CPU has one address space
#define TWK_GLOBAL_AS
#define TWK_LDS_AS
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
#define __builtin_amdgcn_sqrtf(x) std::sqrt((float)(x))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt((double)(x)))
#define __builtin_amdgcn_exp2f(x) std::exp2((float)(x))

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
// The emulated lanes are threads: a wave barrier must synchronise them too.
inline void __builtin_amdgcn_wave_barrier() { hip_emu::g_wave->bar.arrive_and_wait(); }

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

// DPP lane moves of one 32-bit value (the controls the engine uses:
// row_shr:1..15, row_bcast:15, row_bcast:31, wave_shr:1).  Lanes of rows or
// banks outside the masks keep `old`; lanes whose source does not exist get
// 0 with bound_ctrl, else `old`.
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask,
                                       bool bound_ctrl) {
  const int l = hip_emu::t_lane, row = l >> 4, lr = l & 15;
  int from = -1;
  if (ctrl >= 0x111 && ctrl <= 0x11F) {
    const int k = ctrl - 0x110;
    from = lr >= k ? l - k : -1;
  } else if (ctrl == 0x142) {
    from = row >= 1 ? row * 16 - 1 : -1;
  } else if (ctrl == 0x143) {
    from = row >= 2 ? 31 : -1;
  } else if (ctrl == 0x138) {
    from = l >= 1 ? l - 1 : -1;
  } else {
    __builtin_trap();  // control not modelled
  }
  const int v = __hip_emu_exchange(src, from >= 0 ? from : l);
  const bool on = ((row_mask >> row) & 1) && ((bank_mask >> (lr >> 2)) & 1);
  if (!on) return old;
  if (from < 0) return bound_ctrl ? 0 : old;
  return v;
}
inline int __builtin_amdgcn_readlane(int v, int lane) { return __hip_emu_exchange(v, lane); }
