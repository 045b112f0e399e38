// CPU emulation of the few HIP device features the contour engine uses, so
// that the unmodified device code can be compiled with g++ and run on the
// CPU for debugging and testing (test infrastructure only).  One wavefront
// is emulated by 64 cooperative fibers on one thread, run round-robin:
// every cross-lane operation (shuffle, ballot, barrier) is a rendezvous at
// which a lane yields to the next, so all 64 lanes have written before any
// reads.  The fibers switch stacks with a minimal x86-64 register switch
// (callee-saved registers and the stack pointer), no system call.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <cstdlib>

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

// emu_switch(save, to): push the callee-saved registers, store the stack
// pointer in *save, load `to` and pop the registers saved there.
// emu_start: first code of a fiber; calls r13(r12) (never returns).
asm(R"(
.text
.globl emu_switch
.type emu_switch, @function
emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size emu_switch, .-emu_switch
.globl emu_start
.type emu_start, @function
emu_start:
  movq %r12, %rdi
  call *%r13
  ud2
.size emu_start, .-emu_start
)");
extern "C" void emu_switch(void** save, void* to);
extern "C" void emu_start();

namespace hip_emu {
constexpr int kLanes = 64;
constexpr size_t kStack = 1 << 20;
struct Wave {
  alignas(16) unsigned char buf[kLanes][8];
  uint64_t ballot_bits[kLanes];
  void* lane_sp[kLanes];
  void* main_sp = nullptr;
  bool done[kLanes];
  char* stacks = nullptr;
};
inline Wave* g_wave = nullptr;
inline int t_lane = 0;

// Rendezvous: hand over to the scheduler, which runs the next lane.
inline void yield() { emu_switch(&g_wave->lane_sp[t_lane], g_wave->main_sp); }

struct LaneArg {
  void (*fn)(int, void*);
  void* ctx;
};
inline LaneArg g_lane_arg;

inline void lane_entry(void*) {
  const int l = t_lane;
  g_lane_arg.fn(l, g_lane_arg.ctx);
  g_wave->done[l] = true;
  emu_switch(&g_wave->lane_sp[l], g_wave->main_sp);  // never resumed
  std::abort();
}

// Run fn(lane, ctx) on 64 fibers in lockstep until every lane returns.
inline void run_wave(void (*fn)(int, void*), void* ctx) {
  Wave* w = new Wave();
  w->stacks = (char*)std::aligned_alloc(64, kStack * kLanes);
  g_wave = w;
  g_lane_arg = LaneArg{fn, ctx};
  for (int l = 0; l < kLanes; ++l) {
    w->done[l] = false;
    // initial frame: r15 r14 r13 r12 rbx rbp, then the return address into
    // emu_start; 16-byte alignment at the call inside emu_start
    uint64_t* top = (uint64_t*)(w->stacks + kStack * (l + 1));
    uint64_t* sp = top - 9;
    sp[0] = 0;                               // r15
    sp[1] = 0;                               // r14
    sp[2] = (uint64_t)(void*)&lane_entry;    // r13: function
    sp[3] = 0;                               // r12: argument
    sp[4] = 0;                               // rbx
    sp[5] = 0;                               // rbp
    sp[6] = (uint64_t)(void*)&emu_start;     // return address
    w->lane_sp[l] = sp;
  }
  int live = kLanes;
  while (live > 0) {
    live = 0;
    for (int l = 0; l < kLanes; ++l) {
      if (w->done[l]) continue;
      t_lane = l;
      emu_switch(&w->main_sp, w->lane_sp[l]);
      if (!w->done[l]) ++live;
    }
  }
  g_wave = nullptr;
  std::free(w->stacks);
  delete w;
}
}  // namespace hip_emu

inline void __syncthreads() { hip_emu::yield(); }
// The emulated lanes are fibers: a wave barrier is a rendezvous too.
inline void __builtin_amdgcn_wave_barrier() { hip_emu::yield(); }
// Memory fences order nothing here: the fibers of a wave share one address
// space and run one at a time.
#define __builtin_amdgcn_fence(order, scope) ((void)0)

template <class T>
inline T __hip_emu_exchange(T v, int src) {
  static_assert(sizeof(T) <= 8, "8-byte lanes");
  auto& W = *hip_emu::g_wave;
  std::memcpy(W.buf[hip_emu::t_lane], &v, sizeof(T));
  hip_emu::yield();
  T r;
  std::memcpy(&r, W.buf[src & (hip_emu::kLanes - 1)], sizeof(T));
  hip_emu::yield();
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
  hip_emu::yield();
  unsigned long long m = 0;
  for (int i = 0; i < hip_emu::kLanes; ++i) m |= W.ballot_bits[i] << i;
  hip_emu::yield();
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
