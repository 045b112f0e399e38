// twk.hip -- kernels and C ABI of the MI355X binary-lens magnification library.
//
// Paper: Wang, Wang & Dong, arXiv 2501.03322.  Declarations and argument
// contracts are in include/twk.h.
//
// Pipeline of a finite-source call (all on the caller's stream):
//   k_reset      clear the queue counters (a kernel, not a memset, so that
//                the sequence may be captured in a graph)
//   k_prep/k_lc  one lane per source: centre (and stencil) point solves,
//                point-source adequacy test (Sec. 2.3); adequate sources get
//                the point value, the rest are appended to the task queue
//                with their centre roots (wave-aggregated atomics)
//   k_fs<C>      persistent: each 64-lane wave pops tasks from the queue and
//                runs the adaptive contour integration, keeping up to C limb
//                samples' sorted arrays in LDS and continuing in its global
//                slice for larger sources (method cap 4096).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../include/twk.h"
#include "twk_device.h"
#include "twk_fs.h"

using namespace twk;

namespace {

constexpr int LDS_CAP = 512;  // limb samples a source keeps in LDS before spilling

// Counters in device memory (int64 each).
enum {
  C_NTASK = 0,     // tasks queued by the point-source pass
  C_HEAD = 1,      // queue head of the first FS pass
  C_NOVER = 2,     // tasks whose sorted arrays outgrew LDS
  C_HEAD2 = 3,     // unused
  C_SAMPLES = 4,   // limb samples of finished tasks
  C_SW32 = 5,      // FP32 root sweeps (5 roots each)
  C_SW64 = 6,      // FP64 root sweeps
  C_INTERVALS = 7, // intervals linked
  C_RUNS = 8,      // FS runs (including those deferred and re-run)
  C_SPARE = 15,
  C_NCOUNTERS = 16
};

// Point-source adequacy test.  The paper (Sec. 2.3) applies the quadrupole
// test and the ghost-image test before any contour work but gives no
// formulas; the reading used here:
//  - quadrupole: with mu0 at the centre and mean4 the mean of mu at the four
//    points zeta_c +- rho, zeta_c +- i rho, the disk mean exceeds mu0 by
//    about (mean4 - mu0)/2; require CQ |(mean4 - mu0)/2| < tol mu0;
//  - all five points have exactly three images;
//  - ghost test: |f''(g)| |R_g|^2 estimates the distance of the source to
//    the caustic from each ghost g; require it > CG rho everywhere.
constexpr double PS_CQ = 20.0;
constexpr double PS_CG = 8.0;

__device__ inline double ghost_stat(const Lens& L, c64 y, c64 g) {
  c64 eb = cconj(g);
  c64 R = y - g + L.m1 * cinv(eb + L.s) + L.m2 * cinv(eb);
  c64 a1 = g + L.s;
  c64 f2 = -2.0 * (L.m1 * cinv(a1 * a1 * a1) + L.m2 * cinv(g * g * g));
  return cabs64(f2) * cnorm(R);
}

struct PsResult {
  double mu;
  int n;
  uint32_t flags;
  bool adequate;
  c64 roots[5];
};

__device__ inline PsResult point_source_pass(const Lens& L, c64 yc, double rho, double tol,
                                             bool test) {
  PsResult out;
  c64 c[6], r[5];
  coefficients(L, yc, c);
  cold_start(c, r);
  aberth64(c, r, 200);
  Images im;
  finish_images(L, yc, r, im);
  out.mu = point_mag(im);
  out.n = im.n;
  out.flags = im.flags;
#pragma unroll
  for (int k = 0; k < 5; ++k) out.roots[k] = im.z[k];
  if (!test) {
    out.adequate = false;
    return out;
  }
  bool ok = im.n == 3;
  for (int g = 3; g < 5; ++g)
    if (!(ghost_stat(L, yc, im.z[g]) > PS_CG * rho)) ok = false;
  double mus = 0.0;
  const c64 off[4] = {cz(rho, 0.0), cz(0.0, rho), cz(-rho, 0.0), cz(0.0, -rho)};
  for (int k = 0; k < 4; ++k) {
    const c64 y = yc + off[k];
    coefficients(L, y, c);
#pragma unroll
    for (int j = 0; j < 5; ++j) r[j] = out.roots[j];
    if (aberth64(c, r, 60) > 60) {
      cold_start(c, r);
      aberth64(c, r, 200);
    }
    Images ik;
    finish_images(L, y, r, ik);
    mus += point_mag(ik);
    if (ik.n != 3) ok = false;
    for (int g = 3; g < 5; ++g)
      if (!(ghost_stat(L, y, ik.z[g]) > PS_CG * rho)) ok = false;
  }
  const double dq = 0.5 * (0.25 * mus - out.mu);
  if (!(PS_CQ * fabs(dq) < tol * out.mu)) ok = false;
  out.adequate = ok;
  return out;
}

__global__ void k_reset(long long* cnt) {
  if (threadIdx.x < C_NCOUNTERS) cnt[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_point(double s, double q, int64_t n, const double* zx,
                                               const double* zy, double* mag, int32_t* nimg,
                                               uint32_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = zx[i], y = zy[i];
  if (!isfinite(x) || !isfinite(y)) {
    mag[i] = __builtin_nan("");
    nimg[i] = 0;
    flags[i] = F_NONFINITE;
    return;
  }
  const Lens L = make_lens(s, q);
  Images im;
  int it;
  solve_point_cold(L, cz(x - L.z2, y), im, it);
  mag[i] = point_mag(im);
  nimg[i] = im.n;
  flags[i] = im.flags;
}

// Append the calling lanes with `push` set to the task queue: one atomic
// per wave.
__device__ inline int64_t queue_push(bool push, long long* count) {
  const uint64_t mask = __ballot(push);
  if (mask == 0) return -1;
  const int lane = threadIdx.x & (WAVE - 1);
  const int leader = __ffsll((unsigned long long)mask) - 1;
  long long base = 0;
  if (lane == leader) base = atomicAdd((unsigned long long*)count, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  if (!push) return -1;
  return base + __popcll(mask & ((1ull << lane) - 1ull));
}

__device__ inline void emit_source(int64_t out, double s, double q, double zx, double zy,
                                   double rho, double tol, bool all_fs, Task* tasks,
                                   long long* cnt, double* mag, double* err, int32_t* ns,
                                   uint32_t* flags, bool active) {
  bool push = false;
  PsResult ps;
  const Lens L = make_lens(s, q);
  const bool finite = isfinite(zx) && isfinite(zy);
  if (active) {
    if (!finite) {
      mag[out] = __builtin_nan("");
      err[out] = __builtin_nan("");
      ns[out] = 0;
      flags[out] = F_NONFINITE;
    } else {
      ps = point_source_pass(L, cz(zx - L.z2, zy), rho, tol, !all_fs);
      if (ps.adequate) {
        mag[out] = ps.mu;
        err[out] = 0.0;
        ns[out] = 0;
        flags[out] = F_POINT | ps.flags;
      } else {
        push = true;
      }
    }
  }
  const int64_t slot = queue_push(push, &cnt[C_NTASK]);
  if (push) {
    Task t;
    t.out = out;
    t.s = s;
    t.q = q;
    t.rho = rho;
    t.zx = zx;
    t.zy = zy;
#pragma unroll
    for (int k = 0; k < 5; ++k) t.roots[k] = ps.roots[k];
    tasks[slot] = t;
  }
}

__global__ __launch_bounds__(256) void k_prep(double s, double q, int64_t n, const double* zx,
                                              const double* zy, double rho, double tol,
                                              int all_fs, Task* tasks, long long* cnt,
                                              double* mag, double* err, int32_t* ns,
                                              uint32_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < n;
  emit_source(i, s, q, active ? zx[i] : 0.0, active ? zy[i] : 0.0, rho, tol, all_fs != 0, tasks,
              cnt, mag, err, ns, flags, active);
}

// Light curves: element (set k, epoch j) at index k * nepochs + j.  Source
// centre on the straight trajectory of set k (centre-of-mass frame).
__global__ __launch_bounds__(256) void k_lc(int64_t nsets, const double* ps, const double* pq,
                                            const double* pu0, const double* pal,
                                            const double* prho, int64_t nep,
                                            const double* tau, double tol, int all_fs,
                                            Task* tasks, long long* cnt, double* mag,
                                            double* err, int32_t* ns, uint32_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < nsets * nep;
  double s = 1.0, q = 1.0, zx = 0.0, zy = 0.0, rho = 1.0;
  if (active) {
    const int64_t k = i / nep, j = i - k * nep;
    s = ps[k];
    q = pq[k];
    rho = prho[k];
    double sa, ca;
    sincos(pal[k], &sa, &ca);
    const double t = tau[j], u0 = pu0[k];
    zx = t * ca - u0 * sa;
    zy = t * sa + u0 * ca;
  }
  emit_source(i, s, q, zx, zy, rho, tol, all_fs != 0, tasks, cnt, mag, err, ns, flags, active);
}

// Persistent finite-source kernel: each wave pops tasks until the queue is
// drained (every wave reaches the exit: the queue length is fixed before
// launch and each pop advances the head).
template <int LCAP, bool MIXED>
#ifndef TWK_FS_WAVES_PER_EU
#define TWK_FS_WAVES_PER_EU 2
#endif
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TWK_FS_WAVES_PER_EU))) void k_fs(const Task* tasks, const long long* ntask,
                                           long long* head, double tol, char* scratch,
                                           double* mag, double* err, int32_t* ns,
                                           uint32_t* flags, long long* cnt) {
  __shared__ FsLds<LCAP> lds;
  const int lane = threadIdx.x;
  const WaveMem m = wave_mem(scratch, blockIdx.x, METHOD_CAP);
  const long long n = *ntask;
  for (;;) {
    long long t = 0;
    if (lane == 0) t = atomicAdd((unsigned long long*)head, 1ull);
    t = __shfl(t, 0);
    if (t >= n) break;
    const Task task = tasks[t];
    const FsOut o = fs_source<LCAP, MIXED>(task, tol, m, lds, lane);
    if (lane == 0) {
      mag[task.out] = o.mag;
      err[task.out] = o.err;
      ns[task.out] = o.n;
      flags[task.out] = o.flags;
      atomicAdd((unsigned long long*)&cnt[C_SAMPLES], (unsigned long long)o.n);
      atomicAdd((unsigned long long*)&cnt[C_SW32], (unsigned long long)o.sweeps32);
      atomicAdd((unsigned long long*)&cnt[C_SW64], (unsigned long long)o.sweeps64);
      atomicAdd((unsigned long long*)&cnt[C_INTERVALS], (unsigned long long)o.intervals);
      atomicAdd((unsigned long long*)&cnt[C_RUNS], 1ull);
      if (o.spilled) atomicAdd((unsigned long long*)&cnt[C_NOVER], 1ull);
    }
    __syncthreads();
  }
}

}  // namespace

// ------------------------------------------------------------------ host
struct twk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  int last_err = 0;
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
  Task* tasks = nullptr;
  int64_t task_cap = 0;
  long long* cnt = nullptr;
  int waves = 0;
  bool timing = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

int hip_fail(twk_ctx* c, hipError_t e) {
  c->last_err = (int)e;
  return TWK_EDEVICE;
}

#define HIP_TRY(c, expr)                        \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(c, e_); \
  } while (0)

int grow(twk_ctx* c, void** p, size_t* have, size_t need) {
  if (*have >= need) return TWK_OK;
  if (*p) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e);
    (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
  }
  if (hipMalloc(p, need) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return TWK_ENOMEM;
  }
  *have = need;
  return TWK_OK;
}

template <bool MIXED>
int occupancy(int* blocks) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_fs<LDS_CAP, MIXED>, 64, 0);
}

int ensure_fs(twk_ctx* c, int64_t ntask_max) {
  int rc;
  size_t have = (size_t)c->task_cap * sizeof(Task);
  if ((rc = grow(c, (void**)&c->tasks, &have, (size_t)std::max<int64_t>(ntask_max, 1) * sizeof(Task))))
    return rc;
  c->task_cap = (int64_t)(have / sizeof(Task));
  const size_t need = (size_t)c->waves * METHOD_CAP * kSlotBytes;
  return grow(c, (void**)&c->scratch, &c->scratch_bytes, need);
}

template <bool MIXED>
int launch_fs(twk_ctx* c, double tol, double* mag, double* err, int32_t* ns, uint32_t* flags) {
  if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
  hipLaunchKernelGGL((k_fs<LDS_CAP, MIXED>), dim3(c->waves), dim3(64), 0, c->stream, c->tasks,
                     &c->cnt[C_NTASK], &c->cnt[C_HEAD], tol, c->scratch, mag, err, ns, flags,
                     c->cnt);
  HIP_TRY(c, hipGetLastError());
  if (c->timing) {
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
  }
  return TWK_OK;
}

bool finite_pos(double v) { return v > 0.0 && v < 1e300; }

}  // namespace

extern "C" {

const char* twk_strerror(int status) {
  switch (status) {
    case TWK_OK: return "ok";
    case TWK_EINVAL: return "invalid argument";
    case TWK_EDEVICE: return "HIP device error";
    case TWK_ENOMEM: return "device memory allocation failed";
    case TWK_ENOMLP: return "learned predictor requested but no weights loaded";
    default: return "unknown status";
  }
}

int twk_create(twk_ctx** out, int device, void* stream) {
  if (!out) return TWK_EINVAL;
  *out = nullptr;
  twk_ctx* c = new (std::nothrow) twk_ctx();
  if (!c) return TWK_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) {
    delete c;
    return TWK_EDEVICE;
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete c;
    return TWK_EDEVICE;
  }
  c->n_cu = prop.multiProcessorCount;
  int b1 = 0, b2 = 0;
  if (occupancy<false>(&b1) != hipSuccess || occupancy<true>(&b2) != hipSuccess) {
    delete c;
    return TWK_EDEVICE;
  }
  c->waves = std::max(1, std::min(b1, b2)) * c->n_cu;
  if (hipMalloc((void**)&c->cnt, C_NCOUNTERS * sizeof(long long)) != hipSuccess) {
    delete c;
    return TWK_ENOMEM;
  }
  *out = c;
  return TWK_OK;
}

int twk_destroy(twk_ctx* c) {
  if (!c) return TWK_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->scratch);
  (void)hipFree(c->tasks);
  (void)hipFree(c->cnt);
  for (int i = 0; i < 4; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  delete c;
  return TWK_OK;
}

int twk_sync(twk_ctx* c) {
  if (!c) return TWK_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TWK_OK;
}

int twk_last_hip_error(const twk_ctx* c) { return c ? c->last_err : 0; }

int twk_point_mag(twk_ctx* c, double s, double q, int64_t n, const double* zx, const double* zy,
                  double* mag, int32_t* nimg, uint32_t* flags) {
  if (!c || !finite_pos(s) || !finite_pos(q) || n < 0) return TWK_EINVAL;
  if (n == 0) return TWK_OK;
  if (!zx || !zy || !mag || !nimg || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_point, dim3((unsigned)blocks), dim3(256), 0, c->stream, s, q, n, zx, zy, mag,
                     nimg, flags);
  HIP_TRY(c, hipGetLastError());
  return TWK_OK;
}

int twk_finite_mag(twk_ctx* c, double s, double q, int64_t n, const double* zx, const double* zy,
                   double rho, double tol, uint32_t mode, double* mag, double* err, int32_t* ns,
                   uint32_t* flags) {
  if (!c || !finite_pos(s) || !finite_pos(q) || !finite_pos(rho) || !finite_pos(tol) || n < 0)
    return TWK_EINVAL;
  if (mode & ~(TWK_MODE_MIXED | TWK_MODE_ALL_FS)) return TWK_EINVAL;
  if (n == 0) return TWK_OK;
  if (!zx || !zy || !mag || !err || !ns || !flags) return TWK_EINVAL;
  if (n > (int64_t)1 << 40) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  int rc = ensure_fs(c, n);
  if (rc) return rc;
  if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->stream, c->cnt);
  HIP_TRY(c, hipGetLastError());
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)blocks), dim3(256), 0, c->stream, s, q, n, zx, zy, rho,
                     tol, (mode & TWK_MODE_ALL_FS) ? 1 : 0, c->tasks, c->cnt, mag, err, ns, flags);
  HIP_TRY(c, hipGetLastError());
  return (mode & TWK_MODE_MIXED) ? launch_fs<true>(c, tol, mag, err, ns, flags)
                                 : launch_fs<false>(c, tol, mag, err, ns, flags);
}

int twk_lightcurves(twk_ctx* c, int64_t nsets, const double* s, const double* q, const double* u0,
                    const double* alpha, const double* rho, const double* gamma, int64_t nepochs,
                    const double* tau, int32_t n_annuli, double tol, uint32_t mode, double* mag,
                    double* err, int32_t* ns, uint32_t* flags) {
  if (!c || nsets < 0 || nepochs < 0 || !finite_pos(tol) || n_annuli < 1) return TWK_EINVAL;
  if (mode & ~(TWK_MODE_MIXED | TWK_MODE_ALL_FS)) return TWK_EINVAL;
  if (gamma != nullptr && n_annuli != 1) return TWK_EINVAL;  // limb darkening: not yet wired
  const int64_t n = nsets * nepochs;
  if (n == 0) return TWK_OK;
  if (!s || !q || !u0 || !alpha || !rho || !tau || !mag || !err || !ns || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  int rc = ensure_fs(c, n);
  if (rc) return rc;
  if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->stream, c->cnt);
  HIP_TRY(c, hipGetLastError());
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_lc, dim3((unsigned)blocks), dim3(256), 0, c->stream, nsets, s, q, u0, alpha,
                     rho, nepochs, tau, tol, (mode & TWK_MODE_ALL_FS) ? 1 : 0, c->tasks, c->cnt,
                     mag, err, ns, flags);
  HIP_TRY(c, hipGetLastError());
  return (mode & TWK_MODE_MIXED) ? launch_fs<true>(c, tol, mag, err, ns, flags)
                                 : launch_fs<false>(c, tol, mag, err, ns, flags);
}

int twk_last_stats(twk_ctx* c, int64_t* out8) {
  if (!c || !out8) return TWK_EINVAL;
  long long h[C_NCOUNTERS];
  HIP_TRY(c, hipMemcpyAsync(h, c->cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  out8[0] = h[C_NTASK];
  out8[1] = h[C_NOVER];
  out8[2] = h[C_SAMPLES];
  out8[3] = c->waves;
  out8[4] = h[C_SW32];
  out8[5] = h[C_SW64];
  out8[6] = h[C_INTERVALS];
  out8[7] = h[C_RUNS];
  return TWK_OK;
}

int twk_enable_timing(twk_ctx* c, int on) {
  if (!c) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  if (on && !c->ev[0])
    for (int i = 0; i < 4; ++i) HIP_TRY(c, hipEventCreate(&c->ev[i]));
  c->timing = on != 0;
  return TWK_OK;
}

int twk_kernel_times(twk_ctx* c, double* ms4) {
  if (!c || !ms4 || !c->timing) return TWK_EINVAL;
  HIP_TRY(c, hipEventSynchronize(c->ev[3]));
  float a = 0.f, b = 0.f, d = 0.f, t = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
  HIP_TRY(c, hipEventElapsedTime(&b, c->ev[1], c->ev[2]));
  HIP_TRY(c, hipEventElapsedTime(&d, c->ev[2], c->ev[3]));
  HIP_TRY(c, hipEventElapsedTime(&t, c->ev[0], c->ev[3]));
  ms4[0] = a;
  ms4[1] = b;
  ms4[2] = d;
  ms4[3] = t;
  return TWK_OK;
}

}  // extern "C"
