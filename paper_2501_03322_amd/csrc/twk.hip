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
#include <cmath>
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
  C_RUNS = 8,      // contour runs
  C_NFS = 9,       // limb-darkened epochs sent to the annulus contours
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

// Clear all counters (start of a call) or only the queue counters (start of
// a chunk of a call).
__global__ void k_reset(long long* cnt, int queue_only) {
  const int i = threadIdx.x;
  if (i >= C_NCOUNTERS) return;
  if (!queue_only || i == C_NTASK || i == C_HEAD || i == C_NFS) cnt[i] = 0;
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

// Append `count` entries per calling lane (0 or a lane-uniform k) to a
// queue: one atomic per wave; returns this lane's first slot.
__device__ inline int64_t queue_push(bool push, int count, long long* counter) {
  const uint64_t mask = __ballot(push);
  if (mask == 0) return -1;
  const int lane = threadIdx.x & (WAVE - 1);
  const int leader = __ffsll((unsigned long long)mask) - 1;
  long long base = 0;
  if (lane == leader)
    base = atomicAdd((unsigned long long*)counter, (unsigned long long)(__popcll(mask) * count));
  base = __shfl(base, leader);
  if (!push) return -1;
  return base + (long long)count * __popcll(mask & ((1ull << lane) - 1ull));
}

// Point-source pass for one source: answer it by the point value when the
// point-source test passes, else queue its contour task(s).  With na > 1
// annuli (limb darkening), the source is recorded in fs_epoch[] and na
// uniform-disk tasks of radii rho sqrt(k/na), k = 1..na, are queued; their
// results land in the annulus buffers at f*na + k - 1.
__device__ inline void emit_source(int64_t out, double s, double q, double zx, double zy,
                                   double rho, double tol, bool all_fs, int na, Task* tasks,
                                   long long* cnt, int64_t* fs_epoch, double* mag, double* err,
                                   int32_t* ns, uint32_t* flags, bool active) {
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
  int64_t first_out = out;
  if (na > 1) {
    const int64_t f = queue_push(push, 1, &cnt[C_NFS]);
    if (push) {
      fs_epoch[f] = out;
      first_out = f * na;
    }
  }
  const int64_t slot = queue_push(push, na, &cnt[C_NTASK]);
  if (push) {
    Task t;
    t.s = s;
    t.q = q;
    t.zx = zx;
    t.zy = zy;
#pragma unroll
    for (int k = 0; k < 5; ++k) t.roots[k] = ps.roots[k];
    for (int k = 0; k < na; ++k) {
      t.out = first_out + k;
      t.rho = na > 1 ? rho * sqrt((double)(k + 1) / na) : rho;
      tasks[slot + k] = t;
    }
  }
}

__global__ __launch_bounds__(256) void k_prep(double s, double q, int64_t n, const double* zx,
                                              const double* zy, double rho, double tol,
                                              int all_fs, Task* tasks, long long* cnt,
                                              double* mag, double* err, int32_t* ns,
                                              uint32_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < n;
  emit_source(i, s, q, active ? zx[i] : 0.0, active ? zy[i] : 0.0, rho, tol, all_fs != 0, 1, tasks,
              cnt, nullptr, mag, err, ns, flags, active);
}

// Magnification map: pixel (ix, iy) of an nx x ny grid over the box
// [xc - w/2, xc + w/2] x [yc - h/2, yc + h/2], pixel centres, output index
// iy * nx + ix (rows iy0 .. iy0 + nrows - 1 in this launch).
__global__ __launch_bounds__(256) void k_map(double s, double q, double rho, double xc, double yc,
                                             double w, double h, int32_t nx, int32_t ny,
                                             int64_t iy0, int64_t nrows, double tol, int all_fs,
                                             Task* tasks, long long* cnt, double* mag,
                                             double* err, int32_t* ns, uint32_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < nrows * (int64_t)nx;
  double zx = 0.0, zy = 0.0;
  int64_t out = 0;
  if (active) {
    const int64_t iy = iy0 + i / nx, ix = i % nx;
    zx = xc - 0.5 * w + (ix + 0.5) * (w / nx);
    zy = yc - 0.5 * h + (iy + 0.5) * (h / ny);
    out = iy * nx + ix;
  }
  emit_source(out, s, q, zx, zy, rho, tol, all_fs != 0, 1, tasks, cnt, nullptr, mag, err, ns,
              flags, active);
}

// Light curves: element (set k, epoch j) at index k * nepochs + j.  Source
// centre on the straight trajectory of set k (centre-of-mass frame).
__global__ __launch_bounds__(256) void k_lc(int64_t nsets, const double* ps, const double* pq,
                                            const double* pu0, const double* pal,
                                            const double* prho, int64_t nep,
                                            const double* tau, double tol, int all_fs, int na,
                                            Task* tasks, long long* cnt, int64_t* fs_epoch,
                                            double* mag, double* err, int32_t* ns,
                                            uint32_t* flags) {
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
  emit_source(i, s, q, zx, zy, rho, tol, all_fs != 0, na, tasks, cnt, fs_epoch, mag, err, ns,
              flags, active);
}

// Linear limb darkening over na equal-area annuli (x_k = k/na of the squared
// radius): I(r)/mean = 1 - G (1 - 1.5 sqrt(1 - r^2/rho^2)); the annulus mean
// is I_k = 1 - G + G [(1 - x_{k-1})^1.5 - (1 - x_k)^1.5] / (x_k - x_{k-1}).
// The flux of annulus k is I_k (x_k mu_k - x_{k-1} mu_{k-1}) with mu_k the
// uniform-disk magnification of the disk of squared radius x_k rho^2.
__global__ __launch_bounds__(256) void k_ld(const long long* cnt, const int64_t* fs_epoch,
                                            int na, const double* gamma, int64_t nep,
                                            const double* amag, const double* aerr,
                                            const int32_t* ans, const uint32_t* afl, double* mag,
                                            double* err, int32_t* ns, uint32_t* flags) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= cnt[C_NFS]) return;
  const int64_t i = fs_epoch[f];
  const double G = gamma[i / nep];
  double num = 0.0, den = 0.0, e = 0.0, xp = 0.0, mp = 0.0, ep = 0.0;
  int32_t nsum = 0;
  uint32_t fl = 0;
  for (int k = 1; k <= na; ++k) {
    const double x = (double)k / na;
    const double Ik = 1.0 - G + G * (pow(1.0 - xp, 1.5) - pow(1.0 - x, 1.5)) / (x - xp);
    const double mk = amag[f * na + k - 1], ek = aerr[f * na + k - 1];
    num += Ik * (x * mk - xp * mp);
    den += Ik * (x - xp);
    e += Ik * (x * ek + xp * ep);
    nsum += ans[f * na + k - 1];
    fl |= afl[f * na + k - 1];
    xp = x;
    mp = mk;
    ep = ek;
  }
  mag[i] = num / den;
  err[i] = e / den;
  ns[i] = nsum;
  flags[i] = fl;
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
  // limb darkening: epochs sent to the annulus contours and their results
  int64_t* fs_epoch = nullptr;
  size_t fs_epoch_bytes = 0;
  char* ann = nullptr;  // [mag f64 | err f64 | ns i32 | flags u32] x (nfs * na)
  size_t ann_bytes = 0;
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

// Task records per chunk of a call: bounds the queue memory (128 B each).
constexpr int64_t CHUNK_TASKS = (int64_t)1 << 24;

int ensure_fs(twk_ctx* c, int64_t ntask_max) {
  int rc;
  size_t have = (size_t)c->task_cap * sizeof(Task);
  if ((rc = grow(c, (void**)&c->tasks, &have, (size_t)std::max<int64_t>(ntask_max, 1) * sizeof(Task))))
    return rc;
  c->task_cap = (int64_t)(have / sizeof(Task));
  const size_t need = (size_t)c->waves * METHOD_CAP * kSlotBytes;
  return grow(c, (void**)&c->scratch, &c->scratch_bytes, need);
}

int ensure_ld(twk_ctx* c, int64_t nfs_max, int na) {
  int rc;
  if ((rc = grow(c, (void**)&c->fs_epoch, &c->fs_epoch_bytes,
                 (size_t)std::max<int64_t>(nfs_max, 1) * sizeof(int64_t))))
    return rc;
  return grow(c, (void**)&c->ann, &c->ann_bytes, (size_t)std::max<int64_t>(nfs_max, 1) * na * 24);
}

struct AnnBufs {
  double* mag;
  double* err;
  int32_t* ns;
  uint32_t* flags;
};

AnnBufs ann_bufs(twk_ctx* c, int64_t n) {
  char* p = c->ann;
  AnnBufs a;
  a.mag = (double*)p;
  a.err = (double*)(p + (size_t)n * 8);
  a.ns = (int32_t*)(p + (size_t)n * 16);
  a.flags = (uint32_t*)(p + (size_t)n * 20);
  return a;
}

int launch_fs(twk_ctx* c, bool mixed, double tol, double* mag, double* err, int32_t* ns,
              uint32_t* flags) {
  if (mixed)
    hipLaunchKernelGGL((k_fs<LDS_CAP, true>), dim3(c->waves), dim3(64), 0, c->stream, c->tasks,
                       &c->cnt[C_NTASK], &c->cnt[C_HEAD], tol, c->scratch, mag, err, ns, flags,
                       c->cnt);
  else
    hipLaunchKernelGGL((k_fs<LDS_CAP, false>), dim3(c->waves), dim3(64), 0, c->stream, c->tasks,
                       &c->cnt[C_NTASK], &c->cnt[C_HEAD], tol, c->scratch, mag, err, ns, flags,
                       c->cnt);
  HIP_TRY(c, hipGetLastError());
  return TWK_OK;
}

int reset(twk_ctx* c, bool queue_only) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->stream, c->cnt, queue_only ? 1 : 0);
  HIP_TRY(c, hipGetLastError());
  return TWK_OK;
}

int mark(twk_ctx* c, int i, bool on) {
  if (c->timing && on) HIP_TRY(c, hipEventRecord(c->ev[i], c->stream));
  return TWK_OK;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

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
  (void)hipFree(c->fs_epoch);
  (void)hipFree(c->ann);
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
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t chunk = std::min<int64_t>(n, CHUNK_TASKS);
  int rc = ensure_fs(c, chunk);
  if (rc) return rc;
  const int all_fs = (mode & TWK_MODE_ALL_FS) ? 1 : 0;
  const bool mixed = (mode & TWK_MODE_MIXED) != 0;
  if ((rc = mark(c, 0, true)) || (rc = reset(c, false))) return rc;
  for (int64_t i0 = 0; i0 < n; i0 += chunk) {
    const int64_t m = std::min(chunk, n - i0);
    if (i0 > 0 && (rc = reset(c, true))) return rc;
    hipLaunchKernelGGL(k_prep, dim3(blocks_for(m)), dim3(256), 0, c->stream, s, q, m, zx + i0,
                       zy + i0, rho, tol, all_fs, c->tasks, c->cnt, mag + i0, err + i0, ns + i0,
                       flags + i0);
    HIP_TRY(c, hipGetLastError());
    if ((rc = mark(c, 1, i0 == 0))) return rc;
    if ((rc = launch_fs(c, mixed, tol, mag + i0, err + i0, ns + i0, flags + i0))) return rc;
    if ((rc = mark(c, 2, i0 == 0))) return rc;
  }
  return mark(c, 3, true);
}

int twk_mag_map(twk_ctx* c, double s, double q, double rho, double xc, double yc, double width,
                double height, int32_t nx, int32_t ny, double tol, uint32_t mode, double* mag,
                double* err, int32_t* ns, uint32_t* flags) {
  if (!c || !finite_pos(s) || !finite_pos(q) || !finite_pos(rho) || !finite_pos(tol) ||
      !finite_pos(width) || !finite_pos(height) || nx < 0 || ny < 0 || !std::isfinite(xc) ||
      !std::isfinite(yc))
    return TWK_EINVAL;
  if (mode & ~(TWK_MODE_MIXED | TWK_MODE_ALL_FS)) return TWK_EINVAL;
  const int64_t n = (int64_t)nx * ny;
  if (n == 0) return TWK_OK;
  if (!mag || !err || !ns || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(ny, CHUNK_TASKS / nx));
  int rc = ensure_fs(c, rows * nx);
  if (rc) return rc;
  const int all_fs = (mode & TWK_MODE_ALL_FS) ? 1 : 0;
  const bool mixed = (mode & TWK_MODE_MIXED) != 0;
  if ((rc = mark(c, 0, true)) || (rc = reset(c, false))) return rc;
  for (int64_t y0 = 0; y0 < ny; y0 += rows) {
    const int64_t nr = std::min<int64_t>(rows, ny - y0);
    if (y0 > 0 && (rc = reset(c, true))) return rc;
    hipLaunchKernelGGL(k_map, dim3(blocks_for(nr * nx)), dim3(256), 0, c->stream, s, q, rho, xc, yc,
                       width, height, nx, ny, y0, nr, tol, all_fs, c->tasks, c->cnt, mag, err, ns,
                       flags);
    HIP_TRY(c, hipGetLastError());
    if ((rc = mark(c, 1, y0 == 0))) return rc;
    if ((rc = launch_fs(c, mixed, tol, mag, err, ns, flags))) return rc;
    if ((rc = mark(c, 2, y0 == 0))) return rc;
  }
  return mark(c, 3, true);
}

int twk_lightcurves(twk_ctx* c, int64_t nsets, const double* s, const double* q, const double* u0,
                    const double* alpha, const double* rho, const double* gamma, int64_t nepochs,
                    const double* tau, int32_t n_annuli, double tol, uint32_t mode, double* mag,
                    double* err, int32_t* ns, uint32_t* flags) {
  if (!c || nsets < 0 || nepochs < 0 || !finite_pos(tol) || n_annuli < 1 || n_annuli > 64)
    return TWK_EINVAL;
  if (mode & ~(TWK_MODE_MIXED | TWK_MODE_ALL_FS)) return TWK_EINVAL;
  if (gamma == nullptr && n_annuli != 1) return TWK_EINVAL;
  const int64_t n = nsets * nepochs;
  if (n == 0) return TWK_OK;
  if (!s || !q || !u0 || !alpha || !rho || !tau || !mag || !err || !ns || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const bool ld = gamma != nullptr;
  const int na = ld ? n_annuli : 1;
  const int64_t chunk_sets = std::max<int64_t>(1, CHUNK_TASKS / na / nepochs);
  const int64_t chunk_n = std::min(nsets, chunk_sets) * nepochs;
  int rc = ensure_fs(c, chunk_n * na);
  if (rc) return rc;
  if (ld && (rc = ensure_ld(c, chunk_n, na))) return rc;
  const AnnBufs ab = ld ? ann_bufs(c, chunk_n * na) : AnnBufs{nullptr, nullptr, nullptr, nullptr};
  const int all_fs = (mode & TWK_MODE_ALL_FS) ? 1 : 0;
  const bool mixed = (mode & TWK_MODE_MIXED) != 0;
  // The limb-darkened value is a weighted difference of the annulus values,
  // which roughly doubles their relative error: annuli run at tol / 2.
  const double tol_fs = ld ? 0.5 * tol : tol;
  if ((rc = mark(c, 0, true)) || (rc = reset(c, false))) return rc;
  for (int64_t k0 = 0; k0 < nsets; k0 += chunk_sets) {
    const int64_t nk = std::min(chunk_sets, nsets - k0);
    const int64_t o = k0 * nepochs;
    if (k0 > 0 && (rc = reset(c, true))) return rc;
    hipLaunchKernelGGL(k_lc, dim3(blocks_for(nk * nepochs)), dim3(256), 0, c->stream, nk, s + k0,
                       q + k0, u0 + k0, alpha + k0, rho + k0, nepochs, tau, tol, all_fs, na,
                       c->tasks, c->cnt, c->fs_epoch, mag + o, err + o, ns + o, flags + o);
    HIP_TRY(c, hipGetLastError());
    if ((rc = mark(c, 1, k0 == 0))) return rc;
    if (ld) rc = launch_fs(c, mixed, tol_fs, ab.mag, ab.err, ab.ns, ab.flags);
    else rc = launch_fs(c, mixed, tol_fs, mag + o, err + o, ns + o, flags + o);
    if (rc) return rc;
    if ((rc = mark(c, 2, k0 == 0))) return rc;
    if (ld) {
      hipLaunchKernelGGL(k_ld, dim3(blocks_for(nk * nepochs)), dim3(256), 0, c->stream, c->cnt,
                         c->fs_epoch, na, gamma + k0, nepochs, ab.mag, ab.err, ab.ns, ab.flags,
                         mag + o, err + o, ns + o, flags + o);
      HIP_TRY(c, hipGetLastError());
    }
  }
  return mark(c, 3, true);
}

int twk_last_stats(twk_ctx* c, int64_t* out8) {
  if (!c || !out8) return TWK_EINVAL;
  long long h[C_NCOUNTERS];
  HIP_TRY(c, hipMemcpyAsync(h, c->cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  out8[0] = h[C_RUNS];
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
