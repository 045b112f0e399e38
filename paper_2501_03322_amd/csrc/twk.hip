// twk.hip -- kernels and C ABI of the MI355X binary-lens magnification library.
//
// Paper: Wang, Wang & Dong, arXiv 2501.03322.  Declarations and argument
// contracts are in include/twk.h.
//
// Pipeline of a finite-source call (all on the caller's stream):
//   k_reset      clear the queue counters (a kernel, not a memset, so that
//                the sequence may be captured in a graph)
//   k_prep/k_lc  one lane per source (k_lc: a run of four consecutive
//                epochs, each centre solve warm-started from the previous
//                one): centre and stencil point solves, point-source
//                adequacy test (Sec. 2.3); adequate sources get the point
//                value, the rest are appended to the task queue with their
//                centre roots (wave-aggregated atomics)
//   k_stride, k_disperse   queue order: the queue taken in a dispersed
//                order (golden-ratio stride over the groups of annuli)
//   mlp::k_infer, k_stride, k_seg, k_place   (learned path instead) inference
//                on the features the point pass wrote, counting the
//                predicted-long contours per tile; those are queued first,
//                each class dispersed
//   k_fs<C, MIXED>  persistent: each 64-lane wave pops tasks from the queue
//                and runs the adaptive contour integration, keeping up to C
//                limb samples (records and sorted arrays) in LDS and
//                continuing in its global slice for larger sources (method
//                cap 4096); MIXED selects FP32 bulk root sweeps and FP32
//                storage of the correction-term inputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/twk.h"
#include "twk_device.h"
#include "twk_fs.h"
#include "twk_mlp.h"
#include "twk_queue.h"

using namespace twk;

namespace {

// Limb samples a source keeps in LDS (sorted arrays and sample records)
// before continuing in global memory: one persistent-kernel instantiation
// per choice; the tuning picks one.
constexpr int LDS_CAPS[3] = {64, 128, 256};

// Counters in device memory (int64 each).
enum {
  C_NTASK = 0,     // tasks queued by the point-source pass
  C_HEAD = 1,      // queue head of the first FS pass
  C_NOVER = 2,     // tasks whose sorted arrays outgrew LDS
  C_NOUT = 3,      // round-by-round dispatch: sources left unfinished by a round
  C_SAMPLES = 4,   // limb samples of finished tasks
  C_SW32 = 5,      // FP32 root sweeps (5 roots each)
  C_SW64 = 6,      // FP64 root sweeps
  C_INTERVALS = 7, // intervals linked
  C_RUNS = 8,      // contour runs
  C_NFS = 9,       // limb-darkened epochs sent to the annulus contours
  C_BUCKET = 16,   // learned path: tasks per budget class (class 1 counted)
  C_DSTRIDE = 24,  // queue dispersal: stride over the groups (0: queue order)
  C_DGROUP = 25,   // queue dispersal: tasks per group
  C_DINV = 26,     // learned path: inverse strides of classes 0 and 1 (26, 27)
  C_NCOUNTERS = 32
};
constexpr int NBUCKET = 2;  // predicted under 256 samples / 256 or more

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
  double gx, gy;  // mu(zeta_c + rho) - mu(zeta_c - rho), same along i rho
  double ghost0;  // three images at the centre: min ghost statistic
  double pair0;   // five images at the centre: min opposite-parity pair statistic
};

// |f''(midpoint)| |z+ - z-|^2 / 4 minimised over opposite-parity real pairs:
// like the ghost statistic, an estimate of the source's distance to the
// fold that created the pair.
__device__ inline double pair_stat(const Lens& L, const Images& im) {
  const int npos = __popc(im.par);
  double best = INFINITY;
  // static indices (the image record stays in registers); a pair (a, b) is
  // positive-negative when a < npos <= b < n
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a + 1; b < 5; ++b) {
      if (!(a < npos && b >= npos && b < im.n)) continue;
      const c64 mid = 0.5 * (im.z[a] + im.z[b]);
      const c64 a1 = mid + L.s;
      const c64 f2 = -2.0 * (L.m1 * cinv(a1 * a1 * a1) + L.m2 * cinv(mid * mid * mid));
      best = fmin(best, 0.25 * cabs64(f2) * cnorm(im.z[a] - im.z[b]));
    }
  return best;
}

// probe: solve the four stencil points (needed by the test and by the
// learned features); test: decide adequacy; feat: the features are wanted
// (without them the stencil stops at the first point that fails the test).
// start: roots to start the centre solve from (a nearby source's), or null
// for a cold start; a warm start that has not converged in 60 sweeps is
// replaced by a cold one.
__device__ inline PsResult point_source_pass(const Lens& L, c64 yc, double rho, double tol,
                                             bool probe, bool test, bool feat,
                                             const c64* start = nullptr) {
  PsResult out;
  c64 c[6], r[5];
  coefficients(L, yc, c);
  bool cold = start == nullptr;
  if (!cold) {
#pragma unroll
    for (int k = 0; k < 5; ++k) r[k] = start[k];
    cold = aberth64(c, r, 60) > 60;
  }
  if (cold) {
    cold_start(c, r);
    aberth64(c, r, 200);
  }
  Images im;
  finish_images(L, yc, r, im);
  out.mu = point_mag(im);
  out.n = im.n;
  out.flags = im.flags;
  out.adequate = false;
  out.ghost0 = INFINITY;
  out.pair0 = INFINITY;
#pragma unroll
  for (int k = 0; k < 5; ++k) out.roots[k] = im.z[k];
  if (!probe) return out;
  bool ok = im.n == 3;
  if (im.n == 3) {
    for (int g = 3; g < 5; ++g) {
      const double gs = ghost_stat(L, yc, im.z[g]);
      out.ghost0 = fmin(out.ghost0, gs);
      if (!(gs > PS_CG * rho)) ok = false;
    }
  } else {
    out.pair0 = pair_stat(L, im);
  }
  double mus = 0.0;
  out.gx = 0.0;
  out.gy = 0.0;
#pragma unroll 1
  for (int k = 0; k < 4 && (ok || feat); ++k) {
    // stencil point k: zeta_c + rho, + i rho, - rho, - i rho
    const double sx = k == 0 ? rho : (k == 2 ? -rho : 0.0);
    const double sy = k == 1 ? rho : (k == 3 ? -rho : 0.0);
    const c64 y = yc + cz(sx, sy);
    coefficients(L, y, c);
#pragma unroll
    for (int j = 0; j < 5; ++j) r[j] = out.roots[j];
    if (aberth64(c, r, 60) > 60) {
      cold_start(c, r);
      aberth64(c, r, 200);
    }
    Images ik;
    finish_images(L, y, r, ik);
    const double mk = point_mag(ik);
    mus += mk;
    const double sg = k < 2 ? 1.0 : -1.0;
    if (k & 1) out.gy += sg * mk;
    else out.gx += sg * mk;
    if (ik.n != 3) ok = false;
    for (int g = 3; g < 5; ++g)
      if (!(ghost_stat(L, y, ik.z[g]) > PS_CG * rho)) ok = false;
  }
  const double dq = 0.5 * (0.25 * mus - out.mu);
  if (!(PS_CQ * fabs(dq) < tol * out.mu)) ok = false;
  out.adequate = test && ok;
  return out;
}

// The eight inputs of the learned budget (centre-of-mass frame):
// s, log10 q, Re zeta, Im zeta, log10 rho, log10 mu_ps, the signed caustic
// proximity +-log10(1 + X / rho) (+ with three images and X the ghost
// statistic, - with five and X the pair statistic), and log10 of
// rho |grad mu_ps| / mu_ps from central differences over the stencil,
// floored at 1e-30.
// rho: the radius of the stencil the point pass used; rho_f: the radius of
// the disk the features describe (the gradient term scales with it).
__device__ inline void ps_features(double s, double q, double zx, double zy, double rho,
                                   double rho_f, const PsResult& ps, float* f) {
  const double grad = 0.5 * sqrt(ps.gx * ps.gx + ps.gy * ps.gy) * (rho_f / rho);
  const double prox = ps.n == 3 ? log10(1.0 + ps.ghost0 / rho_f) : -log10(1.0 + ps.pair0 / rho_f);
  f[0] = (float)s;
  f[1] = (float)log10(q);
  f[2] = (float)zx;
  f[3] = (float)zy;
  f[4] = (float)log10(rho_f);
  f[5] = (float)log10(ps.mu);
  f[6] = (float)prox;
  f[7] = (float)log10(fmax(grad / ps.mu, 1e-30));
}

// Clear all counters (start of a call) or only the queue counters (start of
// a chunk of a call).
__global__ void k_reset(long long* cnt, int queue_only) {
  const int i = threadIdx.x;
  if (i >= C_NCOUNTERS) return;
  if (!queue_only || i == C_NTASK || i == C_HEAD || i == C_NFS || i >= C_BUCKET) cnt[i] = 0;
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

// Coefficients of the quintic (lens-2 frame, c0..c5 as Re, Im) of n source
// positions: the refined form of the method, or (conventional != 0) the
// conventional form the comparator uses.
__global__ __launch_bounds__(256) void k_coef(double s, double q, int64_t n, const double* zx,
                                              const double* zy, int conventional, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Lens L = make_lens(s, q);
  const c64 y = cz(zx[i] - L.z2, zy[i]);
  c64 c[6];
  if (conventional) coefficients_conventional(L, y, c);
  else coefficients(L, y, c);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    out[12 * i + 2 * k] = c[k].x;
    out[12 * i + 2 * k + 1] = c[k].y;
  }
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
// tfeat (learned path): the source's features, one row per task, or per
// limb-darkened epoch f, whose first task slot then goes to tslot[f].
// carry (optional): on entry, with *warm set, the centre roots of a nearby
// source of the same lens to start from; on return the centre roots of this
// source (and *warm says whether there are any).
__device__ inline void emit_source(int64_t out, double s, double q, double zx, double zy,
                                   double rho, double tol, double tol_fs, bool all_fs, int na,
                                   Task* tasks,
                                   long long* cnt, int64_t* fs_epoch, double* mag, double* err,
                                   int32_t* ns, uint32_t* flags, bool active, float* tfeat,
                                   int32_t* tslot = nullptr, c64* carry = nullptr,
                                   bool* warm = nullptr) {
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
      if (warm) *warm = false;
    } else {
      ps = point_source_pass(L, cz(zx - L.z2, zy), rho, tol, !all_fs || tfeat, !all_fs, tfeat,
                             warm && *warm ? carry : nullptr);
      if (carry) {
#pragma unroll
        for (int k = 0; k < 5; ++k) carry[k] = ps.roots[k];
        *warm = true;
      }
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
    t.tol = tol_fs;
#pragma unroll
    for (int k = 0; k < 5; ++k) t.roots[k] = ps.roots[k];
    for (int k = 0; k < na; ++k) {
      t.out = first_out + k;
      t.rho = na > 1 ? rho * sqrt((double)(k + 1) / na) : rho;
      tasks[slot + k] = t;
    }
    if (tfeat) {
      // features of the source (a limb-darkened epoch: of its outer disk,
      // one row per epoch, shared by its annulus contours)
      float f[8];
      ps_features(s, q, zx, zy, rho, rho, ps, f);
      const int64_t row = na > 1 ? first_out / na : slot;
#pragma unroll
      for (int j = 0; j < 8; ++j) tfeat[row * 8 + j] = f[j];
      if (na > 1) tslot[row] = (int32_t)slot;
    }
  }
}

__global__ __launch_bounds__(256) void k_prep(double s, double q, int64_t n, const double* zx,
                                              const double* zy, double rho, double tol,
                                              int all_fs, Task* tasks, long long* cnt,
                                              double* mag, double* err, int32_t* ns,
                                              uint32_t* flags, float* tfeat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < n;
  emit_source(i, s, q, active ? zx[i] : 0.0, active ? zy[i] : 0.0, rho, tol, tol, all_fs != 0, 1, tasks,
              cnt, nullptr, mag, err, ns, flags, active, tfeat);
}

// Per-element lens and source (time-varying lenses: the caller evaluates
// s, q, rho and the source position at each epoch).  An element whose s, q
// or rho is not finite and positive is answered as a non-finite input.
__global__ __launch_bounds__(256) void k_prep_each(const double* ps, const double* pq, int64_t n,
                                                   const double* zx, const double* zy,
                                                   const double* prho, double tol, int all_fs,
                                                   Task* tasks, long long* cnt, double* mag,
                                                   double* err, int32_t* ns, uint32_t* flags,
                                                   float* tfeat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < n;
  double s = 1.0, q = 1.0, rho = 1.0, x = 0.0, y = 0.0;
  if (active) {
    s = ps[i];
    q = pq[i];
    rho = prho[i];
    x = zx[i];
    y = zy[i];
    if (!(s > 0.0 && s < 1e300 && q > 0.0 && q < 1e300 && rho > 0.0 && rho < 1e300)) {
      s = q = rho = 1.0;
      x = __builtin_nan("");
    }
  }
  emit_source(i, s, q, x, y, rho, tol, tol, all_fs != 0, 1, tasks, cnt, nullptr, mag, err, ns, flags,
              active, tfeat);
}

// Magnification map: pixel (ix, iy) of an nx x ny grid over the box
// [xc - w/2, xc + w/2] x [yc - h/2, yc + h/2], pixel centres, output index
// iy * nx + ix (rows iy0 .. iy0 + nrows - 1 in this launch).
__global__ __launch_bounds__(256) void k_map(double s, double q, double rho, double xc, double yc,
                                             double w, double h, int32_t nx, int32_t ny,
                                             int64_t iy0, int64_t nrows, double tol, int all_fs,
                                             Task* tasks, long long* cnt, double* mag,
                                             double* err, int32_t* ns, uint32_t* flags,
                                             float* tfeat) {
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
  emit_source(out, s, q, zx, zy, rho, tol, tol, all_fs != 0, 1, tasks, cnt, nullptr, mag, err, ns,
              flags, active, tfeat);
}

// Light curves: element (set k, epoch j) at index k * nepochs + j.  Source
// centre on the straight trajectory of set k (centre-of-mass frame).  A lane
// takes LC_RUN consecutive epochs of one set; after the first, each centre
// solve starts from the previous epoch's roots (the source has moved by one
// epoch step), which saves most of a cold start's sweeps.
constexpr int LC_RUN = 4;
__host__ __device__ inline int64_t lc_lanes(int64_t nsets, int64_t nep) {
  return nsets * ((nep + LC_RUN - 1) / LC_RUN);
}
// Relative tolerance of each annulus contour of a limb-darkened epoch.  The
// combination is sum_k (I_k - I_{k+1}) x_k mu_k + I_na x_na mu_na over the
// nested disks (x_k = k/na of the squared radius, I_{na+1} = 0).  When the
// intensity falls outward (Gamma >= 0) every weight is non-negative, so the
// combination's relative error is at most the largest relative error of the
// mu_k: the annuli run at the stated tolerance.  For limb brightening
// (Gamma < 0) the weights alternate in sign and the error grows by at most
// 2 I_na / I_1 - 1 (the combination is at least I_1 times the total flux):
// the annuli run at the tolerance divided by that factor.
__device__ inline double annulus_tol(double tol, double G, int na) {
  if (!(G < 0.0)) return tol;
  const double x1 = 1.0 / na, xl = (na - 1.0) / na;
  const double i1 = 1.0 - G + G * (1.0 - pow(1.0 - x1, 1.5)) / x1;
  const double il = 1.0 - G + G * pow(1.0 - xl, 1.5) / (1.0 - xl);
  const double f = 2.0 * il / i1 - 1.0;
  return i1 > 0.0 && f > 1.0 ? tol / f : tol;
}

__global__ __launch_bounds__(256) void k_lc(int64_t nsets, const double* ps, const double* pq,
                                            const double* pu0, const double* pal,
                                            const double* prho, const double* pgam, int64_t nep,
                                            const double* tau, double tol, int all_fs, int na,
                                            Task* tasks, long long* cnt, int64_t* fs_epoch,
                                            double* mag, double* err, int32_t* ns,
                                            uint32_t* flags, float* tfeat, int32_t* tslot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t runs = (nep + LC_RUN - 1) / LC_RUN;
  const bool lane_on = i < nsets * runs;
  const int64_t k = lane_on ? i / runs : 0, j0 = lane_on ? (i - k * runs) * LC_RUN : 0;
  double s = 1.0, q = 1.0, rho = 1.0, u0 = 0.0, sa = 0.0, ca = 1.0, tol_fs = tol;
  if (lane_on) {
    s = ps[k];
    q = pq[k];
    rho = prho[k];
    u0 = pu0[k];
    sincos(pal[k], &sa, &ca);
    if (na > 1) tol_fs = annulus_tol(tol, pgam[k], na);
  }
  c64 carry[5];
  bool warm = false;
  // every lane runs LC_RUN steps: the queue appends are wave-wide
  for (int e = 0; e < LC_RUN; ++e) {
    const int64_t j = j0 + e;
    const bool active = lane_on && j < nep;
    double zx = 0.0, zy = 0.0;
    if (active) {
      const double t = tau[j];
      zx = t * ca - u0 * sa;
      zy = t * sa + u0 * ca;
    }
    emit_source(k * nep + j, s, q, zx, zy, rho, tol, tol_fs, all_fs != 0, na, tasks, cnt, fs_epoch, mag,
                err, ns, flags, active, tfeat, tslot, carry, &warm);
  }
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

// Features of every epoch of a light-curve batch (inputs of the learned
// budget), with the point value and the adequacy decision.
__global__ __launch_bounds__(256) void k_feat(int64_t nsets, const double* ps, const double* pq,
                                              const double* pu0, const double* pal,
                                              const double* prho, int64_t nep,
                                              const double* tau, double tol, float* feat,
                                              double* mu, int32_t* adequate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsets * nep) return;
  const int64_t k = i / nep, j = i - k * nep;
  double sa, ca;
  sincos(pal[k], &sa, &ca);
  const double t = tau[j], u0 = pu0[k];
  const double zx = t * ca - u0 * sa, zy = t * sa + u0 * ca;
  const Lens L = make_lens(ps[k], pq[k]);
  if (!isfinite(zx) || !isfinite(zy)) {
#pragma unroll
    for (int f = 0; f < 8; ++f) feat[i * 8 + f] = __builtin_nanf("");
    mu[i] = __builtin_nan("");
    adequate[i] = 0;
    return;
  }
  const PsResult r = point_source_pass(L, cz(zx - L.z2, zy), prho[k], tol, true, true, true);
  float f[8];
  ps_features(ps[k], pq[k], zx, zy, prho[k], prho[k], r, f);
#pragma unroll
  for (int c = 0; c < 8; ++c) feat[i * 8 + c] = f[c];
  mu[i] = r.mu;
  adequate[i] = r.adequate ? 1 : 0;
}

// Learned budget: a queued task is in class 1 when its predicted log2
// sample count l2 is LONG_L2 or more (256 samples or more), else in class
// 0.  Each class is dispersed (below) and the class-1 rows are spread
// evenly over the first half of the queue, the class-0 rows filling the
// rest (twk_queue.h): a long contour started late would hold its wave after
// the rest of the launch has finished, and long contours started all at
// once slow each other down.  Measured at eight waves per CU: on the
// limb-darkened batch (five launches) as fast as the dispersed order alone
// and 0.8 % faster than queuing class 1 first; on the uniform batch of
// 1024 x 2000 epochs (one launch) 8 % faster than the dispersed order
// alone.  The prediction does not change how a contour is sampled: every
// contour starts from the paper's 64 uniform samples.  The inference
// kernel counts the class-1 tasks into cnt[C_BUCKET + 1].
constexpr float LONG_L2 = 8.0f;
static_assert(NBUCKET == 2, "two budget classes: the inference kernel counts class 1");

// Queue dispersal.  The point pass queues contours in source order, so the
// expensive contours of a caustic crossing (hundreds of consecutive epochs
// of one light curve, ten annuli each) sit together in the queue and run
// at the same time, and so do runs of cheap ones.  The contour kernel
// takes the queue in a dispersed order instead: queue position p runs
// group (p * g) mod N, with N the groups (a limb-darkened epoch's annuli
// stay together), g coprime to N and close to N / phi (golden ratio), so
// any run of consecutive positions samples the whole queue evenly and the
// waves resident at any time hold a representative mix of contours.
// Measured on the limb-darkened batch: the contour kernel 6 % faster than
// in source order (annuli dispersed one by one: 5 %).
// The stride, its inverse and the position map are in twk_queue.h.
// Dispersal strides of a chunk, one thread.  Without the learned order: one
// stride over the queue's groups (k_disperse); with it: the inverse strides
// of the two classes' rows for the placement.
__global__ void k_stride(long long* cnt, int na, int learned) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int grp = na;  // an epoch's annuli stay together
  long long g, gi;
  if (learned) {
    const long long rows = cnt[na > 1 ? C_NFS : C_NTASK], n1 = cnt[C_BUCKET + 1] / na;
    golden_stride((rows - n1) * (na / grp), &g, &gi);
    cnt[C_DINV] = gi;
    golden_stride(n1 * (na / grp), &g, &gi);
    cnt[C_DINV + 1] = gi;
  } else {
    golden_stride(cnt[C_NTASK] / grp, &g, &gi);
    cnt[C_DSTRIDE] = g;
    cnt[C_DGROUP] = grp;
  }
}

// Queue order without the learned classes: order[p] = group (p * g mod N),
// same task within the group.  A fixed grid strides over the queue.
__global__ __launch_bounds__(256) void k_disperse(const long long* cnt, int32_t* order) {
  const long long n = cnt[C_NTASK];
  const unsigned long long g = (unsigned long long)cnt[C_DSTRIDE];
  const long long grp = cnt[C_DGROUP], ng = n / grp;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x)
    order[p] = (int32_t)dispersed_task(p, g, grp, ng);
}

// Placement, one thread per inference row r: a task (na == 1) or a
// limb-darkened epoch, whose na annulus tasks are slot[r] .. slot[r] + na - 1.
// The class ranks are exact prefix counts (per-tile counts from the
// inference kernel, segment sums from k_seg): the long row of rank a takes
// the dispersed rank a * ginv1 mod N1 in class 1, any other row of rank b
// the dispersed rank b * ginv0 mod N0 in class 0, and the two classes are
// merged with class 1 spread over the first half of the queue.
constexpr int PLACE_SEG = 256;  // 32-row tiles per segment of the prefix

// Sum of v over a block of 256 threads (every thread gets it).
__device__ inline long long block_sum256(long long v, long long* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

// Segment sums of the per-tile long-row counts: block b sums tiles
// b*256 .. b*256 + 255.
__global__ __launch_bounds__(256) void k_seg(const long long* cnt, int na, const int32_t* tl,
                                             int32_t* seg) {
  __shared__ long long sh[4];
  const int64_t ntile = (cnt[na > 1 ? C_NFS : C_NTASK] + 31) / 32;
  if ((int64_t)blockIdx.x * PLACE_SEG >= ntile) return;
  const int64_t t = (int64_t)blockIdx.x * PLACE_SEG + threadIdx.x;
  const long long v = block_sum256(t < ntile ? tl[t] : 0, sh);
  if (threadIdx.x == 0) seg[blockIdx.x] = (int32_t)v;
}

__global__ __launch_bounds__(256) void k_place(const long long* cnt, const float* out,
                                               const int32_t* slot, const int32_t* tl,
                                               const int32_t* seg, int na, int32_t* order) {
  __shared__ long long sh[4];
  __shared__ int wsum[4];
  const int64_t n = cnt[na > 1 ? C_NFS : C_NTASK];
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  if (r0 >= n) return;
  const int64_t t0 = r0 / 32, sg = t0 / PLACE_SEG;
  long long acc = 0;
  for (int64_t j = threadIdx.x; j < sg; j += 256) acc += seg[j];
  for (int64_t j = sg * PLACE_SEG + threadIdx.x; j < t0; j += 256) acc += tl[j];
  const long long before = block_sum256(acc, sh);
  const int64_t r = r0 + threadIdx.x;
  const bool on = r < n;
  const bool lng = on && out[2 * r] >= LONG_L2;
  const unsigned long long m = __ballot(lng);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = __popcll(m);
  __syncthreads();
  long long a = before + __popcll(m & ((1ull << lane) - 1ull));
  for (int k = 0; k < w; ++k) a += wsum[k];
  if (on) {
    const long long c1 = cnt[C_BUCKET + 1];               // class-1 tasks
    const long long rank = lng ? a : r - a;                // row rank in its class
    const long long units = lng ? c1 : n * na - c1;        // tasks of the class
    const unsigned long long gi = (unsigned long long)cnt[C_DINV + (lng ? 1 : 0)];
    const int32_t first = na > 1 ? slot[r] : (int32_t)r;
    const long long n1 = c1 / na, n0 = n - n1;  // rows of the two classes
    const long long q = (long long)(((unsigned long long)rank * gi) % (unsigned long long)(units / na));
    const long long pos = (lng ? merged_place_long(q, n0, n1) : merged_place_other(q, n0, n1)) * na;
    for (int k = 0; k < na; ++k) order[pos + k] = first + k;
  }
}

// Persistent finite-source kernel: each wave pops tasks until the queue is
// drained (every wave reaches the exit: the queue length is fixed before
// launch and each pop advances the head).
template <int LCAP, bool MIXED>
#ifndef TWK_FS_WAVES_PER_EU
#define TWK_FS_WAVES_PER_EU 2
#endif
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TWK_FS_WAVES_PER_EU))) void k_fs(
    const Task* tasks, const long long* ntask, long long* head, char* slices,
    double* mag, double* err, int32_t* ns, uint32_t* flags, long long* cnt,
    const int32_t* order) {
  __shared__ FsLds<LCAP, MIXED> lds;
  const int lane = threadIdx.x;
  const WaveMem<MIXED> m = wave_mem<MIXED>(slices, blockIdx.x);
  const long long n = *ntask;
  unsigned long long w_samples = 0, w_sw32 = 0, w_sw64 = 0, w_int = 0, w_runs = 0, w_over = 0;
  // Phase 1 runs sources on their LDS copies until one outgrows it; phase 2
  // then finishes that one in the wave's global slice; repeat.  The two
  // phases are separate loops of one kernel: neither holds the other's
  // registers and no function is called (a call made the compiler spill
  // the round loop's registers to scratch memory).
  bool drained = false;
  // A wave takes its next queue position while the current source runs
  // (the atomic's latency then overlaps the work; measured 0.8 % on the
  // limb-darkened batch).  Every position a wave takes below n is run by
  // it, and a wave leaves when the position it takes is n or beyond.
  long long t_next = 0;
  if (lane == 0) t_next = atomicAdd((unsigned long long*)head, 1ull);
  while (!drained) {
    long long big = -1;  // the source that outgrew its LDS copy, if any
    FsState st;
    for (;;) {
      long long t = __shfl(t_next, 0);
      if (t >= n) {
        drained = true;
        break;
      }
      if (lane == 0) t_next = atomicAdd((unsigned long long*)head, 1ull);
      if (order) t = order[t];
      const Task task = tasks[t];
      st = fs_fresh();
      if (fs_source_lds<LCAP, MIXED>(task, task.tol, m, lds, lane, NNEW, st)) {
        big = t;
        break;
      }
      const FsOut o = fs_output(task, st, false);
      if (lane == 0) {
        mag[task.out] = o.mag;
        err[task.out] = o.err;
        ns[task.out] = o.n;
        flags[task.out] = o.flags;
        w_samples += (unsigned long long)o.n;
        w_sw32 += (unsigned long long)o.sweeps32;
        w_sw64 += (unsigned long long)o.sweeps64;
        w_int += (unsigned long long)o.intervals;
        w_runs += 1ull;
      }
      __syncthreads();
    }
    if (big >= 0) {
      const Task task = tasks[big];
      fs_source_global<MIXED>(task, task.tol, m, (lint*)lds.ivl, lane, st);
      const FsOut o = fs_output(task, st, true);
      if (lane == 0) {
        mag[task.out] = o.mag;
        err[task.out] = o.err;
        ns[task.out] = o.n;
        flags[task.out] = o.flags;
        w_samples += (unsigned long long)o.n;
        w_sw32 += (unsigned long long)o.sweeps32;
        w_sw64 += (unsigned long long)o.sweeps64;
        w_int += (unsigned long long)o.intervals;
        w_runs += 1ull;
        w_over += 1ull;
      }
      __syncthreads();
    }
  }
  // work counters: one flush per wave, not per source (the counters share a
  // cache line that every wave would otherwise hit once per source)
  if (lane == 0 && w_runs > 0) {
    atomicAdd((unsigned long long*)&cnt[C_SAMPLES], w_samples);
    atomicAdd((unsigned long long*)&cnt[C_SW32], w_sw32);
    atomicAdd((unsigned long long*)&cnt[C_SW64], w_sw64);
    atomicAdd((unsigned long long*)&cnt[C_INTERVALS], w_int);
    atomicAdd((unsigned long long*)&cnt[C_RUNS], w_runs);
    if (w_over) atomicAdd((unsigned long long*)&cnt[C_NOVER], w_over);
  }
}

// Round-by-round dispatch (the paper's, Secs. 3, 4.1): one launch per
// refinement round over the list of unfinished sources of a batch, one
// wave per source.  list_in == null: the batch's first round (every source
// b = block index starts); otherwise the sources listed.  A source that is
// not finished is appended to list_out (count in *n_out).  Sources b of the
// batch are tasks b0 + b (in the learned queue order when order is given);
// each has its global slice b and its state rs[b].
template <bool MIXED, bool CONV>
__global__ __launch_bounds__(64) void k_fs_round(const Task* tasks, int64_t b0,
                                                 const int32_t* order, const int32_t* list_in,
                                                 int32_t* list_out,
                                                 long long* n_out, RoundState* rs, char* slices,
                                                 double* mag, double* err, int32_t* ns,
                                                 uint32_t* flags) {
  __shared__ int ivl[NNEW];
  const int lane = threadIdx.x;
  const bool fresh = list_in == nullptr;
  const int b = fresh ? (int)blockIdx.x : list_in[blockIdx.x];
  int64_t t = b0 + b;
  if (order) t = order[t];
  const Task task = tasks[t];
  const WaveMem<MIXED> m = wave_mem<MIXED>(slices, b);
  FsOut o;
  if (fs_round_step<MIXED, CONV>(task, task.tol, m, (lint*)ivl, lane, NNEW, &rs[b], fresh, &o)) {
    if (lane == 0) {
      mag[task.out] = o.mag;
      err[task.out] = o.err;
      ns[task.out] = o.n;
      flags[task.out] = o.flags;
    }
  } else if (lane == 0) {
    list_out[atomicAdd((unsigned long long*)n_out, 1ull)] = b;
  }
}

// Work counters of a finished batch of the round-by-round dispatch: block
// sums of the sources' totals, one atomic per counter and block.
__global__ __launch_bounds__(256) void k_round_stats(const RoundState* rs, int64_t nb,
                                                     long long* cnt) {
  __shared__ double part[4][256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < nb) {
    v[0] = rs[i].N;
    v[1] = rs[i].sw32;
    v[2] = rs[i].sw64;
    v[3] = rs[i].nint;
  }
  for (int k = 0; k < 4; ++k) part[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 4; ++k) part[k][threadIdx.x] += part[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t runs = std::min<int64_t>(256, nb - (int64_t)blockIdx.x * 256);
    atomicAdd((unsigned long long*)&cnt[C_SAMPLES], (unsigned long long)part[0][0]);
    atomicAdd((unsigned long long*)&cnt[C_SW32], (unsigned long long)part[1][0]);
    atomicAdd((unsigned long long*)&cnt[C_SW64], (unsigned long long)part[2][0]);
    atomicAdd((unsigned long long*)&cnt[C_INTERVALS], (unsigned long long)part[3][0]);
    atomicAdd((unsigned long long*)&cnt[C_RUNS], (unsigned long long)runs);
  }
}

__global__ void k_zero_counter(long long* p) {
  if (threadIdx.x == 0) *p = 0;
}

// Scratch of twk_finite_mag_noalloc, which allocates nothing: counters,
// the queue order and task queue of at most NOALLOC_MAX_N sources, and the
// global slices of at most NOALLOC_WAVES persistent waves (130 MB).  Each
// device the library runs on holds its own copy until the process ends.
constexpr int64_t NOALLOC_MAX_N = 65536;
constexpr int NOALLOC_WAVES = 128;
constexpr size_t NOALLOC_ORDER_OFF = 256;
constexpr size_t NOALLOC_TASK_OFF = NOALLOC_ORDER_OFF + (size_t)NOALLOC_MAX_N * sizeof(int32_t);
constexpr size_t NOALLOC_SLICE_OFF = NOALLOC_TASK_OFF + (size_t)NOALLOC_MAX_N * sizeof(Task);
constexpr size_t NOALLOC_BYTES =
    NOALLOC_SLICE_OFF + (size_t)NOALLOC_WAVES * METHOD_CAP * kSlotBytesMax;
static_assert(C_NCOUNTERS * sizeof(long long) <= NOALLOC_ORDER_OFF, "counters fit");
static_assert(NOALLOC_TASK_OFF % 256 == 0, "tasks aligned");
static_assert(NOALLOC_SLICE_OFF % 256 == 0, "slices aligned");

}  // namespace

static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
// This device's address of `scratch` (host code must not pass the array's
// name to a kernel: that is a host-side stand-in).  Looked up once per
// device, with the device current, by the first context created on it.
std::mutex g_noalloc_mu;
char* g_noalloc[64] = {};

int noalloc_address(int device, char** out) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (device < 0 || device >= 64) return TWK_EDEVICE;
  if (!g_noalloc[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return TWK_EDEVICE;
    }
    g_noalloc[device] = (char*)p;
  }
  *out = g_noalloc[device];
  return TWK_OK;
}
}  // namespace

// ------------------------------------------------------------------ host
struct twk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  int last_err = 0;
  char* slices = nullptr;  // the persistent waves' global slices
  size_t slices_bytes = 0;
  char* noalloc = nullptr;  // this device's address of the file-scope scratch array
  Task* tasks = nullptr;
  int64_t task_cap = 0;
  int32_t* qorder = nullptr;  // dispersed queue order (paths without the learned order)
  size_t qorder_bytes = 0;
  long long* cnt = nullptr;
  int waves = 0;
  // limb darkening: epochs sent to the annulus contours and their results
  int64_t* fs_epoch = nullptr;
  size_t fs_epoch_bytes = 0;
  char* ann = nullptr;  // [mag f64 | err f64 | ns i32 | flags u32] x (nfs * na)
  size_t ann_bytes = 0;
  bool timing = false;
  // per-stage timing: ev[0] and ev[1] bracket the call; chunk k of the call
  // has ev[2 + 4k + j], j = before the point pass, after it, after the
  // learned stage, after the contour kernel
  std::vector<hipEvent_t> ev;
  int64_t ev_chunks = 0;   // chunks whose stages the last timed call marked
  int64_t last_chunks = 0; // contour-kernel launches of the last call
  // launch tuning of the contour stage, and graph replay
  twk_tuning tune{0, 128, 1.0f, 0};
  int occ[3][2] = {{0, 0}, {0, 0}, {0, 0}};  // resident waves per CU [LDS cap][fp64, mixed]
  bool capturing = false;  // no event marks inside a capture
  // captured launch sequences (replayed when a call repeats)
  struct Graph {
    uint64_t key[24];
    hipGraphExec_t exec;
  } graphs[4];
  int n_graphs = 0, graph_next = 0;
  // learned budget
  float* mlp_p = nullptr;           // float32 master parameters
  mlp::bf16x8* mlp_frag = nullptr;  // packed inference operands
  bool mlp_ready = false;
  char* lt = nullptr;               // per task: features, outputs, queue order
  size_t lt_bytes = 0;
  int64_t lt_cap = 0;
  // round-by-round dispatch: per-source global slices, states and the two
  // lists of unfinished sources of a batch
  char* rslices = nullptr;
  size_t rslices_bytes = 0;
  char* rstate = nullptr;
  size_t rstate_bytes = 0;
  int32_t* rlist = nullptr;
  size_t rlist_bytes = 0;
  // training
  char* tr = nullptr;
  size_t tr_bytes = 0;
  float* opt = nullptr;             // gradient, first and second moments
  int32_t* perm = nullptr;
  size_t perm_bytes = 0;
  double* dsum = nullptr;           // per-step losses of an epoch
  size_t dsum_bytes = 0;
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

void drop_graphs(twk_ctx* c) {
  for (int i = 0; i < c->n_graphs; ++i) (void)hipGraphExecDestroy(c->graphs[i].exec);
  c->n_graphs = 0;
  c->graph_next = 0;
}

// Grow a context buffer.  Captured launch sequences hold buffer addresses,
// so any reallocation drops them.
int grow(twk_ctx* c, void** p, size_t* have, size_t need) {
  if (*have >= need) return TWK_OK;
  drop_graphs(c);
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

// Resident contour waves per CU of the FP64 and the mixed kernel for an LDS
// capacity (the mixed kernel's smaller records allow more).
template <int LCAP>
hipError_t occupancy(int* fp64, int* mixed) {
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(fp64, k_fs<LCAP, false>, 64, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(mixed, k_fs<LCAP, true>, 64, 0);
  return e;
}

int occupancy_of(int lds_cap, int* fp64, int* mixed) {
  hipError_t e;
  switch (lds_cap) {
    case 64: e = occupancy<64>(fp64, mixed); break;
    case 256: e = occupancy<256>(fp64, mixed); break;
    default: e = occupancy<128>(fp64, mixed); break;
  }
  return e == hipSuccess ? TWK_OK : TWK_EDEVICE;
}

// Waves per CU a tuning may ask for at an LDS capacity: the larger of the
// two kernels' limits (a launch of the other kernel is clamped to its own).
int max_waves(int lds_cap, int* out) {
  int a = 0, b = 0;
  const int rc = occupancy_of(lds_cap, &a, &b);
  *out = std::max(a, b);
  return rc;
}

int cap_index(int lds_cap) {
  for (int i = 0; i < 3; ++i)
    if (LDS_CAPS[i] == lds_cap) return i;
  return -1;
}

int fs_waves(const twk_ctx* c) { return c->tune.waves_per_cu * c->n_cu; }

// Task records per chunk of a call: bounds the queue memory (136 B and a
// 4 B queue position each, 38 GB at most; the learned path adds 48 B and
// limb darkening 24 B per task).  Fewer, larger chunks pay fewer launch
// tails and per-chunk stages: on the limb-darkened batch (1.2e8 contours)
// chunks of 2^28 tasks run 1.1 % faster than chunks of 2^26.
constexpr int64_t CHUNK_TASKS = (int64_t)1 << 28;

int ensure_fs(twk_ctx* c, int64_t ntask_max) {
  int rc;
  size_t have = (size_t)c->task_cap * sizeof(Task);
  if ((rc = grow(c, (void**)&c->tasks, &have, (size_t)std::max<int64_t>(ntask_max, 1) * sizeof(Task))))
    return rc;
  c->task_cap = (int64_t)(have / sizeof(Task));
  if ((rc = grow(c, (void**)&c->qorder, &c->qorder_bytes,
                 (size_t)std::max<int64_t>(ntask_max, 1) * sizeof(int32_t))))
    return rc;
  c->waves = fs_waves(c);
  const size_t need = (size_t)c->waves * METHOD_CAP * kSlotBytesMax;
  return grow(c, (void**)&c->slices, &c->slices_bytes, need);
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

// Per-task buffers of the learned path, carved from one allocation (48
// bytes per task and the prefix counts).  Inference rows are tasks, or limb-darkened epochs
// (then fewer than the tasks).
struct LearnBufs {
  float* feat;    // [cap x 8] features per row
  float* out;     // [cap x 2] predictions per row
  int32_t* order; // [cap] queue order of the tasks
  int32_t* slot;  // [cap] first task of each limb-darkened epoch's row
  int32_t* tl;    // [cap / 32 + 1] long rows per 32-row tile
  int32_t* seg;   // [cap / 8192 + 1] long rows per segment of 256 tiles
};

LearnBufs learn_bufs(twk_ctx* c) {
  LearnBufs b;
  b.feat = (float*)c->lt;
  b.out = b.feat + 8 * c->lt_cap;
  b.order = (int32_t*)(b.out + 2 * c->lt_cap);
  b.slot = b.order + c->lt_cap;
  b.tl = b.slot + c->lt_cap;
  b.seg = b.tl + c->lt_cap / 32 + 1;
  return b;
}

int ensure_learn(twk_ctx* c, int64_t ntask_max) {
  const int64_t cap = std::max<int64_t>(ntask_max, 1);
  if (c->lt_cap >= cap) return TWK_OK;
  int rc = grow(c, (void**)&c->lt, &c->lt_bytes,
                (size_t)cap * 48 + (size_t)(cap / 32 + cap / (32 * PLACE_SEG) + 2) * 4);
  if (rc) return rc;
  c->lt_cap = cap;
  return TWK_OK;
}

// Learned stage between the point-source pass and the contour kernel:
// predict every queued row's sample count, counting the predicted-long
// tasks (per tile and in total) as the predictions are written; then the
// classes' dispersal strides, the segment sums of the tile counts, and the
// placement of every row (the contours themselves are unchanged).  Grids
// cover the chunk's row capacity; blocks beyond the device-side row count
// return at once.
int learned_stage(twk_ctx* c, int64_t ntask_max, int na) {
  const LearnBufs b = learn_bufs(c);
  hipLaunchKernelGGL(mlp::k_infer, dim3(c->n_cu), dim3(64 * mlp::INFER_WAVES), 0, c->stream,
                     c->mlp_p, c->mlp_frag, (int64_t)0, &c->cnt[na > 1 ? C_NFS : C_NTASK], b.feat,
                     b.out, &c->cnt[C_BUCKET + 1], LONG_L2, na, b.tl);
  HIP_TRY(c, hipGetLastError());
  hipLaunchKernelGGL(k_stride, dim3(1), dim3(64), 0, c->stream, c->cnt, na, 1);
  HIP_TRY(c, hipGetLastError());
  const int64_t rows_max = (ntask_max + na - 1) / na;
  const int64_t tiles_max = (rows_max + 31) / 32;
  hipLaunchKernelGGL(k_seg, dim3((unsigned)((tiles_max + PLACE_SEG - 1) / PLACE_SEG)), dim3(256), 0,
                     c->stream, c->cnt, na, b.tl, b.seg);
  HIP_TRY(c, hipGetLastError());
  hipLaunchKernelGGL(k_place, dim3((unsigned)((rows_max + 255) / 256)), dim3(256), 0, c->stream,
                     c->cnt, b.out, b.slot, b.tl, b.seg, na, b.order);
  HIP_TRY(c, hipGetLastError());
  return TWK_OK;
}

template <int LCAP>
void launch_fs_cap(twk_ctx* c, bool mixed, double* mag, double* err, int32_t* ns,
                   uint32_t* flags, const int32_t* order) {
  // the persistent grid: the tuned waves per CU, at most what the launched
  // kernel can keep resident
  const int ci = cap_index(LCAP);
  const int waves = std::min(c->waves, c->occ[ci][mixed ? 1 : 0] * c->n_cu);
  if (mixed)
    hipLaunchKernelGGL((k_fs<LCAP, true>), dim3(waves), dim3(64), 0, c->stream, c->tasks,
                       &c->cnt[C_NTASK], &c->cnt[C_HEAD], c->slices, mag, err, ns, flags,
                       c->cnt, order);
  else
    hipLaunchKernelGGL((k_fs<LCAP, false>), dim3(waves), dim3(64), 0, c->stream, c->tasks,
                       &c->cnt[C_NTASK], &c->cnt[C_HEAD], c->slices, mag, err, ns, flags,
                       c->cnt, order);
}

int launch_fs(twk_ctx* c, bool mixed, const int32_t* order, double* mag, double* err,
              int32_t* ns, uint32_t* flags) {
  switch (c->tune.lds_cap) {
    case 64: launch_fs_cap<64>(c, mixed, mag, err, ns, flags, order); break;
    case 256: launch_fs_cap<256>(c, mixed, mag, err, ns, flags, order); break;
    default: launch_fs_cap<128>(c, mixed, mag, err, ns, flags, order); break;
  }
  HIP_TRY(c, hipGetLastError());
  return TWK_OK;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Sources per batch of the round-by-round dispatch: each holds a global
// slice for the method's 4096 samples (0.94 MB), so a batch takes 31 GB.
constexpr int64_t ROUND_BATCH = 32768;

// The paper's dispatch: the host reads the number of queued tasks, then
// for each batch of sources launches one round after another over the list
// of unfinished ones, reading the list's length after each round.
int rounds_stage(twk_ctx* c, bool mixed, bool learned, bool conv, double* mag, double* err,
                 int32_t* ns, uint32_t* flags) {
  long long ntask = 0, nout = 0;
  HIP_TRY(c, hipMemcpyAsync(&ntask, &c->cnt[C_NTASK], 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (ntask <= 0) return TWK_OK;
  const int64_t B = std::min<int64_t>(ntask, ROUND_BATCH);
  int rc;
  if ((rc = grow(c, (void**)&c->rslices, &c->rslices_bytes,
                 (size_t)B * METHOD_CAP * kSlotBytesMax)) ||
      (rc = grow(c, (void**)&c->rstate, &c->rstate_bytes, (size_t)B * sizeof(RoundState))) ||
      (rc = grow(c, (void**)&c->rlist, &c->rlist_bytes, (size_t)2 * B * sizeof(int32_t))))
    return rc;
  const int32_t* order = learned ? learn_bufs(c).order : nullptr;
  RoundState* rs = (RoundState*)c->rstate;
  for (int64_t b0 = 0; b0 < ntask; b0 += B) {
    const int64_t nb = std::min<int64_t>(B, ntask - b0);
    const int32_t* lin = nullptr;
    int32_t* lout = c->rlist;
    int64_t nin = nb;
    while (nin > 0) {
      hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, c->stream, &c->cnt[C_NOUT]);
      if (conv)
        hipLaunchKernelGGL((k_fs_round<false, true>), dim3((unsigned)nin), dim3(64), 0, c->stream,
                           c->tasks, b0, order, lin, lout, &c->cnt[C_NOUT], rs, c->rslices, mag, err,
                           ns, flags);
      else if (mixed)
        hipLaunchKernelGGL((k_fs_round<true, false>), dim3((unsigned)nin), dim3(64), 0, c->stream,
                           c->tasks, b0, order, lin, lout, &c->cnt[C_NOUT], rs, c->rslices, mag, err,
                           ns, flags);
      else
        hipLaunchKernelGGL((k_fs_round<false, false>), dim3((unsigned)nin), dim3(64), 0, c->stream,
                           c->tasks, b0, order, lin, lout, &c->cnt[C_NOUT], rs, c->rslices, mag, err,
                           ns, flags);
      HIP_TRY(c, hipGetLastError());
      HIP_TRY(c, hipMemcpyAsync(&nout, &c->cnt[C_NOUT], 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      nin = nout;
      lin = lout;
      lout = lout == c->rlist ? c->rlist + B : c->rlist;
    }
    hipLaunchKernelGGL(k_round_stats, dim3(blocks_for(nb)), dim3(256), 0, c->stream, rs, nb,
                       c->cnt);
    HIP_TRY(c, hipGetLastError());
  }
  return TWK_OK;
}

int reset(twk_ctx* c, bool queue_only) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->stream, c->cnt, queue_only ? 1 : 0);
  HIP_TRY(c, hipGetLastError());
  return TWK_OK;
}

// Event j of chunk k (j = 0: before the point pass, 1: after it, 2: after
// the learned stage, 3: after the contour kernel).
int mark(twk_ctx* c, int64_t k, int j) {
  if (c->timing && !c->capturing && k < c->ev_chunks)
    HIP_TRY(c, hipEventRecord(c->ev[2 + 4 * k + j], c->stream));
  return TWK_OK;
}

int mark_call(twk_ctx* c, int j) {
  if (c->timing && !c->capturing) HIP_TRY(c, hipEventRecord(c->ev[j], c->stream));
  return TWK_OK;
}

// Before issuing a call of `chunks` chunks: events for every stage of every
// chunk (created here, outside any capture).
int prepare_call(twk_ctx* c, int64_t chunks) {
  c->last_chunks = chunks;
  if (!c->timing) return TWK_OK;
  const size_t need = 2 + 4 * (size_t)chunks;
  while (c->ev.size() < need) {
    hipEvent_t e = nullptr;
    HIP_TRY(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
  c->ev_chunks = chunks;
  return TWK_OK;
}

bool finite_pos(double v) { return v > 0.0 && v < 1e300; }

// Largest accepted element count of a batch call (sets x epochs x annuli):
// far beyond any device memory, and it keeps every size product in range.
constexpr int64_t MAX_ELEMS = (int64_t)1 << 48;
// Elements of one launch of a one-lane-per-element kernel: the dispatch's
// work-item count must stay below 2^32.
constexpr int64_t LAUNCH_MAX = (int64_t)1 << 30;
bool batch_size_ok(int64_t nsets, int64_t nepochs, int64_t na) {
  return nsets >= 0 && nepochs >= 0 && nepochs <= LAUNCH_MAX &&
         (nepochs == 0 || nsets <= MAX_ELEMS / nepochs) && nsets * nepochs <= MAX_ELEMS / na;
}

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
  int wpc = 0;
  for (int i = 0; i < 3; ++i) {
    if (occupancy_of(LDS_CAPS[i], &c->occ[i][0], &c->occ[i][1]) != TWK_OK ||
        c->occ[i][0] < 1 || c->occ[i][1] < 1) {
      delete c;
      return TWK_EDEVICE;
    }
  }
  if (max_waves(128, &wpc) != TWK_OK || wpc < 1) {
    delete c;
    return TWK_EDEVICE;
  }
  c->tune.waves_per_cu = wpc;
  c->waves = fs_waves(c);
  if (hipMalloc((void**)&c->cnt, C_NCOUNTERS * sizeof(long long)) != hipSuccess) {
    delete c;
    return TWK_ENOMEM;
  }
  if (noalloc_address(device, &c->noalloc) != TWK_OK) {
    (void)hipFree(c->cnt);
    delete c;
    return TWK_EDEVICE;
  }
  *out = c;
  return TWK_OK;
}

int twk_destroy(twk_ctx* c) {
  if (!c) return TWK_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->slices);
  (void)hipFree(c->tasks);
  (void)hipFree(c->qorder);
  (void)hipFree(c->cnt);
  (void)hipFree(c->fs_epoch);
  (void)hipFree(c->ann);
  (void)hipFree(c->rslices);
  (void)hipFree(c->rstate);
  (void)hipFree(c->rlist);
  drop_graphs(c);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  (void)hipFree(c->mlp_p);
  (void)hipFree(c->mlp_frag);
  (void)hipFree(c->lt);
  (void)hipFree(c->tr);
  (void)hipFree(c->opt);
  (void)hipFree(c->perm);
  (void)hipFree(c->dsum);
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
  if (!c || !finite_pos(s) || !finite_pos(q) || n < 0 || n > MAX_ELEMS) return TWK_EINVAL;
  if (n == 0) return TWK_OK;
  if (!zx || !zy || !mag || !nimg || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  for (int64_t i0 = 0; i0 < n; i0 += LAUNCH_MAX) {
    const int64_t m = std::min(LAUNCH_MAX, n - i0);
    hipLaunchKernelGGL(k_point, dim3(blocks_for(m)), dim3(256), 0, c->stream, s, q, m, zx + i0,
                       zy + i0, mag + i0, nimg + i0, flags + i0);
    HIP_TRY(c, hipGetLastError());
  }
  return TWK_OK;
}

int twk_coefficients(twk_ctx* c, double s, double q, int64_t n, const double* zx, const double* zy,
                     int32_t form, double* c12) {
  if (!c || !finite_pos(s) || !finite_pos(q) || n < 0 || n > MAX_ELEMS ||
      (form != TWK_COEF_REFINED && form != TWK_COEF_CONVENTIONAL))
    return TWK_EINVAL;
  if (n == 0) return TWK_OK;
  if (!zx || !zy || !c12) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  for (int64_t i0 = 0; i0 < n; i0 += LAUNCH_MAX) {
    const int64_t m = std::min(LAUNCH_MAX, n - i0);
    hipLaunchKernelGGL(k_coef, dim3(blocks_for(m)), dim3(256), 0, c->stream, s, q, m, zx + i0,
                       zy + i0, form == TWK_COEF_CONVENTIONAL ? 1 : 0, c12 + 12 * i0);
    HIP_TRY(c, hipGetLastError());
  }
  return TWK_OK;
}

}  // extern "C"

namespace {

constexpr uint32_t KNOWN_MODES =
    TWK_MODE_MIXED | TWK_MODE_MLP | TWK_MODE_ALL_FS | TWK_MODE_ROUNDS | TWK_MODE_CONVENTIONAL;

// Identity of a call for graph replay: entry point (ORed with ROUNDS_KEY
// for the round-by-round dispatch), scalar arguments (as bits), device
// pointers and tuning.
constexpr uint64_t ROUNDS_KEY = 1ull << 32;
struct CallKey {
  uint64_t w[24] = {};
  int n = 0;
  CallKey& u(uint64_t v) {
    w[n++] = v;
    return *this;
  }
  CallKey& d(double v) {
    uint64_t b;
    std::memcpy(&b, &v, 8);
    return u(b);
  }
  CallKey& p(const void* v) { return u((uint64_t)(uintptr_t)v); }
};

CallKey& tuning_key(CallKey& k, const twk_ctx* c) {
  uint32_t sh;
  std::memcpy(&sh, &c->tune.budget_shift, 4);
  return k.u((uint64_t)c->tune.waves_per_cu | ((uint64_t)c->tune.lds_cap << 20) |
             ((uint64_t)sh << 32));
}

// Issue the launch sequence of a call, or, with graph replay on, replay
// the captured sequence of an identical earlier call (capturing it the
// first time).  Nothing inside `issue` may allocate or synchronise.
// With timing on, a replayed call is timed as a whole (the stage times
// read 0, the rest of the call is the whole call).
int launch_graph(twk_ctx* c, hipGraphExec_t ex) {
  c->ev_chunks = 0;
  if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
  HIP_TRY(c, hipGraphLaunch(ex, c->stream));
  if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
  return TWK_OK;
}

template <class F>
int run_captured(twk_ctx* c, const CallKey& key, F&& issue) {
  // the round-by-round dispatch reads counts on the host between launches
  // and cannot be captured
  if (!c->tune.graphs || (key.w[0] & ROUNDS_KEY)) return issue();
  for (int i = 0; i < c->n_graphs; ++i)
    if (std::memcmp(c->graphs[i].key, key.w, sizeof(key.w)) == 0)
      return launch_graph(c, c->graphs[i].exec);
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  const int rc = issue();
  c->capturing = false;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : hip_fail(c, e);
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return hip_fail(c, ei);
  int slot;
  if (c->n_graphs < 4) {
    slot = c->n_graphs++;
  } else {
    slot = c->graph_next;
    c->graph_next = (c->graph_next + 1) % 4;
    (void)hipGraphExecDestroy(c->graphs[slot].exec);
  }
  std::memcpy(c->graphs[slot].key, key.w, sizeof(key.w));
  c->graphs[slot].exec = ex;
  return launch_graph(c, ex);
}

// Mode bits: unknown bits are rejected; the learned budget needs weights.
int check_mode(twk_ctx* c, uint32_t mode) {
  if (mode & ~KNOWN_MODES) return TWK_EINVAL;
  if ((mode & TWK_MODE_CONVENTIONAL) && (mode & (TWK_MODE_MIXED | TWK_MODE_MLP))) return TWK_EINVAL;
  if ((mode & TWK_MODE_MLP) && !c->mlp_ready) return TWK_ENOMLP;
  return TWK_OK;
}

// After the point-source pass of chunk k: learned stage (if any), then the
// contour kernel, each bracketed by the chunk's stage events.
int contour_stage(twk_ctx* c, int64_t k, uint32_t mode, int64_t ntask_max, int na, double* mag,
                  double* err, int32_t* ns, uint32_t* flags) {
  int rc;
  const bool mixed = (mode & TWK_MODE_MIXED) != 0, learned = (mode & TWK_MODE_MLP) != 0;
  if ((rc = mark(c, k, 1))) return rc;
  if (learned && (rc = learned_stage(c, ntask_max, na))) return rc;
  if ((rc = mark(c, k, 2))) return rc;
  if (mode & (TWK_MODE_ROUNDS | TWK_MODE_CONVENTIONAL)) {
    rc = rounds_stage(c, mixed, learned, (mode & TWK_MODE_CONVENTIONAL) != 0, mag, err, ns, flags);
  } else {
    if (!learned) {
      hipLaunchKernelGGL(k_stride, dim3(1), dim3(64), 0, c->stream, c->cnt, na, 0);
      HIP_TRY(c, hipGetLastError());
      hipLaunchKernelGGL(k_disperse, dim3(8 * c->n_cu), dim3(256), 0, c->stream, c->cnt, c->qorder);
      HIP_TRY(c, hipGetLastError());
    }
    rc = launch_fs(c, mixed, learned ? learn_bufs(c).order : c->qorder, mag, err, ns, flags);
  }
  if (rc) return rc;
  return mark(c, k, 3);
}

uint64_t entry_key(int id, uint32_t mode) {
  return (uint64_t)id | ((mode & (TWK_MODE_ROUNDS | TWK_MODE_CONVENTIONAL)) ? ROUNDS_KEY : 0ull);
}

// Every source by contour (the point-source test skipped)?
int all_fs_of(uint32_t mode) { return (mode & (TWK_MODE_ALL_FS | TWK_MODE_CONVENTIONAL)) ? 1 : 0; }

}  // namespace

extern "C" {

int twk_finite_mag(twk_ctx* c, double s, double q, int64_t n, const double* zx, const double* zy,
                   double rho, double tol, uint32_t mode, double* mag, double* err, int32_t* ns,
                   uint32_t* flags) {
  if (!c || !finite_pos(s) || !finite_pos(q) || !finite_pos(rho) || !finite_pos(tol) || n < 0 ||
      n > MAX_ELEMS)
    return TWK_EINVAL;
  int rc = check_mode(c, mode);
  if (rc) return rc;
  if (n == 0) return TWK_OK;
  if (!zx || !zy || !mag || !err || !ns || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t chunk = std::min<int64_t>(n, CHUNK_TASKS);
  const bool learned = (mode & TWK_MODE_MLP) != 0;
  if ((rc = ensure_fs(c, chunk))) return rc;
  if (learned && (rc = ensure_learn(c, chunk))) return rc;
  const int all_fs = all_fs_of(mode);
  float* tfeat = learned ? learn_bufs(c).feat : nullptr;
  CallKey key;
  key.u(entry_key(1, mode)).d(s).d(q).u((uint64_t)n).p(zx).p(zy).d(rho).d(tol).u(mode).p(mag).p(err).p(ns).p(flags);
  if ((rc = prepare_call(c, (n + chunk - 1) / chunk))) return rc;
  return run_captured(c, tuning_key(key, c), [&]() -> int {
    int r;
    if ((r = mark_call(c, 0)) || (r = reset(c, false))) return r;
    for (int64_t i0 = 0; i0 < n; i0 += chunk) {
      const int64_t m = std::min(chunk, n - i0);
      if (i0 > 0 && (r = reset(c, true))) return r;
      if ((r = mark(c, i0 / chunk, 0))) return r;
      hipLaunchKernelGGL(k_prep, dim3(blocks_for(m)), dim3(256), 0, c->stream, s, q, m, zx + i0,
                         zy + i0, rho, tol, all_fs, c->tasks, c->cnt, mag + i0, err + i0, ns + i0,
                         flags + i0, tfeat);
      HIP_TRY(c, hipGetLastError());
      if ((r = contour_stage(c, i0 / chunk, mode, m, 1, mag + i0, err + i0, ns + i0, flags + i0)))
        return r;
    }
    return mark_call(c, 1);
  });
}

int twk_finite_mag_each(twk_ctx* c, int64_t n, const double* s, const double* q,
                        const double* zx, const double* zy, const double* rho, double tol,
                        uint32_t mode, double* mag, double* err, int32_t* ns, uint32_t* flags) {
  if (!c || !finite_pos(tol) || n < 0 || n > MAX_ELEMS) return TWK_EINVAL;
  int rc = check_mode(c, mode);
  if (rc) return rc;
  if (n == 0) return TWK_OK;
  if (!s || !q || !zx || !zy || !rho || !mag || !err || !ns || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t chunk = std::min<int64_t>(n, CHUNK_TASKS);
  const bool learned = (mode & TWK_MODE_MLP) != 0;
  if ((rc = ensure_fs(c, chunk))) return rc;
  if (learned && (rc = ensure_learn(c, chunk))) return rc;
  const int all_fs = all_fs_of(mode);
  float* tfeat = learned ? learn_bufs(c).feat : nullptr;
  CallKey key;
  key.u(entry_key(4, mode)).u((uint64_t)n).p(s).p(q).p(zx).p(zy).p(rho).d(tol).u(mode).p(mag).p(err).p(ns).p(flags);
  if ((rc = prepare_call(c, (n + chunk - 1) / chunk))) return rc;
  return run_captured(c, tuning_key(key, c), [&]() -> int {
    int r;
    if ((r = mark_call(c, 0)) || (r = reset(c, false))) return r;
    for (int64_t i0 = 0; i0 < n; i0 += chunk) {
      const int64_t m = std::min(chunk, n - i0);
      if (i0 > 0 && (r = reset(c, true))) return r;
      if ((r = mark(c, i0 / chunk, 0))) return r;
      hipLaunchKernelGGL(k_prep_each, dim3(blocks_for(m)), dim3(256), 0, c->stream, s + i0, q + i0,
                         m, zx + i0, zy + i0, rho + i0, tol, all_fs, c->tasks, c->cnt, mag + i0,
                         err + i0, ns + i0, flags + i0, tfeat);
      HIP_TRY(c, hipGetLastError());
      if ((r = contour_stage(c, i0 / chunk, mode, m, 1, mag + i0, err + i0, ns + i0, flags + i0)))
        return r;
    }
    return mark_call(c, 1);
  });
}

}  // extern "C"

namespace {
template <int LCAP>
void launch_noalloc_fs(twk_ctx* c, bool mixed, long long* cnt, Task* tasks, const int32_t* order,
                       char* sl, double* mag, double* err, int32_t* ns, uint32_t* flags) {
  const int ci = cap_index(LCAP);
  const int waves = std::min(NOALLOC_WAVES, c->occ[ci][mixed ? 1 : 0] * c->n_cu);
  if (mixed)
    hipLaunchKernelGGL((k_fs<LCAP, true>), dim3(waves), dim3(64), 0, c->stream, tasks,
                       &cnt[C_NTASK], &cnt[C_HEAD], sl, mag, err, ns, flags, cnt, order);
  else
    hipLaunchKernelGGL((k_fs<LCAP, false>), dim3(waves), dim3(64), 0, c->stream, tasks,
                       &cnt[C_NTASK], &cnt[C_HEAD], sl, mag, err, ns, flags, cnt, order);
}
}  // namespace

extern "C" {

int twk_finite_mag_noalloc(twk_ctx* c, double s, double q, int64_t n, const double* zx,
                           const double* zy, double rho, double tol, uint32_t mode, double* mag,
                           double* err, int32_t* ns, uint32_t* flags) {
  if (!c || !finite_pos(s) || !finite_pos(q) || !finite_pos(rho) || !finite_pos(tol) || n < 0 ||
      n > NOALLOC_MAX_N || (mode & ~(TWK_MODE_MIXED | TWK_MODE_ALL_FS)))
    return TWK_EINVAL;
  if (n == 0) return TWK_OK;
  if (!zx || !zy || !mag || !err || !ns || !flags) return TWK_EINVAL;
  if (!c->noalloc) return TWK_EDEVICE;
  HIP_TRY(c, hipSetDevice(c->device));
  long long* cnt = (long long*)c->noalloc;
  Task* tasks = (Task*)(c->noalloc + NOALLOC_TASK_OFF);
  char* sl = c->noalloc + NOALLOC_SLICE_OFF;
  const bool mixed = (mode & TWK_MODE_MIXED) != 0;
  const int all_fs = all_fs_of(mode);
  // the counters start at zero by a kernel (no memset node if captured)
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->stream, cnt, 0);
  HIP_TRY(c, hipGetLastError());
  hipLaunchKernelGGL(k_prep, dim3(blocks_for(n)), dim3(256), 0, c->stream, s, q, n, zx, zy, rho, tol,
                     all_fs, tasks, cnt, mag, err, ns, flags, (float*)nullptr);
  HIP_TRY(c, hipGetLastError());
  int32_t* order = (int32_t*)(c->noalloc + NOALLOC_ORDER_OFF);
  hipLaunchKernelGGL(k_stride, dim3(1), dim3(64), 0, c->stream, cnt, 1, 0);
  HIP_TRY(c, hipGetLastError());
  hipLaunchKernelGGL(k_disperse, dim3(c->n_cu), dim3(256), 0, c->stream, cnt, order);
  HIP_TRY(c, hipGetLastError());
  switch (c->tune.lds_cap) {
    case 64: launch_noalloc_fs<64>(c, mixed, cnt, tasks, order, sl, mag, err, ns, flags); break;
    case 256: launch_noalloc_fs<256>(c, mixed, cnt, tasks, order, sl, mag, err, ns, flags); break;
    default: launch_noalloc_fs<128>(c, mixed, cnt, tasks, order, sl, mag, err, ns, flags); break;
  }
  HIP_TRY(c, hipGetLastError());
  return TWK_OK;
}

int twk_mag_map(twk_ctx* c, double s, double q, double rho, double xc, double yc, double width,
                double height, int32_t nx, int32_t ny, double tol, uint32_t mode, double* mag,
                double* err, int32_t* ns, uint32_t* flags) {
  if (!c || !finite_pos(s) || !finite_pos(q) || !finite_pos(rho) || !finite_pos(tol) ||
      !finite_pos(width) || !finite_pos(height) || nx < 0 || ny < 0 || !std::isfinite(xc) ||
      !std::isfinite(yc))
    return TWK_EINVAL;
  int rc = check_mode(c, mode);
  if (rc) return rc;
  const int64_t n = (int64_t)nx * ny;
  if (n == 0) return TWK_OK;
  if (!mag || !err || !ns || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(ny, CHUNK_TASKS / nx));
  const bool learned = (mode & TWK_MODE_MLP) != 0;
  if ((rc = ensure_fs(c, rows * nx))) return rc;
  if (learned && (rc = ensure_learn(c, rows * nx))) return rc;
  const int all_fs = all_fs_of(mode);
  float* tfeat = learned ? learn_bufs(c).feat : nullptr;
  CallKey key;
  key.u(entry_key(2, mode)).d(s).d(q).d(rho).d(xc).d(yc).d(width).d(height).u((uint64_t)nx).u((uint64_t)ny).d(tol)
      .u(mode).p(mag).p(err).p(ns).p(flags);
  if ((rc = prepare_call(c, (ny + rows - 1) / rows))) return rc;
  return run_captured(c, tuning_key(key, c), [&]() -> int {
    int r;
    if ((r = mark_call(c, 0)) || (r = reset(c, false))) return r;
    for (int64_t y0 = 0; y0 < ny; y0 += rows) {
      const int64_t nr = std::min<int64_t>(rows, ny - y0);
      if (y0 > 0 && (r = reset(c, true))) return r;
      if ((r = mark(c, y0 / rows, 0))) return r;
      hipLaunchKernelGGL(k_map, dim3(blocks_for(nr * nx)), dim3(256), 0, c->stream, s, q, rho, xc,
                         yc, width, height, nx, ny, y0, nr, tol, all_fs, c->tasks, c->cnt, mag, err,
                         ns, flags, tfeat);
      HIP_TRY(c, hipGetLastError());
      if ((r = contour_stage(c, y0 / rows, mode, nr * nx, 1, mag, err, ns, flags)))
        return r;
    }
    return mark_call(c, 1);
  });
}

int twk_lightcurves(twk_ctx* c, int64_t nsets, const double* s, const double* q, const double* u0,
                    const double* alpha, const double* rho, const double* gamma, int64_t nepochs,
                    const double* tau, int32_t n_annuli, double tol, uint32_t mode, double* mag,
                    double* err, int32_t* ns, uint32_t* flags) {
  if (!c || !finite_pos(tol) || n_annuli < 1 || n_annuli > 64 ||
      !batch_size_ok(nsets, nepochs, n_annuli))
    return TWK_EINVAL;
  int rc = check_mode(c, mode);
  if (rc) return rc;
  if (gamma == nullptr && n_annuli != 1) return TWK_EINVAL;
  const int64_t n = nsets * nepochs;
  if (n == 0) return TWK_OK;
  if (!s || !q || !u0 || !alpha || !rho || !tau || !mag || !err || !ns || !flags) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const bool ld = gamma != nullptr;
  const int na = ld ? n_annuli : 1;
  const int64_t chunk_sets = std::max<int64_t>(1, CHUNK_TASKS / na / nepochs);
  const int64_t chunk_n = std::min(nsets, chunk_sets) * nepochs;
  const bool learned = (mode & TWK_MODE_MLP) != 0;
  if ((rc = ensure_fs(c, chunk_n * na))) return rc;
  if (learned && (rc = ensure_learn(c, chunk_n * na))) return rc;
  if (ld && (rc = ensure_ld(c, chunk_n, na))) return rc;
  const AnnBufs ab = ld ? ann_bufs(c, chunk_n * na) : AnnBufs{nullptr, nullptr, nullptr, nullptr};
  const int all_fs = all_fs_of(mode);
  float* tfeat = learned ? learn_bufs(c).feat : nullptr;
  int32_t* tslot = learned ? learn_bufs(c).slot : nullptr;
  CallKey key;
  key.u(entry_key(3, mode)).u((uint64_t)nsets).p(s).p(q).p(u0).p(alpha).p(rho).p(gamma).u((uint64_t)nepochs).p(tau)
      .u((uint64_t)n_annuli).d(tol).u(mode).p(mag).p(err).p(ns).p(flags);
  if ((rc = prepare_call(c, (nsets + chunk_sets - 1) / chunk_sets))) return rc;
  return run_captured(c, tuning_key(key, c), [&]() -> int {
    int r;
    if ((r = mark_call(c, 0)) || (r = reset(c, false))) return r;
    for (int64_t k0 = 0; k0 < nsets; k0 += chunk_sets) {
      const int64_t nk = std::min(chunk_sets, nsets - k0);
      const int64_t o = k0 * nepochs;
      if (k0 > 0 && (r = reset(c, true))) return r;
      if ((r = mark(c, k0 / chunk_sets, 0))) return r;
      hipLaunchKernelGGL(k_lc, dim3(blocks_for(lc_lanes(nk, nepochs))), dim3(256), 0, c->stream, nk,
                         s + k0, q + k0, u0 + k0, alpha + k0, rho + k0, ld ? gamma + k0 : nullptr,
                         nepochs, tau, tol, all_fs,
                         na, c->tasks, c->cnt, c->fs_epoch, mag + o, err + o, ns + o, flags + o,
                         tfeat, tslot);
      HIP_TRY(c, hipGetLastError());
      if (ld) r = contour_stage(c, k0 / chunk_sets, mode, nk * nepochs * na, na, ab.mag, ab.err,
                                ab.ns, ab.flags);
      else r = contour_stage(c, k0 / chunk_sets, mode, nk * nepochs, 1, mag + o, err + o, ns + o,
                             flags + o);
      if (r) return r;
      if (ld) {
        hipLaunchKernelGGL(k_ld, dim3(blocks_for(nk * nepochs)), dim3(256), 0, c->stream, c->cnt,
                           c->fs_epoch, na, gamma + k0, nepochs, ab.mag, ab.err, ab.ns, ab.flags,
                           mag + o, err + o, ns + o, flags + o);
        HIP_TRY(c, hipGetLastError());
      }
    }
    return mark_call(c, 1);
  });
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
  out8[7] = c->last_chunks;
  return TWK_OK;
}

int twk_enable_timing(twk_ctx* c, int on) {
  if (!c) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  while (on && c->ev.size() < 2) {
    hipEvent_t e = nullptr;
    HIP_TRY(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
  c->timing = on != 0;
  c->ev_chunks = 0;
  return TWK_OK;
}

int twk_kernel_times(twk_ctx* c, double* ms5) {
  if (!c || !ms5 || !c->timing) return TWK_EINVAL;
  HIP_TRY(c, hipEventSynchronize(c->ev[1]));
  double st[3] = {0.0, 0.0, 0.0};
  for (int64_t k = 0; k < c->ev_chunks; ++k)
    for (int j = 0; j < 3; ++j) {
      float v = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&v, c->ev[2 + 4 * k + j], c->ev[2 + 4 * k + j + 1]));
      st[j] += v;
    }
  float t = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&t, c->ev[0], c->ev[1]));
  for (int j = 0; j < 3; ++j) ms5[j] = st[j];
  ms5[3] = t - st[0] - st[1] - st[2];
  ms5[4] = t;
  return TWK_OK;
}

int twk_features(twk_ctx* c, int64_t nsets, const double* s, const double* q, const double* u0,
                 const double* alpha, const double* rho, int64_t nepochs, const double* tau,
                 double tol, float* feat, double* mu_ps, int32_t* adequate) {
  if (!c || !finite_pos(tol) || !batch_size_ok(nsets, nepochs, 1)) return TWK_EINVAL;
  const int64_t n = nsets * nepochs;
  if (n == 0) return TWK_OK;
  if (!s || !q || !u0 || !alpha || !rho || !tau || !feat || !mu_ps || !adequate) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t kc = std::max<int64_t>(1, LAUNCH_MAX / nepochs);  // sets per launch
  for (int64_t k0 = 0; k0 < nsets; k0 += kc) {
    const int64_t nk = std::min(kc, nsets - k0), o = k0 * nepochs;
    hipLaunchKernelGGL(k_feat, dim3(blocks_for(nk * nepochs)), dim3(256), 0, c->stream, nk,
                       s + k0, q + k0, u0 + k0, alpha + k0, rho + k0, nepochs, tau, tol,
                       feat + o * 8, mu_ps + o, adequate + o);
    HIP_TRY(c, hipGetLastError());
  }
  return TWK_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ learned part (host)
namespace {

using mlp::NPARAM;

int mlp_alloc(twk_ctx* c) {
  if (c->mlp_p) return TWK_OK;
  if (hipMalloc((void**)&c->mlp_p, NPARAM * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&c->mlp_frag, mlp::NFRAG * 64 * sizeof(mlp::bf16x8)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(c->mlp_p);
    (void)hipFree(c->mlp_frag);
    c->mlp_p = nullptr;
    c->mlp_frag = nullptr;
    return TWK_ENOMEM;
  }
  return TWK_OK;
}

int mlp_pack(twk_ctx* c) {
  hipLaunchKernelGGL(mlp::k_pack, dim3(mlp::NFRAG), dim3(64), 0, c->stream, c->mlp_p, c->mlp_frag);
  HIP_TRY(c, hipGetLastError());
  c->mlp_ready = true;
  return TWK_OK;
}

bool params_valid(const float* h) {
  for (int i = 0; i < NPARAM; ++i)
    if (!std::isfinite(h[i])) return false;
  for (int j = 0; j < mlp::NF; ++j)
    if (!(h[mlp::OFF_STD + j] > 0.0f)) return false;
  return true;
}

// splitmix64 (Steele, Lea & Flood 2014): the generator behind weight
// initialisation and minibatch shuffles.
uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& x) { return ((splitmix64(x) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

// Box-Muller transform of two uniforms.
double normal(uint64_t& x) {
  const double u1 = uniform01(x), u2 = uniform01(x);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

// Training workspace for minibatches of B rows (float32 unless noted).
struct TrainBufs {
  float *X, *yb, *yf, *Z[3], *H[3], *O, *dO, *dA, *dB, *lrow, *work;
};
constexpr int KSPLIT_MAX = 16;

size_t train_floats(int64_t B) {
  return (size_t)B * (8 + 1 + 1 + 6 * mlp::HID + 2 + 2 + 2 * mlp::HID + 1) +
         (size_t)KSPLIT_MAX * mlp::HID * mlp::HID;
}

TrainBufs train_bufs(float* base, int64_t B) {
  TrainBufs t;
  float* p = base;
  auto take = [&](size_t n) { float* r = p; p += n; return r; };
  t.X = take(B * 8);
  t.yb = take(B);
  t.yf = take(B);
  for (int l = 0; l < 3; ++l) {
    t.Z[l] = take(B * mlp::HID);
    t.H[l] = take(B * mlp::HID);
  }
  t.O = take(B * 2);
  t.dO = take(B * 2);
  t.dA = take(B * mlp::HID);
  t.dB = take(B * mlp::HID);
  t.lrow = take(B);
  t.work = take((size_t)KSPLIT_MAX * mlp::HID * mlp::HID);
  return t;
}

int ensure_train(twk_ctx* c, int64_t B, int64_t nperm, int64_t nsteps) {
  int rc;
  if ((rc = grow(c, (void**)&c->tr, &c->tr_bytes, train_floats(B) * sizeof(float)))) return rc;
  size_t have = c->opt ? (size_t)3 * NPARAM * sizeof(float) : 0;
  if ((rc = grow(c, (void**)&c->opt, &have, (size_t)3 * NPARAM * sizeof(float)))) return rc;
  if ((rc = grow(c, (void**)&c->perm, &c->perm_bytes,
                 (size_t)std::max<int64_t>(nperm, 1) * sizeof(int32_t))))
    return rc;
  return grow(c, (void**)&c->dsum, &c->dsum_bytes, (size_t)std::max<int64_t>(nsteps, 1) * 8);
}

unsigned ew_blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// C = A B on the matrix cores (layout strides as in mlp::Gemm); K is split
// for the weight gradients, whose contraction runs over the batch.
int gemm(twk_ctx* c, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
         int64_t sbn, float* C, int64_t scm, int64_t scn, int M, int N, int K, float* work) {
  mlp::Gemm g{A, sam, sak, B, sbk, sbn, C, scm, scn, M, N, K, 1, work};
  if (K >= 512) g.ksplit = std::min(KSPLIT_MAX, K / 256);
  dim3 grid((M + 31) / 32, (N + 31) / 32, g.ksplit);
  hipLaunchKernelGGL(mlp::k_gemm, grid, dim3(64), 0, c->stream, g);
  HIP_TRY(c, hipGetLastError());
  if (g.ksplit > 1) {
    hipLaunchKernelGGL(mlp::k_split_sum, dim3(ew_blocks((int64_t)M * N)), dim3(256), 0, c->stream,
                       work, g.ksplit, M, N, C, scm, scn);
    HIP_TRY(c, hipGetLastError());
  }
  return TWK_OK;
}

// Forward and backward pass of one standardised minibatch already in t.X,
// t.yb, t.yf: gradient of the mean loss into G (flat parameter layout; the
// standardisation entries are left alone), batch loss sum into *lsum.
int forward_backward(twk_ctx* c, const TrainBufs& t, int64_t rows, float delta, float* G,
                     double* lsum) {
  using namespace mlp;
  const float* P = c->mlp_p;
  const int R = (int)rows;
  int rc;
  const int64_t offW[4] = {OFF_W0, OFF_W1, OFF_W2, OFF_W3};
  const int64_t offB[4] = {OFF_B0, OFF_B1, OFF_B2, OFF_B3};
  // forward
  const float* in = t.X;
  int64_t kin = NF;
  for (int l = 0; l < 3; ++l) {
    if ((rc = gemm(c, in, kin, 1, P + offW[l], HID, 1, t.Z[l], HID, 1, R, HID, (int)kin, t.work)))
      return rc;
    hipLaunchKernelGGL(k_bias_act, dim3(ew_blocks(rows * HID)), dim3(256), 0, c->stream, t.Z[l],
                       P + offB[l], t.H[l], rows, HID);
    HIP_TRY(c, hipGetLastError());
    in = t.H[l];
    kin = HID;
  }
  if ((rc = gemm(c, t.H[2], HID, 1, P + OFF_W3, NO, 1, t.O, NO, 1, R, NO, HID, t.work))) return rc;
  hipLaunchKernelGGL(k_bias_act, dim3(ew_blocks(rows * NO)), dim3(256), 0, c->stream, t.O,
                     P + OFF_B3, (float*)nullptr, rows, NO);
  HIP_TRY(c, hipGetLastError());
  hipLaunchKernelGGL(k_loss, dim3(ew_blocks(rows)), dim3(256), 0, c->stream, t.O, t.yb, t.yf,
                     delta, rows, t.dO, t.lrow);
  HIP_TRY(c, hipGetLastError());
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, c->stream, t.lrow, rows, lsum);
  HIP_TRY(c, hipGetLastError());
  // backward: dZ of layer l lives in dz (width w); its input activation is
  // H[l-1] (X for layer 0)
  const float* dz = t.dO;
  int w = NO;
  float* spare[2] = {t.dA, t.dB};
  for (int l = 3; l >= 0; --l) {
    const float* a = l > 0 ? t.H[l - 1] : t.X;
    const int ka = l > 0 ? HID : NF;
    // dW_l = a^T dz  (ka x w), contraction over the batch
    if ((rc = gemm(c, a, 1, ka, dz, w, 1, G + offW[l], w, 1, ka, w, R, t.work))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3((w + 127) / 128), dim3(128), 0, c->stream, dz, rows, w,
                       G + offB[l]);
    HIP_TRY(c, hipGetLastError());
    if (l == 0) break;
    // dH_{l-1} = dz W_l^T, then dZ_{l-1} = dH_{l-1} gelu'(Z_{l-1})
    float* dh = spare[l & 1];
    if ((rc = gemm(c, dz, w, 1, P + offW[l], 1, w, dh, HID, 1, R, HID, w, t.work))) return rc;
    hipLaunchKernelGGL(k_gelu_bwd, dim3(ew_blocks(rows * HID)), dim3(256), 0, c->stream, dh,
                       t.Z[l - 1], rows * HID);
    HIP_TRY(c, hipGetLastError());
    dz = dh;
    w = HID;
  }
  return TWK_OK;
}

}  // namespace

extern "C" {

int twk_mlp_set(twk_ctx* c, const float* host, int64_t n) {
  if (!c || !host || n != NPARAM || !params_valid(host)) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  int rc = mlp_alloc(c);
  if (rc) return rc;
  HIP_TRY(c, hipMemcpyAsync(c->mlp_p, host, NPARAM * sizeof(float), hipMemcpyHostToDevice,
                            c->stream));
  if ((rc = mlp_pack(c))) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TWK_OK;
}

int twk_mlp_get(twk_ctx* c, float* host, int64_t n) {
  if (!c || !host || n != NPARAM) return TWK_EINVAL;
  if (!c->mlp_ready) return TWK_ENOMLP;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(host, c->mlp_p, NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TWK_OK;
}

static const char kMagic[8] = {'T', 'W', 'K', 'M', 'L', 'P', '0', '1'};

int twk_mlp_save(twk_ctx* c, const char* path) {
  if (!c || !path) return TWK_EINVAL;
  float* h = (float*)std::malloc(NPARAM * sizeof(float));
  if (!h) return TWK_ENOMEM;
  int rc = twk_mlp_get(c, h, NPARAM);
  if (rc == TWK_OK) {
    FILE* f = std::fopen(path, "wb");
    const int32_t n = NPARAM;
    if (!f) rc = TWK_EINVAL;
    else {
      if (std::fwrite(kMagic, 1, 8, f) != 8 || std::fwrite(&n, 4, 1, f) != 1 ||
          std::fwrite(h, sizeof(float), NPARAM, f) != (size_t)NPARAM)
        rc = TWK_EINVAL;
      if (std::fclose(f) != 0) rc = TWK_EINVAL;
    }
  }
  std::free(h);
  return rc;
}

int twk_mlp_load(twk_ctx* c, const char* path) {
  if (!c || !path) return TWK_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return TWK_EINVAL;
  char magic[8];
  int32_t n = 0;
  float* h = (float*)std::malloc(NPARAM * sizeof(float));
  int rc = TWK_OK;
  if (!h) rc = TWK_ENOMEM;
  else if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, kMagic, 8) != 0 ||
           std::fread(&n, 4, 1, f) != 1 || n != NPARAM ||
           std::fread(h, sizeof(float), NPARAM, f) != (size_t)NPARAM)
    rc = TWK_EINVAL;
  std::fclose(f);
  if (rc == TWK_OK) rc = twk_mlp_set(c, h, NPARAM);
  std::free(h);
  return rc;
}

int twk_mlp_infer(twk_ctx* c, int64_t n, const float* feat, float* out) {
  if (!c || n < 0 || n > MAX_ELEMS) return TWK_EINVAL;
  if (!c->mlp_ready) return TWK_ENOMLP;
  if (n == 0) return TWK_OK;
  if (!feat || !out) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t tiles = (n + 31) / 32;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(c->n_cu * 2, (tiles + 3) / 4));
  hipLaunchKernelGGL(mlp::k_infer, dim3((unsigned)blocks), dim3(64 * mlp::INFER_WAVES), 0,
                     c->stream, c->mlp_p, c->mlp_frag, n, (const long long*)nullptr, feat, out,
                     (long long*)nullptr, 0.0f, 1, (int32_t*)nullptr);
  HIP_TRY(c, hipGetLastError());
  return TWK_OK;
}

int twk_mlp_grad(twk_ctx* c, int64_t n, const float* feat, const float* yb, const float* yf,
                 float huber_delta, float* grad, double* loss) {
  if (!c || n < 1 || n > TWK_MLP_GRAD_MAX_ROWS || !feat || !yb || !yf || !grad || !loss ||
      !(huber_delta > 0.0f))
    return TWK_EINVAL;
  if (!c->mlp_ready) return TWK_ENOMLP;
  HIP_TRY(c, hipSetDevice(c->device));
  int rc = ensure_train(c, n, 1, 1);
  if (rc) return rc;
  const TrainBufs t = train_bufs((float*)c->tr, n);
  hipLaunchKernelGGL(mlp::k_gather, dim3(ew_blocks(n)), dim3(256), 0, c->stream, feat, yb, yf,
                     (const int32_t*)nullptr, n, c->mlp_p, t.X, t.yb, t.yf);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemsetAsync(grad, 0, 16 * sizeof(float), c->stream));
  if ((rc = forward_backward(c, t, n, huber_delta, grad, c->dsum))) return rc;
  double s = 0.0;
  HIP_TRY(c, hipMemcpyAsync(&s, c->dsum, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *loss = s / (double)n;
  return TWK_OK;
}

int twk_mlp_train(twk_ctx* c, int64_t n, const float* feat, const float* yb, const float* yf,
                  const twk_train_cfg* cfg, float* loss_hist) {
  if (!c || !cfg || !feat || !yb || !yf || cfg->epochs < 1 || cfg->batch < 32 ||
      cfg->batch > TWK_MLP_GRAD_MAX_ROWS || n < cfg->batch || !(cfg->lr > 0.0f) ||
      !(cfg->lr_end >= 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
      !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f) ||
      !(cfg->huber_delta > 0.0f) || n > (int64_t)INT32_MAX)
    return TWK_EINVAL;
  if (!cfg->init && !c->mlp_ready) return TWK_ENOMLP;
  HIP_TRY(c, hipSetDevice(c->device));
  int rc = mlp_alloc(c);
  if (rc) return rc;
  const int64_t B = cfg->batch;
  const int64_t steps = n / B;
  if ((rc = ensure_train(c, B, n, steps))) return rc;
  uint64_t rng = cfg->seed;
  float* G = c->opt;
  float* m1 = c->opt + NPARAM;
  float* m2 = c->opt + 2 * NPARAM;
  if (cfg->init) {
    // standardisation from the data (double sums per block, added in order)
    const int nb = 256;
    double* part = nullptr;
    if (hipMalloc((void**)&part, nb * 16 * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return TWK_ENOMEM;
    }
    hipLaunchKernelGGL(mlp::k_feat_stats, dim3(nb), dim3(256), 0, c->stream, feat, n, part);
    std::vector<double> hp((size_t)nb * 16);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(part);
    if (e != hipSuccess) return hip_fail(c, e);
    std::vector<float> h(NPARAM, 0.0f);
    for (int j = 0; j < mlp::NF; ++j) {
      double s1 = 0.0, s2 = 0.0;
      for (int b = 0; b < nb; ++b) {
        s1 += hp[b * 16 + j];
        s2 += hp[b * 16 + 8 + j];
      }
      const double mean = s1 / n, var = std::max(s2 / n - mean * mean, 0.0);
      h[mlp::OFF_MEAN + j] = (float)mean;
      h[mlp::OFF_STD + j] = (float)std::max(std::sqrt(var), 1e-6);
    }
    // He-normal weights, zero biases
    const int64_t offW[4] = {mlp::OFF_W0, mlp::OFF_W1, mlp::OFF_W2, mlp::OFF_W3};
    const int fan[4] = {mlp::NF, mlp::HID, mlp::HID, mlp::HID};
    const int width[4] = {mlp::HID, mlp::HID, mlp::HID, mlp::NO};
    for (int l = 0; l < 4; ++l) {
      const double sd = std::sqrt(2.0 / fan[l]);
      for (int64_t i = 0; i < (int64_t)fan[l] * width[l]; ++i)
        h[offW[l] + i] = (float)(sd * normal(rng));
    }
    HIP_TRY(c, hipMemcpyAsync(c->mlp_p, h.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  HIP_TRY(c, hipMemsetAsync(c->opt, 0, (size_t)3 * NPARAM * sizeof(float), c->stream));
  const TrainBufs t = train_bufs((float*)c->tr, B);
  std::vector<int32_t> perm((size_t)n);
  std::vector<double> ls((size_t)steps);
  const int64_t total = (int64_t)cfg->epochs * steps;
  int64_t it = 0;
  for (int ep = 0; ep < cfg->epochs; ++ep) {
    // Fisher-Yates shuffle of the rows
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
      const int64_t j = (int64_t)(uniform01(rng) * (double)(i + 1));
      std::swap(perm[i], perm[std::min(j, i)]);
    }
    HIP_TRY(c, hipMemcpyAsync(c->perm, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice,
                              c->stream));
    for (int64_t st = 0; st < steps; ++st, ++it) {
      hipLaunchKernelGGL(mlp::k_gather, dim3(ew_blocks(B)), dim3(256), 0, c->stream, feat, yb, yf,
                         c->perm + st * B, B, c->mlp_p, t.X, t.yb, t.yf);
      HIP_TRY(c, hipGetLastError());
      if ((rc = forward_backward(c, t, B, cfg->huber_delta, G, c->dsum + st))) return rc;
      const double frac = total > 1 ? (double)it / (double)(total - 1) : 0.0;
      const float lr = (float)(cfg->lr + (cfg->lr_end - cfg->lr) * frac);
      const double k = (double)(it + 1);
      const float c1 = (float)(1.0 - std::pow((double)cfg->beta1, k));
      const float c2 = (float)(1.0 - std::pow((double)cfg->beta2, k));
      hipLaunchKernelGGL(mlp::k_adam, dim3(ew_blocks(NPARAM - 16)), dim3(256), 0, c->stream,
                         c->mlp_p, G, m1, m2, (int64_t)16, (int64_t)NPARAM, lr, cfg->beta1,
                         cfg->beta2, cfg->eps, c1, c2);
      HIP_TRY(c, hipGetLastError());
    }
    HIP_TRY(c, hipMemcpyAsync(ls.data(), c->dsum, (size_t)steps * 8, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (loss_hist) {
      double s = 0.0;
      for (int64_t st = 0; st < steps; ++st) s += ls[st];
      loss_hist[ep] = (float)(s / (double)(steps * B));
    }
  }
  if ((rc = mlp_pack(c))) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TWK_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuning
extern "C" {

int twk_get_tuning(twk_ctx* c, twk_tuning* out) {
  if (!c || !out) return TWK_EINVAL;
  *out = c->tune;
  return TWK_OK;
}

int twk_set_tuning(twk_ctx* c, const twk_tuning* t) {
  if (!c || !t) return TWK_EINVAL;
  if (cap_index(t->lds_cap) < 0 || !(t->budget_shift >= -2.0f && t->budget_shift <= 4.0f) ||
      (t->graphs != 0 && t->graphs != 1))
    return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  int mx = 0;
  if (max_waves(t->lds_cap, &mx) != TWK_OK) return TWK_EDEVICE;
  if (t->waves_per_cu < 1 || t->waves_per_cu > mx) return TWK_EINVAL;
  // capture needs a created stream (the legacy null stream cannot be captured)
  if (t->graphs && c->stream == nullptr) return TWK_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  drop_graphs(c);
  c->tune = *t;
  return TWK_OK;
}

int twk_autotune(twk_ctx* c, int64_t nsets, const double* s, const double* q, const double* u0,
                 const double* alpha, const double* rho, const double* gamma, int64_t nepochs,
                 const double* tau, int32_t n_annuli, double tol, uint32_t mode, int32_t trials,
                 twk_tuning* best) {
  if (!c || trials < 1 || trials > 100 || nsets < 1 || nepochs < 1 ||
      !batch_size_ok(nsets, nepochs, n_annuli > 0 ? n_annuli : 1))
    return TWK_EINVAL;
  int rc = check_mode(c, mode);
  if (rc) return rc;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t n = nsets * nepochs;
  char* out = nullptr;
  if (hipMalloc((void**)&out, (size_t)n * 24) != hipSuccess) {
    (void)hipGetLastError();
    return TWK_ENOMEM;
  }
  double* mag = (double*)out;
  double* err = (double*)(out + (size_t)n * 8);
  int32_t* ns = (int32_t*)(out + (size_t)n * 16);
  uint32_t* fl = (uint32_t*)(out + (size_t)n * 20);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const twk_tuning start = c->tune;
  const bool timing = c->timing;
  c->timing = false;
  twk_tuning cur = start, top = start;
  cur.graphs = 0;
  double best_ms = 1e300;
  auto measure = [&](const twk_tuning& t, double* ms) -> int {
    int r;
    if ((r = twk_set_tuning(c, &t))) return r;
    // the first call sizes the buffers; then the fastest of `trials` calls
    if ((r = twk_lightcurves(c, nsets, s, q, u0, alpha, rho, gamma, nepochs, tau, n_annuli, tol,
                             mode, mag, err, ns, fl)))
      return r;
    double m = 1e300;
    for (int k = 0; k < trials; ++k) {
      HIP_TRY(c, hipEventRecord(e0, c->stream));
      if ((r = twk_lightcurves(c, nsets, s, q, u0, alpha, rho, gamma, nepochs, tau, n_annuli, tol,
                               mode, mag, err, ns, fl)))
        return r;
      HIP_TRY(c, hipEventRecord(e1, c->stream));
      HIP_TRY(c, hipEventSynchronize(e1));
      float f = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&f, e0, e1));
      m = std::min(m, (double)f);
    }
    *ms = m;
    return TWK_OK;
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = hip_fail(c, hipGetLastError());
  } else {
    // persistent grid and LDS capacity
    for (int ci = 0; ci < 3 && rc == TWK_OK; ++ci) {
      int mx = 0;
      if ((rc = max_waves(LDS_CAPS[ci], &mx)) != TWK_OK) break;
      int last = 0;
      for (int f = 1; f <= 4 && rc == TWK_OK && mx > 0; ++f) {
        const int w = std::max(1, (mx * f) / 4);
        if (w == last) continue;
        last = w;
        cur.lds_cap = LDS_CAPS[ci];
        cur.waves_per_cu = w;
        double ms;
        if ((rc = measure(cur, &ms)) == TWK_OK && ms < best_ms) {
          best_ms = ms;
          top = cur;
        }
      }
    }
  }
  (void)hipStreamSynchronize(c->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  c->timing = timing;
  top.graphs = start.graphs;
  if (rc == TWK_OK) rc = twk_set_tuning(c, &top);
  else (void)twk_set_tuning(c, &start);
  if (rc == TWK_OK && best) *best = top;
  return rc;
}

}  // extern "C"
