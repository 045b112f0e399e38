// Host driver that runs the device contour engine (fs_source) of the HIP
// library on the CPU, one emulated 64-lane wavefront per source, and the
// device point-source classification, exposing a small C ABI to the tests.
// Test infrastructure only: the product library never uses it.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../paper_2501_03322_amd/csrc/twk_fs.h"
#include "../../paper_2501_03322_amd/csrc/twk_gelu.h"
#include "../../paper_2501_03322_amd/csrc/twk_queue.h"

using namespace twk;

namespace {
#ifndef EMU_LCAP
#define EMU_LCAP 512
#endif
constexpr int LCAP = EMU_LCAP;

template <bool MIXED>
struct WaveJob {
  const Task* T;
  double tol;
  int n0;
  WaveMem<MIXED> m;
  FsLds<LCAP, MIXED>* lds;
  FsOut* out;
  // round-by-round dispatch
  RoundState* rs;
  bool fresh;
  bool done;
};

template <bool MIXED>
void lane_source(int l, void* p) {
  auto* j = (WaveJob<MIXED>*)p;
  FsOut o = fs_source<LCAP, MIXED>(*j->T, j->tol, j->m, *j->lds, l, j->n0);
  if (l == 0) *j->out = o;
}

template <bool MIXED>
void lane_round(int l, void* p) {
  auto* j = (WaveJob<MIXED>*)p;
  FsOut o;
  const bool d = fs_round_step<MIXED>(*j->T, j->tol, j->m, (lint*)j->lds->ivl, l, j->n0, j->rs,
                                      j->fresh, &o);
  if (l == 0) {
    j->done = d;
    if (d) *j->out = o;
  }
}

template <bool MIXED>
void run_wave_t(const Task& T, double tol, int n0, FsOut* out) {
  std::vector<char> scratch((size_t)METHOD_CAP * kSlotBytesMax);
  auto* lds = new FsLds<LCAP, MIXED>();
  WaveJob<MIXED> j{&T, tol, n0, wave_mem<MIXED>(scratch.data(), 0), lds, out, nullptr, false, false};
  hip_emu::run_wave(&lane_source<MIXED>, &j);
  delete lds;
}

// The round-by-round dispatch: one emulated launch per round until the
// source is finished; returns the number of launches.
template <bool MIXED>
int run_rounds_t(const Task& T, double tol, int n0, FsOut* out) {
  std::vector<char> scratch((size_t)METHOD_CAP * kSlotBytesMax);
  auto* lds = new FsLds<LCAP, MIXED>();
  RoundState rs{};
  WaveJob<MIXED> j{&T, tol, n0, wave_mem<MIXED>(scratch.data(), 0), lds, out, &rs, true, false};
  int launches = 0;
  while (!j.done) {
    hip_emu::run_wave(&lane_round<MIXED>, &j);
    j.fresh = false;
    ++launches;
  }
  delete lds;
  return launches;
}

void run_wave(const Task& T, double tol, bool mixed, int n0, FsOut* out) {
  if (mixed) run_wave_t<true>(T, tol, n0, out);
  else run_wave_t<false>(T, tol, n0, out);
}
}  // namespace

extern "C" {

// The contour queue's dispersal arithmetic (twk_queue.h), as the kernels
// use it.
void emu_golden_stride(long long n, long long* g, long long* ginv) { golden_stride(n, g, ginv); }
long long emu_dispersed_task(long long p, unsigned long long g, long long grp, long long ng) {
  return dispersed_task(p, g, grp, ng);
}
long long emu_merged_place(int long_row, long long q, long long n0, long long n1) {
  return long_row ? merged_place_long(q, n0, n1) : merged_place_other(q, n0, n1);
}

// Centre roots by the device cold-start solve, then the contour engine
// starting from a uniform grid of n0 samples (a multiple of 64, at most the
// LDS capacity the emulation is built with).
int emu_finite_mag(double s, double q, double zx, double zy, double rho, double tol, int mixed,
                   int n0, double* mag, double* err, int* nsamp, unsigned* flags, double* sweeps) {
  const Lens L = make_lens(s, q);
  const c64 yc = cz(zx - L.z2, zy);
  Images im;
  int it;
  solve_point_cold(L, yc, im, it);
  Task T;
  T.out = 0;
  T.s = s;
  T.q = q;
  T.rho = rho;
  T.zx = zx;
  T.zy = zy;
  T.tol = tol;
  for (int k = 0; k < 5; ++k) T.roots[k] = im.z[k];
  FsOut o;
  if (n0 < 64 || n0 > LCAP || n0 % 64) return -1;
  run_wave(T, tol, mixed != 0, n0, &o);
  *mag = o.mag;
  *err = o.err;
  *nsamp = o.n;
  *flags = o.flags;
  if (sweeps) {
    sweeps[0] = o.sweeps32;
    sweeps[1] = o.sweeps64;
    sweeps[2] = o.intervals;
  }
  return 0;
}

// The same source by the round-by-round dispatch (one emulated launch per
// refinement round, records in the global slice between launches).
int emu_finite_mag_rounds(double s, double q, double zx, double zy, double rho, double tol,
                          int mixed, double* mag, double* err, int* nsamp, unsigned* flags,
                          double* sweeps, int* launches) {
  const Lens L = make_lens(s, q);
  Images im;
  int it;
  solve_point_cold(L, cz(zx - L.z2, zy), im, it);
  Task T;
  T.out = 0;
  T.s = s;
  T.q = q;
  T.rho = rho;
  T.zx = zx;
  T.zy = zy;
  T.tol = tol;
  for (int k = 0; k < 5; ++k) T.roots[k] = im.z[k];
  FsOut o;
  *launches = mixed ? run_rounds_t<true>(T, tol, NNEW, &o) : run_rounds_t<false>(T, tol, NNEW, &o);
  *mag = o.mag;
  *err = o.err;
  *nsamp = o.n;
  *flags = o.flags;
  sweeps[0] = o.sweeps32;
  sweeps[1] = o.sweeps64;
  sweeps[2] = o.intervals;
  return 0;
}

// sin and cos of n limb angles by the device routine
void emu_limb_sincos(int n, const double* theta, double* sn, double* cs) {
  for (int i = 0; i < n; ++i) limb_sincos(theta[i], &sn[i], &cs[i]);
}

void emu_gelu(int n, const float* x, float* y, float* dy) {
  for (int i = 0; i < n; ++i) {
    y[i] = mlp::gelu(x[i]);
    dy[i] = mlp::gelu_grad(x[i]);
  }
}

int emu_point(double s, double q, double zx, double zy, double* mag, int* n, unsigned* flags,
              double* img10) {
  const Lens L = make_lens(s, q);
  Images im;
  int it;
  solve_point_cold(L, cz(zx - L.z2, zy), im, it);
  *mag = point_mag(im);
  *n = im.n;
  *flags = im.flags;
  for (int k = 0; k < 5; ++k) {
    img10[2 * k] = im.z[k].x + L.z2;
    img10[2 * k + 1] = im.z[k].y;
  }
  return 0;
}
}
