// twk_device.h -- device numerics for the binary-lens hot path (gfx950).
//
// Paper: Wang, Wang & Dong, "Twinkle: A GPU-based binary-lens microlensing
// code with contour integration method" (arXiv 2501.03322).
//
// Everything here runs per lane: one lane owns one point source (a source
// centre, a stencil point or one limb sample).  Complex numbers are carried
// as two doubles (or two floats for the mixed-precision root iterations).
// Frame: lens-2 frame of Sec. 2.2, y = zeta - z2, eta = z - z2; lens 1 at -s.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace twk {

// ---------------------------------------------------------------- complex
struct c64 {
  double x, y;
};
struct c32 {
  float x, y;
};

__device__ __forceinline__ c64 cz(double x, double y) { return c64{x, y}; }
__device__ __forceinline__ c64 operator+(c64 a, c64 b) { return c64{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c64 operator-(c64 a, c64 b) { return c64{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c64 operator-(c64 a) { return c64{-a.x, -a.y}; }
__device__ __forceinline__ c64 operator*(c64 a, c64 b) {
  return c64{__builtin_fma(a.x, b.x, -a.y * b.y), __builtin_fma(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ c64 operator*(double s, c64 a) { return c64{s * a.x, s * a.y}; }
__device__ __forceinline__ c64 operator+(c64 a, double s) { return c64{a.x + s, a.y}; }
__device__ __forceinline__ c64 operator-(c64 a, double s) { return c64{a.x - s, a.y}; }
__device__ __forceinline__ c64 cconj(c64 a) { return c64{a.x, -a.y}; }
__device__ __forceinline__ double cnorm(c64 a) { return __builtin_fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ double cabs64(c64 a) { return sqrt(cnorm(a)); }

// Square root of x >= 0 for lengths that only rank candidates or meet a
// threshold (linking distances, residual lengths): Goldschmidt's iteration
// from the hardware reciprocal square root (one coupled step, then one
// Newton correction), within about one ulp; x = 0 gives 0.
__device__ __forceinline__ double sqrt_fast(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  g = __builtin_fma(__builtin_fma(-g, g, x), h, g);
  return x > 0.0 ? g : 0.0;
}
__device__ __forceinline__ double cabs_fast(c64 a) { return sqrt_fast(cnorm(a)); }
// a ^ b = Im(conj(a) b);  a . b = Re(conj(a) b)
__device__ __forceinline__ double cwedge(c64 a, c64 b) { return __builtin_fma(a.x, b.y, -a.y * b.x); }
__device__ __forceinline__ double cdot(c64 a, c64 b) { return __builtin_fma(a.x, b.x, a.y * b.y); }

// Reciprocal of a finite nonzero double to full precision: hardware
// estimate plus two Newton steps (each squares the relative error).  The
// quotients on the hot path never need IEEE rounding, only full precision.
__device__ __forceinline__ double rcp64(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = __builtin_fma(-a, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-a, r, 1.0);
  return __builtin_fma(r, e, r);
}
// a * b + c with four fused multiply-adds
__device__ __forceinline__ c64 cfma(c64 a, c64 b, c64 c) {
  return c64{__builtin_fma(a.x, b.x, __builtin_fma(-a.y, b.y, c.x)),
             __builtin_fma(a.x, b.y, __builtin_fma(a.y, b.x, c.y))};
}
__device__ __forceinline__ c64 cinv(c64 b) {
  double r = rcp64(cnorm(b));
  return c64{b.x * r, -b.y * r};
}
__device__ __forceinline__ c64 cdiv(c64 a, c64 b) { return a * cinv(b); }

__device__ __forceinline__ c32 operator+(c32 a, c32 b) { return c32{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c32 operator-(c32 a, c32 b) { return c32{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c32 operator*(c32 a, c32 b) {
  return c32{__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ float cnorm(c32 a) { return __builtin_fmaf(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ c32 cfma(c32 a, c32 b, c32 c) {
  return c32{__builtin_fmaf(a.x, b.x, __builtin_fmaf(-a.y, b.y, c.x)),
             __builtin_fmaf(a.x, b.y, __builtin_fmaf(a.y, b.x, c.y))};
}
__device__ __forceinline__ c32 cinv(c32 b) {
  float r = __builtin_amdgcn_rcpf(cnorm(b));
  return c32{b.x * r, -b.y * r};
}

// ---------------------------------------------------------------- angles
// sin and cos of a limb angle (|theta| <= 8; the engine's angles lie in
// [0, 2 pi]).  Cody-Waite reduction by pi/2: theta = k pi/2 + r with pi/2
// split into three doubles whose first two carry 33 significant bits, so
// that k times each part is exact for the few quadrants used and r is exact
// to about 1e-17; then the Taylor series of sin r through r^15 and of cos r
// through r^16 on |r| <= pi/4 (truncation below 1e-16 relative), by Horner's
// rule in r^2.  About one ulp; the library routine carries a reduction for
// any argument, which this path does not need.
__device__ __forceinline__ void limb_sincos(double theta, double* sn, double* cs) {
  constexpr double PIO2_1 = 1.5707963267341256;     // pi/2, first 33 bits
  constexpr double PIO2_2 = 6.077100506303966e-11;  // next 33 bits
  constexpr double PIO2_3 = 2.0222662487959506e-21; // remainder
  const double kf = __builtin_rint(theta * 0.6366197723675814);
  const int k = (int)kf;
  const double r = ((theta - kf * PIO2_1) - kf * PIO2_2) - kf * PIO2_3;
  const double r2 = r * r;
  // 1/n! with alternating signs
  double ps = 1.0 / 1307674368000.0;   // r^15: -1/15!, sign applied below
  ps = __builtin_fma(ps, -r2, 1.0 / 6227020800.0);
  ps = __builtin_fma(ps, -r2, 1.0 / 39916800.0);
  ps = __builtin_fma(ps, -r2, 1.0 / 362880.0);
  ps = __builtin_fma(ps, -r2, 1.0 / 5040.0);
  ps = __builtin_fma(ps, -r2, 1.0 / 120.0);
  ps = __builtin_fma(ps, -r2, 1.0 / 6.0);
  const double s = __builtin_fma(-ps * r2, r, r);
  double pc = 1.0 / 20922789888000.0;  // r^16: +1/16!
  pc = __builtin_fma(pc, -r2, 1.0 / 87178291200.0);
  pc = __builtin_fma(pc, -r2, 1.0 / 479001600.0);
  pc = __builtin_fma(pc, -r2, 1.0 / 3628800.0);
  pc = __builtin_fma(pc, -r2, 1.0 / 40320.0);
  pc = __builtin_fma(pc, -r2, 1.0 / 720.0);
  pc = __builtin_fma(pc, -r2, 1.0 / 24.0);
  pc = __builtin_fma(pc, -r2, 0.5);
  const double c = __builtin_fma(-pc, r2, 1.0);
  const int q = k & 3;
  *sn = q == 0 ? s : (q == 1 ? c : (q == 2 ? -s : -c));
  *cs = q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
}

// ---------------------------------------------------------------- lens
// Sec. 2.1: masses normalised by the total mass; m1 = 1/(1+q), m2 = q/(1+q);
// lens 2 at z2 = s/(1+q) in the centre-of-mass frame.
struct Lens {
  double s, m1, m2, z2;
};
__device__ __forceinline__ Lens make_lens(double s, double q) {
  double r = 1.0 / (1.0 + q);
  return Lens{s, r, q * r, s * r};
}

// Sec. 2.2, Eq. method-transformed: the cancellation-free coefficients of
// sum_i c_i eta^i = 0, with v_c = conj(y) + s, v_p = 1 + s conj(y).
// Each coefficient is a sum of terms of the same order in q, so none of the
// subtractions of the conventional form appears.
__device__ __forceinline__ void coefficients(const Lens& L, c64 y, c64 c[6]) {
  const double s = L.s, m2 = L.m2, ms = m2 * s;
  const c64 yb = cconj(y);
  const c64 iy = cz(0.0, y.y);
  const c64 vc = yb + s;
  const c64 vp = cz(1.0 + s * y.x, -s * y.y);
  const double revp = 1.0 + s * y.x, revc = y.x + s, re1sy = 1.0 - s * y.x;
  c[5] = -(yb * vc);
  c[4] = ((yb * y) - 1.0 - 2.0 * s * yb) * vc + ms;
  c[3] = (2.0 * y - s) * ((vp * vc) + 2.0 * iy - ms) + (4.0 * (cz(ms, 0.0) - y)) * iy;
  c[2] = cz(revp * revp * revc, y.y * revp * re1sy) + (s * y.y * y.y) * ((s * vc) + 2.0) +
         ms * (2.0 * (yb * (y - s)) - cz(1.0 - s * y.x, -s * y.y));
  c[1] = ms * (((2.0 * y) + s) * vp + s * cz(-m2, 2.0 * s * y.y));
  c[0] = (s * s * m2 * m2) * y;
}

// Comparator only: the conventional coefficients of Sec. 2.2, Eq.
// lens-poly-orig (the printed symbol `a` of c3 reads -s, the position of
// lens 1 in this frame).  c3 and c2 add terms of order 1 and of order q
// that cancel against each other for small q, which costs the digits the
// refined form keeps (Fig. 1).  Used by the comparator mode and by
// twk_coefficients; never by the method's path.
__device__ __forceinline__ void coefficients_conventional(const Lens& L, c64 y, c64 c[6]) {
  const double s = L.s, m1 = L.m1, m2 = L.m2, s2 = s * s, s3 = s2 * s;
  const c64 yb = cconj(y);
  const c64 u = yb * (y - 2.0 * s);  // conj(y) (y - 2 s)
  c[5] = -(yb * (yb + s));
  c[4] = yb * (u - 1.0) + s * (u - m1);
  c[3] = 2.0 * (yb * y) - s3 * yb + s2 * (yb * (2.0 * y - yb) - m1) +
         s * (y + 2.0 * (yb * ((yb * y) - m2)));
  c[2] = y * (s3 * yb + 1.0) + s * (2.0 * (1.0 + m2) * (y * yb) + m1) +
         s2 * ((m1 - m2) * yb + y * (yb * yb + (1.0 + m2)));
  c[1] = (m2 * s) * (s * (y * (2.0 * yb + s) + m1) + 2.0 * y);
  c[0] = (s2 * m2 * m2) * y;
}

// ---------------------------------------------------------------- roots
// All five roots by the Aberth-Ehrlich simultaneous iteration (each root is
// corrected by Newton's ratio deflated against the others), updating in
// place (Gauss-Seidel order).  Warm starts come from a neighbouring limb
// sample, cold starts from a circle.  The paper delegates this step to the
// Skowron & Gould solver; any all-roots method of full precision serves.
__device__ __forceinline__ void horner64(const c64 c[6], c64 x, c64& p, c64& d) {
  d = c[5];
  p = cfma(c[5], x, c[4]);
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    d = cfma(d, x, p);
    p = cfma(p, x, c[k]);
  }
}

__device__ __forceinline__ void cold_start(const c64 c[6], c64 r[5]) {
  // circle of radius |c0/c5|^(1/5) (geometric mean of the root moduli)
  double rad = pow(sqrt(cnorm(c[0]) / cnorm(c[5])), 0.2);
  if (!(rad > 0.0) || !(rad < 1e30)) rad = 1.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double a = 1.2566370614359172 * k + 0.7;
    r[k] = cz(rad * cos(a), rad * sin(a));
  }
}

// Stopping rule shared by both precisions.  A sweep's largest relative
// correction d bounds the error before the sweep; Aberth converges cubically
// for simple roots, the error after the sweep being about 4 d^3 / sigma^2
// for a relative separation sigma of the nearest two roots (linear
// convergence once the error exceeds sigma).  Stop when d < 1e-14; or when
// d < 1e-6 and no two roots lie within 1e-3 (relative) of each other; or when
// d < 1e-5 and none lie within 0.05 (error after the sweep below 2e-12 of the
// root; the lens-equation polish that follows takes real images to full
// precision).  Returns the number of sweeps used (maxit + 1 when not
// converged).
__device__ inline int aberth64(const c64 c[6], c64 r[5], int maxit) {
  for (int it = 0; it < maxit; ++it) {
    double worst = 0.0;
    bool close = false;  // some root within 1e-3 (relative) of another
    bool near = false;   // some root within 0.05 (relative) of another
    // Gauss-Seidel order: root 0 is corrected against roots 1..4, then the
    // roots rotate by one place; after five steps the order is restored.
    // Only static register indices appear.
#pragma unroll 1
    for (int k = 0; k < 5; ++k) {
      const c64 x = r[0];
      c64 p, d;
      horner64(c, x, p, d);
      c64 rep = cz(0.0, 0.0);
      double n2min = 1e300;
#pragma unroll
      for (int j = 1; j < 5; ++j) {
        const c64 dd = x - r[j];
        const double n2 = cnorm(dd);
        n2min = fmin(n2min, n2);
        const double ir = rcp64(n2);
        rep = rep + cz(dd.x * ir, -dd.y * ir);
      }
      const double x2 = fmax(cnorm(x), 1e-300);
      close = close || n2min <= 1e-6 * x2;
      near = near || n2min <= 2.5e-3 * x2;
      // Newton's ratio deflated against the other roots, in one division
      c64 w = p * cinv(cfma(-p, rep, d));
      double nw = cnorm(w);
      if (!(nw < 1e300)) {  // vanishing derivative or coincident iterates
        const double a = 1.0 + fabs(x.x) + fabs(x.y);  // step scale ~ 1 + |x|
        w = cz(-1e-3 * a, 7e-4 * a);
        nw = 1.0;
        worst = 1.0;
      }
      const c64 xn = x - w;
      // relative size of the correction; only its order of magnitude matters
      worst = fmax(worst, nw * __builtin_amdgcn_rcp(fmax(cnorm(xn), 1e-300)));
      r[0] = r[1];
      r[1] = r[2];
      r[2] = r[3];
      r[3] = r[4];
      r[4] = xn;
    }
    if (worst < 1e-28 || (worst < 1e-12 && !close) || (worst < 1e-10 && !near)) return it + 1;
  }
  return maxit + 1;
}

// Mixed precision: the bulk sweeps in FP32 (polynomial scaled by 1/c5 so
// that FP32 keeps its range) from a start given in FP64; the caller then
// polishes with FP64 sweeps.  FP32 stops at a relative correction below
// 0.03: by cubic convergence the roots are then within about 1e-5 of the
// root (FP32's rounding level when the correction was much smaller), which
// one FP64 sweep takes to full precision for separated roots (the FP64 stop
// rule decides).  Stopping there rather than at 1e-3 saves the second FP32
// sweep of limb points started far from their roots (the first round of a
// source starts from the roots at its centre).  A lane that has not
// got there within the sweep cap (near-double roots converge linearly and
// FP32 rounding stalls them) hands over to the FP64 sweeps, which cost the
// same on a VALU without packed FP32 and can finish the job; the cap keeps
// one such lane from holding the wave in FP32.
__device__ inline int aberth32(const c64 c64c[6], c64 r64[5], int maxit) {
  const c64 inv5 = cinv(c64c[5]);
  c32 c[6], r[5];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const c64 t = c64c[k] * inv5;
    c[k] = c32{(float)t.x, (float)t.y};
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) r[k] = c32{(float)r64[k].x, (float)r64[k].y};
  int it = 0;
  for (; it < maxit; ++it) {
    float worst = 0.f;
    // Gauss-Seidel order as in the FP64 sweep (root k against roots k+1
    // .. 4, then 0 .. k-1), written out for each k with static register
    // indices instead of rotating the roots: the rotation's register
    // moves cost 1.3 % of a limb-darkened batch call.  (The FP64 sweep
    // keeps the rotation: unrolled, it lengthened the point-source pass
    // and raised the contour kernel's register spills.)
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const c32 x = r[k];
      c32 d = c[5], p = cfma(c[5], x, c[4]);
#pragma unroll
      for (int j = 3; j >= 0; --j) {
        d = cfma(d, x, p);
        p = cfma(p, x, c[j]);
      }
      c32 rep = c32{0.f, 0.f};
#pragma unroll
      for (int jj = 1; jj < 5; ++jj) rep = rep + cinv(x - r[(k + jj) % 5]);
      c32 w = p * cinv(cfma(c32{-p.x, -p.y}, rep, d));
      float nw = cnorm(w);
      if (!(nw < 1e30f)) {
        w = c32{1e-3f, -7e-4f};
        nw = 1.f;
        worst = 1.f;
      }
      const c32 xn = x - w;
      worst = fmaxf(worst, nw * __builtin_amdgcn_rcpf(fmaxf(cnorm(xn), 1e-30f)));
      r[k] = xn;
    }
    if (worst < 1e-3f) {
      ++it;
      break;
    }
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) r64[k] = cz((double)r[k].x, (double)r[k].y);
  return it;
}

// ---------------------------------------------------------------- images
// Residual of a root (Sec. 2.4.1) in the lens-2 frame:
//   R = y - eta + m1/(conj(eta) + s) + m2/conj(eta).
// f(z) = m1/(z1-z) + m2/(z2-z) (Eq. jacobian): in this frame
//   f'  = m1/(eta+s)^2 + m2/eta^2,  f'' = -2 m1/(eta+s)^3 - 2 m2/eta^3.
struct Images {
  c64 z[5];      // positive-parity real images, negative ones, then the ghost pair
  double J[5];
  int n;         // 3 or 5
  uint32_t par;  // bit k set: image k has positive parity (the first ones)
  uint32_t flags;
  double margin; // second-largest |R| over the noise level
};

enum : uint32_t {
  F_POINT = 1u << 0,
  F_CAP = 1u << 1,
  F_ANOMALY = 1u << 2,
  F_SLOPE = 1u << 3,
  F_NONFINITE = 1u << 4,
  F_NEARDEGEN = 1u << 5,
};

__device__ __forceinline__ c64 residual(const Lens& L, c64 y, c64 eta) {
  const c64 eb = cconj(eta);
  return y - eta + L.m1 * cinv(eb + L.s) + L.m2 * cinv(eb);
}

// Polish: near the critical curve a real image is a near-double root of the
// quintic, and the polynomial solve leaves it with an error far above
// rounding, correlated within the pair, so that the pair's residuals can
// mimic a ghost pair.  Real images solve the lens equation itself: each
// root gets one Newton step on it, dz = (R - conj(f') conj(R)) / J, kept
// only when the step is tiny against the distance to the nearer lens
// (<= 1e-8 min(|eta|, |eta + s|)) and at least halves |R|; a ghost has no
// nearby solution and its step is refused.  A step below 1e-15 of that
// distance is rounding noise and is not taken (the root is already
// converged).  On return R holds the residual of each (possibly polished)
// root.
// The residual, f' and J of a point all follow from the two inverses
// 1/(eta + s) and 1/eta (1/conj(x) = conj(1/x)); on return J[k] is the
// Jacobian at the final root.
struct LensPoint {
  c64 R, fp;
  double J;
};
__device__ __forceinline__ LensPoint lens_point(const Lens& L, c64 y, c64 e) {
  const c64 ia1 = cinv(e + L.s), ie = cinv(e);
  LensPoint o;
  o.R = y - e + L.m1 * cconj(ia1) + L.m2 * cconj(ie);
  o.fp = L.m1 * (ia1 * ia1) + L.m2 * (ie * ie);
  o.J = 1.0 - cnorm(o.fp);
  return o;
}

__device__ inline void polish_lens(const Lens& L, c64 y, c64 r[5], c64 R[5], double J[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const c64 e = r[k];
    const LensPoint p = lens_point(L, y, e);
    const c64 dz = rcp64(p.J) * (p.R - cconj(p.fp) * cconj(p.R));
    const double scale = fmin(cnorm(e), cnorm(e + L.s));
    R[k] = p.R;
    J[k] = p.J;
    // a step worth taking: beyond the root's rounding, tiny against the
    // distances to the lenses (a ghost's step is large)
    const double d2 = cnorm(dz);
    if (d2 <= 1e-16 * scale && d2 > 1e-30 * scale) {
      const c64 cand = e + dz;
      const LensPoint pc = lens_point(L, y, cand);
      if (cnorm(pc.R) < 0.25 * cnorm(p.R)) {
        r[k] = cand;
        R[k] = pc.R;
        J[k] = pc.J;
      }
    }
  }
}

// Residual detector.  The five residuals sum to zero (Eqs. sum_r, sum_r2),
// so a ghost pair shows as two residuals of equal length and opposite
// direction standing far above the numerical noise of the solve.  Noise:
// the largest of the third-largest |R|, the computed |sum R| (zero in exact
// arithmetic, so it measures this solve's rounding, coefficients included)
// and the rounding scale sigma = 64 eps (|y| + |eta| + m1/|eta+s| + m2/|eta|)
// of the three other roots.  Ghosts: the second largest |R| exceeds KGAP
// times the noise.  A margin within a factor 30 of KGAP is flagged
// near-degenerate; a ghost pair of unequal length is flagged anomalous.
#ifndef TWK_KGAP
#define TWK_KGAP 100.0  // a test build may blind the detector with a huge value
#endif
constexpr double KGAP = TWK_KGAP;
constexpr double EPS64 = 2.220446049250313e-16;

// sqrt to FP32 precision (the hardware square root, about 1 ulp), for the
// rounding scale of the noise level only (whose reciprocals are the
// hardware estimate too)
__device__ __forceinline__ double sqrt_rough(double x) {
  return (double)__builtin_amdgcn_sqrtf((float)x);
}

__device__ inline void classify(const Lens& L, c64 y, const c64 r[5], const c64 R[5],
                                const double J[5], Images& im) {
  // squared residual lengths rank the roots; lengths are taken only where
  // a value is needed (the two largest and the noise level)
  double aR2[5], sg[5];
  const double ay = sqrt_rough(cnorm(y));
  c64 Rs = cz(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    aR2[k] = cnorm(R[k]);
    Rs = Rs + R[k];
    const double ae2 = cnorm(r[k]), as2 = cnorm(r[k] + L.s);
    sg[k] = 64.0 * EPS64 *
            (ay + sqrt_rough(ae2) + L.m1 * sqrt_rough(__builtin_amdgcn_rcp(as2)) +
             L.m2 * sqrt_rough(__builtin_amdgcn_rcp(ae2)));
  }
  // the two largest residuals (first index wins ties)
  int a = 0;
#pragma unroll
  for (int k = 1; k < 5; ++k)
    if (aR2[k] > aR2[a]) a = k;
  int b = a == 0 ? 1 : 0;
#pragma unroll
  for (int k = 0; k < 5; ++k)
    if (k != a && aR2[k] > aR2[b]) b = k;
  double noise2 = cnorm(Rs), ra2 = 0.0, rb2 = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (k != a && k != b) noise2 = fmax(noise2, fmax(aR2[k], sg[k] * sg[k]));
    if (k == a) ra2 = aR2[k];
    if (k == b) rb2 = aR2[k];
  }
  const double ra = sqrt_fast(ra2), rb = sqrt_fast(rb2);
  const double margin = rb * rcp64(sqrt_fast(noise2));
  const bool ghosts = margin > KGAP;
  im.margin = margin;
  im.flags = 0;
  if (margin > KGAP / 30.0 && margin < KGAP * 30.0) im.flags |= F_NEARDEGEN;
  if (ghosts && fabs(ra - rb) > 0.1 * ra) im.flags |= F_ANOMALY;
  // Parity: the parity sum of the real images is -1 (Sec. 2.3), one
  // positive image of three, two of five; the positive ones are the
  // (n - 1)/2 real images of largest J.  That is sign(J) whenever sign(J)
  // obeys the sum; where it does not, the pair merging on the critical curve
  // has |J| below the rounding of its near-double root and the rank gives
  // the pair one image of each parity (flagged near-degenerate).
  // Order the roots: positive-parity real images, negative-parity real
  // images, ghosts (stable bubble sort on a 0/1/2 key; static indices).
  const int nreal = ghosts ? 3 : 5, npos_want = ghosts ? 1 : 2;
  int key[5], nsign = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    im.J[k] = J[k];
    im.z[k] = r[k];
    const bool g = ghosts && (k == a || k == b);
    int above = 0;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const bool gm = ghosts && (m == a || m == b);
      if (m != k && !gm && (J[m] > J[k] || (J[m] == J[k] && m < k))) ++above;
    }
    key[k] = g ? 2 : (above < npos_want ? 0 : 1);
    if (!g && J[k] > 0.0) ++nsign;
  }
  if (nsign != npos_want) im.flags |= F_NEARDEGEN;
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
#pragma unroll
    for (int i = 0; i < 4 - pass; ++i) {
      const bool sw = key[i] > key[i + 1];
      const c64 z0 = im.z[i], z1 = im.z[i + 1];
      const double j0 = im.J[i], j1 = im.J[i + 1];
      const int k0 = key[i], k1 = key[i + 1];
      im.z[i] = sw ? z1 : z0;
      im.z[i + 1] = sw ? z0 : z1;
      im.J[i] = sw ? j1 : j0;
      im.J[i + 1] = sw ? j0 : j1;
      key[i] = sw ? k1 : k0;
      key[i + 1] = sw ? k0 : k1;
    }
  }
  im.n = nreal;
  im.par = (1u << npos_want) - 1u;
}

// Roots -> polished roots, residuals and classification.
__device__ inline void finish_images(const Lens& L, c64 y, c64 r[5], Images& im) {
  c64 R[5];
  double J[5];
  polish_lens(L, y, r, R, J);
  classify(L, y, r, R, J, im);
}

// Comparator only: the classification of older codes.  A root is a real
// image when its lens-equation residual is below a fixed absolute
// threshold (LEGACY_THR, in Einstein radii), no lens-equation polish, and
// parity is sign(J).  Five real images when the five residuals are all
// below the threshold, otherwise the three smallest; a parity sum other
// than -1 is flagged anomalous.
constexpr double LEGACY_THR = 1e-6;
__device__ inline void finish_images_legacy(const Lens& L, c64 y, const c64 r[5], Images& im) {
  double aR2[5], J[5];
  int nbelow = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const LensPoint p = lens_point(L, y, r[k]);
    aR2[k] = cnorm(p.R);
    J[k] = p.J;
    nbelow += aR2[k] < LEGACY_THR * LEGACY_THR ? 1 : 0;
  }
  // the two largest residuals are the ghosts unless all five are below
  int a = 0;
#pragma unroll
  for (int k = 1; k < 5; ++k)
    if (aR2[k] > aR2[a]) a = k;
  int b = a == 0 ? 1 : 0;
#pragma unroll
  for (int k = 0; k < 5; ++k)
    if (k != a && aR2[k] > aR2[b]) b = k;
  const bool ghosts = nbelow < 5;
  int key[5], npos = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    im.J[k] = J[k];
    im.z[k] = r[k];
    const bool g = ghosts && (k == a || k == b);
    key[k] = g ? 2 : (J[k] > 0.0 ? 0 : 1);
    npos += key[k] == 0 ? 1 : 0;
  }
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
#pragma unroll
    for (int i = 0; i < 4 - pass; ++i) {
      const bool sw = key[i] > key[i + 1];
      const c64 z0 = im.z[i], z1 = im.z[i + 1];
      const double j0 = im.J[i], j1 = im.J[i + 1];
      const int k0 = key[i], k1 = key[i + 1];
      im.z[i] = sw ? z1 : z0;
      im.z[i + 1] = sw ? z0 : z1;
      im.J[i] = sw ? j1 : j0;
      im.J[i + 1] = sw ? j0 : j1;
      key[i] = sw ? k1 : k0;
      key[i + 1] = sw ? k0 : k1;
    }
  }
  im.n = ghosts ? 3 : 5;
  im.par = (1u << npos) - 1u;
  im.margin = 0.0;
  im.flags = (2 * npos - im.n != -1) ? F_ANOMALY : 0u;
}

__device__ __forceinline__ double point_mag(const Images& im) {
  double mu = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k)
    if (k < im.n) mu += 1.0 / fabs(im.J[k]);
  return mu;
}

// Full FP64 point solve from a cold start.
__device__ inline void solve_point_cold(const Lens& L, c64 y, Images& im, int& iters) {
  c64 c[6], r[5];
  coefficients(L, y, c);
  cold_start(c, r);
  iters = aberth64(c, r, 200);
  finish_images(L, y, r, im);
}

// Limb derivatives (Sec. 2.3, Eq. area_cal) for a real image at eta, with
// zeta' = i rho e^{i theta}:
//   z'      = (zeta' - conj(f') conj(zeta')) / J
//   z' ^ z'' = (rho^2 + Im(z'^2 zeta' f'')) / J
__device__ __forceinline__ void limb_derivs(const Lens& L, c64 eta, double J, c64 zp1, double rho,
                                            c64& dz, double& w) {
  c64 a1 = eta + L.s;
  c64 ia1 = cinv(a1), ie = cinv(eta);
  c64 ia2 = ia1 * ia1, ie2 = ie * ie;
  c64 fp = L.m1 * ia2 + L.m2 * ie2;
  c64 fpp = -2.0 * (L.m1 * (ia2 * ia1) + L.m2 * (ie2 * ie));
  const double iJ = rcp64(J);
  dz = iJ * (zp1 - cconj(fp) * cconj(zp1));
  w = iJ * (rho * rho + ((dz * dz) * zp1 * fpp).y);
}

}  // namespace twk
