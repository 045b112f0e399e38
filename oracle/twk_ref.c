/*
 * twk_ref.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Slow, single-threaded, written to be checked by eye against the paper:
 *   Wang, Wang & Dong, "Twinkle: A GPU-based binary-lens microlensing code
 *   with contour integration method", arXiv 2501.03322.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code with the HIP path.
 *
 * Every floating-point quantity is IEEE binary64.  Build with
 * -ffp-contract=off so that no operation is fused behind the reader's back.
 *
 * Readings of passages that the paper leaves ambiguous or garbled are marked
 * "READING" below; each one is listed with its justification in the design
 * notes of the repository.
 *
 * Parity pins (what fixes each part independently of this code) live in the
 * test suite: symbolic re-derivation of the quintic, LAPACK companion roots,
 * the zero residual-sum identity, the Paczynski and Witt-Mao closed forms,
 * finite differences of the limb derivatives, and inverse ray shooting.
 */
#include "twk_ref.h"

#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define PI_D 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Lens set-up: Sec. 2.1 (lens equation and binary positions).          */
/* ------------------------------------------------------------------ */
typedef struct {
  double s, q;
  double m1, m2; /* masses normalised by the total mass            */
  double z1, z2; /* lens positions on the real axis, CM frame       */
} lens_t;

static lens_t lens_make(double s, double q) {
  lens_t L;
  L.s = s;
  L.q = q;
  L.m1 = 1.0 / (1.0 + q);
  L.m2 = q / (1.0 + q);
  L.z1 = -q * s / (1.0 + q);
  L.z2 = s / (1.0 + q);
  return L;
}

static int lens_ok(double s, double q) {
  return isfinite(s) && isfinite(q) && s > 0.0 && q > 0.0;
}

/* ------------------------------------------------------------------ */
/* Coefficients: Sec. 2.2, Eq. method-transformed (refined form).       */
/* y = zeta - z2 is the source in the lens-2 frame; lens 1 is at -s.    */
/* "Im(y) i" is the purely imaginary number i*Im(y); Re(.) of v_p, v_c  */
/* and 1 - s y are real parts.                                           */
/* ------------------------------------------------------------------ */
static void coeffs_refined(const lens_t *L, cplx y, cplx c[6]) {
  const double s = L->s, m2 = L->m2;
  const cplx yb = conj(y);
  const double yr = creal(y), yi = cimag(y);
  const cplx iy = CMPLX(0.0, yi);   /* Im(y) i           */
  const cplx vc = yb + s;           /* v_c = conj(y) + s */
  const cplx vp = 1.0 + s * yb;     /* v_p = 1 + s conj(y) */
  const double re_vp = 1.0 + s * yr;
  const double re_vc = yr + s;
  const double re_1sy = 1.0 - s * yr;

  c[5] = -yb * vc;
  c[4] = (yb * y - 1.0 - 2.0 * s * yb) * vc + m2 * s;
  c[3] = (2.0 * y - s) * (vp * vc + 2.0 * iy - m2 * s) + 4.0 * (m2 * s - y) * iy;
  c[2] = re_vp * re_vp * re_vc + CMPLX(0.0, yi * re_vp * re_1sy) +
         s * yi * yi * (2.0 + s * vc) +
         m2 * s * (2.0 * yb * (y - s) - (1.0 - s * y));
  c[1] = m2 * s * ((s + 2.0 * y) * vp + s * (2.0 * s * iy - m2));
  c[0] = s * s * m2 * m2 * y;
}

/* Conventional form, Sec. 2.2 Eq. lens-poly-orig.  READING: the symbol `a`
 * printed in c3 stands for -s (symbolic re-derivation of the quintic). */
static void coeffs_conventional(const lens_t *L, cplx y, cplx c[6]) {
  const double s = L->s, m1 = L->m1, m2 = L->m2;
  const cplx yb = conj(y);
  const double a = -s;
  c[5] = -yb * (yb + s);
  c[4] = yb * (yb * (-2.0 * s + y) - 1.0) + s * (yb * (-2.0 * s + y) - m1);
  c[3] = 2.0 * yb * y - s * s * s * yb + s * s * (yb * (2.0 * y - yb) - m1) -
         a * (y + 2.0 * yb * (yb * y - m2));
  c[2] = y * (1.0 + s * s * s * yb) + s * (m1 + 2.0 * y * yb * (1.0 + m2)) +
         s * s * (yb * (m1 - m2) + y * (1.0 + m2 + yb * yb));
  c[1] = m2 * s * (s * (m1 + y * (2.0 * yb + s)) + 2.0 * y);
  c[0] = s * s * m2 * m2 * y;
}

/* ------------------------------------------------------------------ */
/* Roots: the paper uses Skowron & Gould (2012); any method that finds   */
/* all five roots to working precision serves.  The oracle uses the      */
/* Aberth-Ehrlich simultaneous iteration from a cold start on a circle,  */
/* followed by Newton steps on the undeflated polynomial.                */
/* ------------------------------------------------------------------ */
static void horner2(const cplx c[6], cplx x, cplx *p, cplx *dp) {
  cplx b = c[5], d = 0.0;
  for (int k = 4; k >= 0; --k) {
    d = d * x + b;
    b = b * x + c[k];
  }
  *p = b;
  *dp = d;
}

static int roots5(const cplx c[6], cplx r[5]) {
  /* Fujiwara's bound on the root moduli, and the geometric mean of the
   * moduli |c0/c5|^(1/5): start on a circle of the latter radius (clamped
   * into the bound), which keeps the cold start near the roots. */
  if (c[5] == 0.0) {
    for (int k = 0; k < 5; ++k) r[k] = CMPLX(NAN, NAN);
    return 0;
  }
  double bound = 0.0;
  for (int k = 1; k <= 5; ++k) {
    double a = cabs(c[5 - k] / c[5]);
    if (k == 5) a *= 0.5;
    double t = pow(a, 1.0 / k);
    if (t > bound) bound = t;
  }
  bound *= 2.0;
  double rad = pow(cabs(c[0] / c[5]), 0.2);
  if (!(rad > 0.0) || rad > bound) rad = 0.5 * bound;
  for (int k = 0; k < 5; ++k) {
    double ang = 2.0 * PI_D * k / 5.0 + 0.4;
    r[k] = rad * CMPLX(cos(ang), sin(ang));
  }
  int it;
  int settled = 0;
  for (it = 1; it <= 500; ++it) {
    double worst = 0.0;
    for (int k = 0; k < 5; ++k) {
      cplx p, dp;
      horner2(c, r[k], &p, &dp);
      if (p == 0.0) continue;
      cplx ratio = p / dp;
      cplx rep = 0.0;
      for (int j = 0; j < 5; ++j)
        if (j != k) rep += 1.0 / (r[k] - r[j]);
      cplx w = ratio / (1.0 - ratio * rep);
      if (!isfinite(creal(w)) || !isfinite(cimag(w))) {
        /* dp vanished or two iterates coincide: nudge and continue. */
        r[k] += 1e-3 * rad * CMPLX(0.6, 0.8);
        worst = 1.0;
        continue;
      }
      r[k] -= w;
      double rel = cabs(w) / fmax(cabs(r[k]), DBL_MIN);
      if (rel > worst) worst = rel;
    }
    if (worst < 4.0 * DBL_EPSILON) {
      if (++settled >= 2) break;
    } else {
      settled = 0;
    }
  }
  /* Newton polish on the full polynomial, kept only if |P| decreases. */
  for (int k = 0; k < 5; ++k) {
    for (int pass = 0; pass < 2; ++pass) {
      cplx p, dp;
      horner2(c, r[k], &p, &dp);
      if (p == 0.0 || dp == 0.0) break;
      cplx cand = r[k] - p / dp;
      cplx p2, dp2;
      horner2(c, cand, &p2, &dp2);
      if (cabs(p2) < cabs(p)) r[k] = cand;
      else break;
    }
  }
  return it;
}

/* ------------------------------------------------------------------ */
/* Image classification.                                                 */
/* Residual (Sec. 2.4.1): R = zeta - r + m1/(conj(r) - conj(z1))          */
/*                            + m2/(conj(r) - conj(z2)),                  */
/* in the lens-2 frame: R = y - eta + m1/(conj(eta) + s) + m2/conj(eta). */
/* Jacobian (Eq. jacobian): f(z) = m1/(z1-z) + m2/(z2-z), J = 1 - |f'|^2. */
/* ------------------------------------------------------------------ */
typedef struct {
  int n;            /* real images (3 or 5)                    */
  cplx z[5];        /* lens-2 frame; real images first, ghosts last */
  cplx R[5];        /* residuals in the same order              */
  double J[5];      /* Jacobians in the same order               */
  int par[5];       /* parity (+1, -1) of the real images          */
  double margin;    /* second-largest |R| over the noise level  */
  uint32_t flags;
} images_t;

static cplx residual(const lens_t *L, cplx y, cplx eta) {
  cplx eb = conj(eta);
  return y - eta + L->m1 / (eb + L->s) + L->m2 / eb;
}

static cplx fprime(const lens_t *L, cplx eta) {
  /* f'(z) = m1/(z1-z)^2 + m2/(z2-z)^2 ; z1-z = -(eta+s), z2-z = -eta */
  cplx a = eta + L->s;
  return L->m1 / (a * a) + L->m2 / (eta * eta);
}

static cplx fsecond(const lens_t *L, cplx eta) {
  /* f''(z) = 2 m1/(z1-z)^3 + 2 m2/(z2-z)^3 */
  cplx a = eta + L->s;
  return -2.0 * L->m1 / (a * a * a) - 2.0 * L->m2 / (eta * eta * eta);
}

/* READING of the residual detector (the paper states the principle only):
 * the five residuals sum to zero exactly, so a ghost pair shows as two
 * residuals of equal length, opposite direction, standing far above the
 * numerical noise of the solve.  The noise level is the largest of: the
 * third-largest |R|, the rounding scale sigma = 64 eps (|y| + |eta| +
 * m1/|eta+s| + m2/|eta|) of the three roots with the smallest residuals, and
 * the computed |sum R| (which vanishes in exact arithmetic, so its value
 * measures the rounding of this particular solve, coefficients included).
 * The two largest residuals are a ghost pair when the second largest
 * exceeds kgap times the noise; otherwise all five roots are real.  A
 * violation of equal length is flagged; a margin within a factor 30 of
 * kgap is flagged as near-degenerate. */
static void classify(const lens_t *L, cplx y, const cplx r[5], double kgap,
                     images_t *out) {
  cplx R[5];
  double aR[5], sig[5];
  int o[5];
  for (int k = 0; k < 5; ++k) {
    R[k] = residual(L, y, r[k]);
    aR[k] = cabs(R[k]);
    sig[k] = 64.0 * DBL_EPSILON *
             (cabs(y) + cabs(r[k]) + L->m1 / cabs(r[k] + L->s) +
              L->m2 / cabs(r[k]));
    o[k] = k;
  }
  /* insertion sort, decreasing |R|; ties keep root order */
  for (int i = 1; i < 5; ++i) {
    int t = o[i], j = i - 1;
    while (j >= 0 && aR[o[j]] < aR[t]) {
      o[j + 1] = o[j];
      --j;
    }
    o[j + 1] = t;
  }
  cplx Rsum = R[0] + R[1] + R[2] + R[3] + R[4];
  double noise = fmax(aR[o[2]], cabs(Rsum));
  for (int k = 2; k < 5; ++k)
    if (sig[o[k]] > noise) noise = sig[o[k]];
  double margin = aR[o[1]] / noise;
  int ghosts = margin > kgap;
  out->margin = margin;
  out->flags = 0;
  if (margin > kgap / 30.0 && margin < kgap * 30.0)
    out->flags |= TWK_REF_FLAG_NEARDEGEN;
  int order[5];
  int m = 0;
  if (ghosts) {
    if (fabs(aR[o[0]] - aR[o[1]]) > 0.1 * aR[o[0]])
      out->flags |= TWK_REF_FLAG_ANOMALY;
    for (int k = 0; k < 5; ++k)
      if (k != o[0] && k != o[1]) order[m++] = k;
    order[m++] = o[0];
    order[m++] = o[1];
    out->n = 3;
  } else {
    for (int k = 0; k < 5; ++k) order[m++] = k;
    out->n = 5;
  }
  for (int k = 0; k < 5; ++k) {
    int i = order[k];
    out->z[k] = r[i];
    out->R[k] = R[i];
    cplx fp = fprime(L, r[i]);
    out->J[k] = 1.0 - creal(fp * conj(fp));
  }
  /* Parity.  The parity sum of the real images is -1 (Sec. 2.3): one
   * positive image of three, two of five.  READING: the positive images
   * are the (n - 1)/2 real images of largest J.  This is sign(J) whenever
   * sign(J) obeys the sum; where it does not, an image of the pair that is
   * merging on the critical curve has |J| below the rounding of its
   * near-double root, and the rank assigns the pair one image of each
   * parity.  Such a correction is flagged near-degenerate. */
  int npos = (out->n - 1) / 2, nsign = 0;
  for (int k = 0; k < 5; ++k) {
    int above = 0;
    for (int m2 = 0; m2 < out->n; ++m2)
      if (out->J[m2] > out->J[k] || (out->J[m2] == out->J[k] && m2 < k)) ++above;
    out->par[k] = (k < out->n && above < npos) ? 1 : -1;
    if (k < out->n && out->J[k] > 0.0) ++nsign;
  }
  if (nsign != npos) out->flags |= TWK_REF_FLAG_NEARDEGEN;
}

/* Near the critical curve a real image is a near-double root of the
 * quintic and the polynomial solve leaves it with errors far above
 * rounding, correlated within the pair, so that the pair's residuals can
 * mimic a ghost pair.  Real images solve the lens equation itself, so each
 * root receives one Newton step on the lens equation (z' + conj(f')
 * conj(z') = -F gives dz = (R - conj(f') conj(R))/J), kept only when the
 * step is tiny (a root correction, <= 1e-8 (1 + |eta|)) and lowers |R|.
 * A ghost has no nearby solution: its step is large and is refused. */
static void polish_lens(const lens_t *L, cplx y, cplx r[5]) {
  for (int k = 0; k < 5; ++k) {
    cplx R = residual(L, y, r[k]);
    cplx fp = fprime(L, r[k]);
    double J = 1.0 - creal(fp * conj(fp));
    cplx dz = (R - conj(fp) * conj(R)) / J;
    double scale = fmin(cabs(r[k]), cabs(r[k] + L->s));
    if (!(cabs(dz) <= 1e-8 * scale)) continue;
    cplx cand = r[k] + dz;
    if (cabs(residual(L, y, cand)) < 0.5 * cabs(R)) r[k] = cand;
  }
}

static void solve_point(const lens_t *L, cplx y, double kgap, images_t *im) {
  cplx c[6], r[5];
  coeffs_refined(L, y, c);
  roots5(c, r);
  polish_lens(L, y, r);
  classify(L, y, r, kgap, im);
}

/* ------------------------------------------------------------------ */
/* Public: coefficients, roots, images, point magnification.             */
/* ------------------------------------------------------------------ */
int twk_ref_coeffs(double s, double q, double zx, double zy, double *out) {
  if (!lens_ok(s, q) || !out) return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  cplx c[6];
  coeffs_refined(&L, CMPLX(zx - L.z2, zy), c);
  for (int k = 0; k < 6; ++k) {
    out[2 * k] = creal(c[k]);
    out[2 * k + 1] = cimag(c[k]);
  }
  return TWK_REF_OK;
}

int twk_ref_coeffs_conventional(double s, double q, double zx, double zy,
                                double *out) {
  if (!lens_ok(s, q) || !out) return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  cplx c[6];
  coeffs_conventional(&L, CMPLX(zx - L.z2, zy), c);
  for (int k = 0; k < 6; ++k) {
    out[2 * k] = creal(c[k]);
    out[2 * k + 1] = cimag(c[k]);
  }
  return TWK_REF_OK;
}

int twk_ref_roots(const double *c12, double *roots10) {
  if (!c12 || !roots10) return TWK_REF_EINVAL;
  cplx c[6], r[5];
  for (int k = 0; k < 6; ++k) c[k] = CMPLX(c12[2 * k], c12[2 * k + 1]);
  if (c[5] == 0.0) return TWK_REF_EINVAL;
  int it = roots5(c, r);
  for (int k = 0; k < 5; ++k) {
    roots10[2 * k] = creal(r[k]);
    roots10[2 * k + 1] = cimag(r[k]);
  }
  return it;
}

int twk_ref_images(double s, double q, double zx, double zy, double *img10,
                   double *res10, double *jac5, int32_t *n_real,
                   uint32_t *flags) {
  if (!lens_ok(s, q) || !isfinite(zx) || !isfinite(zy)) return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  images_t im;
  solve_point(&L, CMPLX(zx - L.z2, zy), 100.0, &im);
  for (int k = 0; k < 5; ++k) {
    if (img10) {
      img10[2 * k] = creal(im.z[k]) + L.z2;
      img10[2 * k + 1] = cimag(im.z[k]);
    }
    if (res10) {
      res10[2 * k] = creal(im.R[k]);
      res10[2 * k + 1] = cimag(im.R[k]);
    }
    if (jac5) jac5[k] = im.J[k];
  }
  if (n_real) *n_real = im.n;
  if (flags) *flags = im.flags;
  return TWK_REF_OK;
}

static double mu_point(const images_t *im) {
  double mu = 0.0;
  for (int k = 0; k < im->n; ++k) mu += 1.0 / fabs(im->J[k]);
  return mu;
}

int twk_ref_point_mag(double s, double q, int64_t n, const double *zx,
                      const double *zy, double *mag, int32_t *n_images,
                      uint32_t *flags) {
  if (!lens_ok(s, q) || n < 0 || (n > 0 && (!zx || !zy || !mag)))
    return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  for (int64_t i = 0; i < n; ++i) {
    if (!isfinite(zx[i]) || !isfinite(zy[i])) {
      mag[i] = NAN;
      if (n_images) n_images[i] = 0;
      if (flags) flags[i] = TWK_REF_FLAG_NONFINITE;
      continue;
    }
    images_t im;
    solve_point(&L, CMPLX(zx[i] - L.z2, zy[i]), 100.0, &im);
    mag[i] = mu_point(&im);
    if (n_images) n_images[i] = im.n;
    if (flags) flags[i] = im.flags;
  }
  return TWK_REF_OK;
}

/* ------------------------------------------------------------------ */
/* Limb derivatives.  The source limb is zeta(theta) = zeta_c + rho      */
/* e^{i theta}, counter-clockwise from +x (Sec. 2.3).  The lens equation */
/* zeta = z + conj(f(z)) differentiated once gives                       */
/*   zeta' = z' + conj(f') conj(z'),                                     */
/* hence z' = (zeta' - conj(f') conj(zeta'))/J (READING of the printed    */
/* formula, which must carry conj(f')), and differentiated twice gives   */
/*   zeta'' = z'' + conj(f'' z'^2) + conj(f') conj(z''),                 */
/* which the oracle solves for z'' directly.  z' ^ z'' = Im(conj(z') z''). */
/* ------------------------------------------------------------------ */
typedef struct {
  double theta;
  images_t im;
  cplx dz[5];   /* z' of the real images          */
  double w[5];  /* z' ^ z'' of the real images    */
  int n_eff;    /* real images after the slope detector */
  int demote[2];/* indices of a pair demoted to ghosts, or -1 */
} sample_t;

static void limb_derivs(const lens_t *L, double rho, double theta,
                        sample_t *sm) {
  cplx e = CMPLX(cos(theta), sin(theta));
  cplx zp = CMPLX(0.0, rho) * e; /* zeta'  = i rho e^{i theta} */
  cplx zpp = -rho * e;           /* zeta'' = -rho e^{i theta}  */
  for (int k = 0; k < sm->im.n; ++k) {
    cplx eta = sm->im.z[k];
    cplx fp = fprime(L, eta), fpp = fsecond(L, eta);
    double J = sm->im.J[k];
    cplx d1 = (zp - conj(fp) * conj(zp)) / J;
    cplx g = zpp - conj(fpp * d1 * d1);
    cplx d2 = (g - conj(fp) * conj(g)) / J;
    sm->dz[k] = d1;
    sm->w[k] = cimag(conj(d1) * d2);
  }
}

int twk_ref_limb_derivs(double s, double q, double zcx, double zcy,
                        double rho, double theta, double *img10,
                        double *dz10, double *wedge5, int32_t *n_real) {
  if (!lens_ok(s, q) || !(rho > 0.0)) return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  sample_t sm;
  cplx y = CMPLX(zcx - L.z2, zcy) + rho * CMPLX(cos(theta), sin(theta));
  solve_point(&L, y, 100.0, &sm.im);
  limb_derivs(&L, rho, theta, &sm);
  for (int k = 0; k < 5; ++k) {
    if (img10) {
      img10[2 * k] = creal(sm.im.z[k]) + L.z2;
      img10[2 * k + 1] = cimag(sm.im.z[k]);
    }
    if (dz10) {
      dz10[2 * k] = k < sm.im.n ? creal(sm.dz[k]) : 0.0;
      dz10[2 * k + 1] = k < sm.im.n ? cimag(sm.dz[k]) : 0.0;
    }
    if (wedge5) wedge5[k] = k < sm.im.n ? sm.w[k] : 0.0;
  }
  if (n_real) *n_real = sm.im.n;
  return TWK_REF_OK;
}

/* ------------------------------------------------------------------ */
/* Linking of adjacent samples (Sec. 2.3).                               */
/* Same-parity images of adjacent samples are linked by the assignment   */
/* with the least total distance.  When the counts differ, one positive  */
/* and one negative image of the sample with more images are left over:  */
/* that pair is created (or destroyed) on the critical curve and is      */
/* joined to itself.                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
  int na, nb;        /* real images at each end (after slope detector)  */
  int nlink;
  int la[5], lb[5];  /* linked image indices at a and b                 */
  int par[5];        /* parity of each link                             */
  int kind;          /* 0 none, +1 pair created at b, -1 destroyed at a */
  int cp, cn;        /* indices of the + and - image of that pair        */
  int anomaly;
} links_t;

/* effective real-image list of a sample (slope detector applied) */
static int eff_list(const sample_t *sm, int idx[5]) {
  int m = 0;
  for (int k = 0; k < sm->im.n; ++k) {
    if (k == sm->demote[0] || k == sm->demote[1]) continue;
    idx[m++] = k;
  }
  return m;
}

/* Least total distance injection of the smaller list into the larger.
 * Enumeration order: lexicographic over ordered choices; first minimum
 * wins on ties. */
static void assign(const cplx *za, const int *ia, int na, const cplx *zb,
                   const int *ib, int nb, int *ma, int *mb, int *nm) {
  if (na == 0 || nb == 0) {
    *nm = 0;
    return;
  }
  /* swap so that a is the smaller side */
  int swapped = 0;
  if (na > nb) {
    const cplx *tz = za; za = zb; zb = tz;
    const int *ti = ia; ia = ib; ib = ti;
    int t = na; na = nb; nb = t;
    swapped = 1;
  }
  double best = INFINITY;
  int bestp[3] = {0, 1, 2};
  int p[3];
  /* ordered choices of na distinct elements from nb (na <= 3, nb <= 3) */
  for (p[0] = 0; p[0] < nb; ++p[0]) {
    if (na == 1) {
      double d = cabs(za[ia[0]] - zb[ib[p[0]]]);
      if (d < best) { best = d; bestp[0] = p[0]; }
      continue;
    }
    for (p[1] = 0; p[1] < nb; ++p[1]) {
      if (p[1] == p[0]) continue;
      if (na == 2) {
        double d = cabs(za[ia[0]] - zb[ib[p[0]]]) + cabs(za[ia[1]] - zb[ib[p[1]]]);
        if (d < best) { best = d; bestp[0] = p[0]; bestp[1] = p[1]; }
        continue;
      }
      for (p[2] = 0; p[2] < nb; ++p[2]) {
        if (p[2] == p[0] || p[2] == p[1]) continue;
        double d = cabs(za[ia[0]] - zb[ib[p[0]]]) + cabs(za[ia[1]] - zb[ib[p[1]]]) +
                   cabs(za[ia[2]] - zb[ib[p[2]]]);
        if (d < best) { best = d; bestp[0] = p[0]; bestp[1] = p[1]; bestp[2] = p[2]; }
      }
    }
  }
  for (int k = 0; k < na; ++k) {
    int x = ia[k], yv = ib[bestp[k]];
    if (swapped) { ma[k] = yv; mb[k] = x; }
    else { ma[k] = x; mb[k] = yv; }
  }
  *nm = na;
}

static void link_samples(const sample_t *a, const sample_t *b, links_t *lk) {
  int ea[5], eb[5];
  int na = eff_list(a, ea), nb = eff_list(b, eb);
  int pa[5], npa = 0, ma_[5], nma = 0, pb[5], npb = 0, mb_[5], nmb = 0;
  for (int k = 0; k < na; ++k) {
    if (a->im.par[ea[k]] > 0) pa[npa++] = ea[k]; else ma_[nma++] = ea[k];
  }
  for (int k = 0; k < nb; ++k) {
    if (b->im.par[eb[k]] > 0) pb[npb++] = eb[k]; else mb_[nmb++] = eb[k];
  }
  lk->na = na;
  lk->nb = nb;
  lk->nlink = 0;
  lk->kind = 0;
  lk->cp = lk->cn = -1;
  lk->anomaly = 0;
  /* A binary lens has at most two positive and three negative real images
   * (parity sum -1, Sec. 2.3); more than three of one parity only arise
   * from a misjudged ghost pair.  Such an interval is anomalous and linked
   * no further. */
  if (npa > 3 || nma > 3 || npb > 3 || nmb > 3) {
    lk->anomaly = 1;
    return;
  }
  int xa[3], xb[3], nm;
  /* positive parity class */
  assign(a->im.z, pa, npa, b->im.z, pb, npb, xa, xb, &nm);
  for (int k = 0; k < nm; ++k) {
    lk->la[lk->nlink] = xa[k];
    lk->lb[lk->nlink] = xb[k];
    lk->par[lk->nlink] = 1;
    lk->nlink++;
  }
  int usedp_a[5] = {0}, usedp_b[5] = {0};
  for (int k = 0; k < nm; ++k) { usedp_a[xa[k]] = 1; usedp_b[xb[k]] = 1; }
  /* negative parity class */
  assign(a->im.z, ma_, nma, b->im.z, mb_, nmb, xa, xb, &nm);
  int usedn_a[5] = {0}, usedn_b[5] = {0};
  for (int k = 0; k < nm; ++k) {
    lk->la[lk->nlink] = xa[k];
    lk->lb[lk->nlink] = xb[k];
    lk->par[lk->nlink] = -1;
    lk->nlink++;
    usedn_a[xa[k]] = 1;
    usedn_b[xb[k]] = 1;
  }
  /* left-over images */
  int lpa = -1, lna = -1, lpb = -1, lnb = -1, cnt_a = 0, cnt_b = 0;
  for (int k = 0; k < npa; ++k) if (!usedp_a[pa[k]]) { lpa = pa[k]; cnt_a++; }
  for (int k = 0; k < nma; ++k) if (!usedn_a[ma_[k]]) { lna = ma_[k]; cnt_a++; }
  for (int k = 0; k < npb; ++k) if (!usedp_b[pb[k]]) { lpb = pb[k]; cnt_b++; }
  for (int k = 0; k < nmb; ++k) if (!usedn_b[mb_[k]]) { lnb = mb_[k]; cnt_b++; }
  if (cnt_a == 0 && cnt_b == 0) return;
  if (cnt_a == 0 && cnt_b == 2 && lpb >= 0 && lnb >= 0) {
    lk->kind = 1; lk->cp = lpb; lk->cn = lnb;
  } else if (cnt_b == 0 && cnt_a == 2 && lpa >= 0 && lna >= 0) {
    lk->kind = -1; lk->cp = lpa; lk->cn = lna;
  } else {
    lk->anomaly = 1;
  }
}

/* ------------------------------------------------------------------ */
/* Area and error of one interval (Sec. 2.3 Stokes area with trapezium  */
/* and parabolic corrections, Eq. area_cal and the cross-caustic form;  */
/* Sec. 2.5 errors, Eqs. area_normal and area_cross).                    */
/* Wedge a^b = Im(conj(a) b); dot a.b = Re(conj(a) b).                    */
/* Positive images run with theta, negative against it, so each linked   */
/* piece enters the area with the parity as sign.                        */
/* ------------------------------------------------------------------ */
static double wedge(cplx a, cplx b) { return cimag(conj(a) * b); }
static double dot(cplx a, cplx b) { return creal(conj(a) * b); }

typedef struct {
  double dA, E;
  int cross;
  int anomaly;
} piece_t;

/* The piece of a pair created (kind > 0, boundary from the - image to the
 * + image) or destroyed (kind < 0, from + to -) inside an interval of width
 * dth, from the pair's positions, limb derivatives and z' ^ z'' at the
 * sample where it exists: chord plus the cross-caustic correction
 * (Sec. 2.3) and errors E1 + E2 + E3 (Sec. 2.5, Eq. area_cross).  flip
 * (diagnostic only; 0 is the reading used): bit 0 negates the correction
 * of a created pair, bit 1 that of a destroyed pair.  *E2 receives E2. */
static void cross_piece(cplx zp, cplx zm, cplx dp, cplx dm, double wp,
                        double wm, int kind, double dth, int flip,
                        double *dA, double *E, double *E2out) {
  double dth2 = dth * dth;
  double dd = sqrt(fabs(dot(dp, dm)));
  double sep = cabs(zp - zm);
  double dtt = sep / dd;  /* effective step across the critical curve */
  double dtt3 = dtt * dtt * dtt;
  double dAp = (wp - wm) * dtt3 / 24.0;
  if ((kind > 0 && (flip & 1)) || (kind < 0 && (flip & 2))) dAp = -dAp;
  /* boundary runs from the - image to the + image where the pair is
   * created, and from + to - where it is destroyed */
  double chord = kind > 0 ? 0.5 * wedge(zm, zp) : 0.5 * wedge(zp, zm);
  *dA = chord + dAp;
  double E1 = fabs(wp + wm) * dtt3 / 48.0;
  /* READING of the garbled cross-caustic E2: "-" for a pair created
   * along +theta, "+" for a destroyed one. */
  double sgn = kind > 0 ? 1.0 : -1.0;
  double E2 = 1.5 * fabs(dot(zp - zm, dp - dm) - sgn * 2.0 * sep * dd) * dtt;
  double E3 = 0.1 * fabs(dAp) * dth2;
  *E = E1 + E2 + E3;
  *E2out = E2;
}

int twk_ref_cross_piece(const double *zp, const double *zm, const double *dp,
                        const double *dm, double wp, double wm, int32_t kind,
                        double dth, int32_t flip, double *dA, double *E,
                        double *E2) {
  if (!zp || !zm || !dp || !dm || !dA || !E || !E2 || kind == 0)
    return TWK_REF_EINVAL;
  cross_piece(CMPLX(zp[0], zp[1]), CMPLX(zm[0], zm[1]), CMPLX(dp[0], dp[1]),
              CMPLX(dm[0], dm[1]), wp, wm, kind, dth, flip, dA, E, E2);
  return TWK_REF_OK;
}

static piece_t interval_piece(const sample_t *a, const sample_t *b,
                              double dth, int flip) {
  links_t lk;
  link_samples(a, b, &lk);
  piece_t out = {0.0, 0.0, 0, lk.anomaly};
  double dth2 = dth * dth, dth3 = dth2 * dth;
  for (int k = 0; k < lk.nlink; ++k) {
    int i = lk.la[k], j = lk.lb[k];
    cplx za = a->im.z[i], zb = b->im.z[j];
    cplx da = a->dz[i], db = b->dz[j];
    double wa = a->w[i], wb = b->w[j];
    double p = (double)lk.par[k];
    double dAt = 0.5 * wedge(za, zb);
    double dAp1 = (wa + wb) * dth3 / 24.0;
    double dAp2 = wedge(zb - za, db - da) * dth / 12.0;
    double dAp = 0.5 * (dAp1 + dAp2);
    out.dA += p * (dAt + dAp);
    double E1 = fabs(wa - wb) * dth3 / 48.0;
    double ch = cabs(za - zb);
    double E2 = 1.5 * fabs(dAp * (ch * ch / (dth2 * fabs(dot(da, db))) - 1.0));
    double E3 = 0.1 * fabs(dAp) * dth2;
    double E4 = fabs(dAp1 - dAp2);
    out.E += E1 + E2 + E3 + E4;
  }
  if (lk.kind != 0) {
    /* the created pair lives at b, the destroyed pair at a */
    const sample_t *c = lk.kind > 0 ? b : a;
    double dA, E, E2;
    cross_piece(c->im.z[lk.cp], c->im.z[lk.cn], c->dz[lk.cp], c->dz[lk.cn],
                c->w[lk.cp], c->w[lk.cn], lk.kind, dth, flip, &dA, &E, &E2);
    out.dA += dA;
    out.E += E;
    out.cross = 1;
  }
  return out;
}

/* ------------------------------------------------------------------ */
/* Slope detector (Sec. 2.4.2).                                           */
/* The detector acts only near caustics, where a ghost pair may pass the  */
/* residual test as real.  READING: a 5-image sample is "suspect" when    */
/* the two largest residuals still stand above the noise by more than     */
/* SUSPECT (but below the gap factor); only suspect samples can be        */
/* reclassified.  At a change of the real-image count next to a suspect   */
/* 5-image sample, D is the difference (+ minus -) of the left-over pair  */
/* at that sample and G the ghost-pair difference at the 3-image sample.  */
/* The crossing is accepted when D and G are perpendicular enough,        */
/* |Re(conj(D) G)| <= cos(pi/4) |D| |G|.  Otherwise the pair is followed  */
/* into the 5-image run, demoting each suspect sample passed: the walk     */
/* stops at the first step whose consecutive pair differences are         */
/* perpendicular, or at the first non-suspect sample (the crossing lies    */
/* there).  When the whole run is walked, the run is deleted.              */
/* Pair differences below PAIR_FLOOR (1 + |z|) are below the resolution   */
/* of near-double roots in binary64; the direction test is meaningless    */
/* there and the crossing is accepted as found.                           */
/* ------------------------------------------------------------------ */
#define SUSPECT 8.0
#define PAIR_FLOOR 1e-7

static int perp_enough(cplx D, cplx G, cplx zref) {
  double floor_ = PAIR_FLOOR * (1.0 + cabs(zref));
  if (cabs(D) < floor_ || cabs(G) < floor_) return 1;
  return fabs(dot(D, G)) <= 0.70710678118654752440 * cabs(D) * cabs(G);
}

static int suspect(const sample_t *sm) { return sm->im.n == 5 && sm->im.margin > SUSPECT; }

static void reset_demotions(sample_t *sm, int nsm) {
  for (int i = 0; i < nsm; ++i) {
    sm[i].demote[0] = sm[i].demote[1] = -1;
    sm[i].n_eff = sm[i].im.n;
  }
}

/* follow the pair (cp, cn) of sample c0 to sample c1 through the 5<->5
 * links (full image sets); returns 0 if the pair is lost */
static int follow_pair(const sample_t *c0, const sample_t *c1, int *cp, int *cn) {
  sample_t t0 = *c0, t1 = *c1;
  t0.demote[0] = t0.demote[1] = t1.demote[0] = t1.demote[1] = -1;
  links_t l2;
  link_samples(&t0, &t1, &l2);
  int np = -1, nn = -1;
  for (int u = 0; u < l2.nlink; ++u) {
    if (l2.la[u] == *cp) np = l2.lb[u];
    if (l2.la[u] == *cn) nn = l2.lb[u];
  }
  if (np < 0 || nn < 0) return 0;
  *cp = np;
  *cn = nn;
  return 1;
}

/* Walk from the boundary sample b (3 images) into the run: positions of
 * the run are visited as run[0], run[step], ... (step = +1 entering at the
 * start, -1 entering at the end).  Returns the number of samples demoted. */
static int walk_run(sample_t *sm, const int *ord, int N, int kb, int first, int len,
                    int from_start) {
  int j0 = from_start ? 0 : len - 1;
  int dj = from_start ? 1 : -1;
  sample_t *b = &sm[ord[kb]];
  sample_t *c = &sm[ord[(first + j0) % N]];
  if (!suspect(c) || c->demote[0] >= 0) return 0;
  links_t lk;
  if (from_start) link_samples(b, c, &lk);
  else link_samples(c, b, &lk);
  int want = from_start ? 1 : -1;
  if (lk.kind != want) return 0;
  int cp = lk.cp, cn = lk.cn;
  cplx D = c->im.z[cp] - c->im.z[cn];
  cplx G = b->im.z[3] - b->im.z[4];
  if (perp_enough(D, G, c->im.z[cp])) return 0;
  int demoted = 0;
  for (int j = j0; j >= 0 && j < len; j += dj) {
    sample_t *cj = &sm[ord[(first + j) % N]];
    if (cj->demote[0] >= 0) break;
    cj->demote[0] = cp;
    cj->demote[1] = cn;
    cj->n_eff = 3;
    ++demoted;
    int jn = j + dj;
    if (jn < 0 || jn >= len) break; /* whole run walked: deleted */
    sample_t *cn1 = &sm[ord[(first + jn) % N]];
    if (!suspect(cn1)) break;
    int np = cp, nn = cn;
    if (!follow_pair(cj, cn1, &np, &nn)) break;
    cplx D1 = cn1->im.z[np] - cn1->im.z[nn];
    if (perp_enough(cj->im.z[cp] - cj->im.z[cn], D1, cj->im.z[cp])) break;
    cp = np;
    cn = nn;
  }
  return demoted;
}

/* ord: sorted sample indices, N of them (cyclic).  Returns the number of
 * reclassified samples. */
static int slope_detector(sample_t *sm, const int *ord, int N) {
  int changed = 0;
  int anchor = -1;
  for (int i = 0; i < N; ++i)
    if (sm[ord[i]].im.n == 3) { anchor = i; break; }
  if (anchor < 0) return 0;
  int i = 0;
  while (i < N) {
    if (sm[ord[(anchor + i) % N]].im.n != 5) { ++i; continue; }
    int start = i, len = 0;
    while (i < N && sm[ord[(anchor + i) % N]].im.n == 5) { ++len; ++i; }
    int k_in = (anchor + start - 1 + N) % N;
    int k_out = (anchor + start + len) % N;
    int first = (anchor + start) % N;
    changed += walk_run(sm, ord, N, k_in, first, len, 1);
    changed += walk_run(sm, ord, N, k_out, first, len, 0);
  }
  return changed;
}

/* ------------------------------------------------------------------ */
/* Contour integration with adaptive sampling (Secs. 2.3, 2.5, 3).        */
/*  - start from n0 uniform limb angles theta_j = 2 pi j / n0 (READING);  */
/*  - area A = sum of interval pieces, error E = sum of interval errors;  */
/*  - stop when E <= tol |A| (relative tolerance, READING);               */
/*  - otherwise weight each interval by max(E_i - tol|A|/N_int, 0)        */
/*    (tolerance subtraction), build the normalised cumulative weight,    */
/*    and invert it at quantiles (j + 1/2)/nnew by linear interpolation   */
/*    inside each interval (inverse transform sampling);                  */
/*  - the sample cap ends the refinement; mu and err are still returned.  */
/* ------------------------------------------------------------------ */
typedef struct {
  double sum, comp;
} nsum_t;

/* Neumaier's compensated summation */
static void nsum_add(nsum_t *s, double x) {
  double t = s->sum + x;
  if (fabs(s->sum) >= fabs(x)) s->comp += (s->sum - t) + x;
  else s->comp += (x - t) + s->sum;
  s->sum = t;
}

static void sample_at(const lens_t *L, cplx yc, double rho, double theta,
                      double kgap, sample_t *sm) {
  sm->theta = theta;
  cplx y = yc + rho * CMPLX(cos(theta), sin(theta));
  solve_point(L, y, kgap, &sm->im);
  limb_derivs(L, rho, theta, sm);
  sm->n_eff = sm->im.n;
  sm->demote[0] = sm->demote[1] = -1;
}

/* Narrowest interval of limb angle that is refined further. */
#define THETA_FLOOR 1e-9

void twk_ref_cfg_default(twk_ref_cfg *cfg, double tol) {
  cfg->tol = tol;
  cfg->n0 = 64;
  cfg->nnew = 64;
  cfg->cap = 4096;
  cfg->grow = 0;
  cfg->slope = 1;
  cfg->kgap = 100.0;
  cfg->cross_flip = 0;
  cfg->cross_tol = 1.0;
}

static int contour(const lens_t *L, cplx yc, double rho, const twk_ref_cfg *cfg,
                   double *mag, double *err, int32_t *nsamp, uint32_t *flags,
                   double *theta_out, int32_t max_out) {
  int cap = cfg->cap;
  sample_t *sm = (sample_t *)malloc(sizeof(sample_t) * (size_t)cap);
  int *ord = (int *)malloc(sizeof(int) * (size_t)cap);
  int *ord2 = (int *)malloc(sizeof(int) * (size_t)cap);
  double *wcum = (double *)malloc(sizeof(double) * ((size_t)cap + 1));
  double *Ei = (double *)malloc(sizeof(double) * (size_t)cap);
  double *Wi = (double *)malloc(sizeof(double) * (size_t)cap);
  double *newth = (double *)malloc(sizeof(double) * (size_t)cap);
  int *newiv = (int *)malloc(sizeof(int) * (size_t)cap);
  if (!sm || !ord || !ord2 || !wcum || !Ei || !Wi || !newth || !newiv) {
    free(sm); free(ord); free(ord2); free(wcum); free(Ei); free(Wi); free(newth); free(newiv);
    return TWK_REF_ENOMEM;
  }
  uint32_t fl = 0;
  int N = cfg->n0 < cap ? cfg->n0 : cap;
  for (int j = 0; j < N; ++j) {
    sample_at(L, yc, rho, 2.0 * PI_D * j / N, cfg->kgap, &sm[j]);
    ord[j] = j;
  }
  const double tol = cfg->tol;
  double A = 0.0, E = 0.0;
  for (;;) {
    for (int i = 0; i < N; ++i) fl |= sm[i].im.flags & (TWK_REF_FLAG_ANOMALY | TWK_REF_FLAG_NEARDEGEN);
    if (cfg->slope) {
      reset_demotions(sm, N);
      if (slope_detector(sm, ord, N) > 0) fl |= TWK_REF_FLAG_SLOPE;
    }
    nsum_t sa = {0.0, 0.0};
    double se = 0.0;
    for (int i = 0; i < N; ++i) {
      const sample_t *a = &sm[ord[i]];
      const sample_t *b = &sm[ord[(i + 1) % N]];
      double dth = (i + 1 < N ? b->theta : b->theta + 2.0 * PI_D) - a->theta;
      piece_t pc = interval_piece(a, b, dth, cfg->cross_flip);
      if (pc.anomaly) fl |= TWK_REF_FLAG_ANOMALY;
      nsum_add(&sa, pc.dA);
      Ei[i] = pc.E;
      Wi[i] = dth;
      se += pc.E;
    }
    A = sa.sum + sa.comp;
    E = se;
    /* a contour with both three- and five-image samples crosses a caustic:
     * there the tolerance is scaled by cfg->cross_tol */
    int seen3 = 0, seen5 = 0;
    for (int i = 0; i < N; ++i) {
      seen3 |= sm[i].im.n == 3;
      seen5 |= sm[i].im.n == 5;
    }
    const double tol_r = (seen3 && seen5) ? cfg->cross_tol * tol : tol;
    if (E <= tol_r * fabs(A)) break;
    int nnew = cfg->nnew;
    if (cfg->grow > 0 && N / cfg->grow > nnew) nnew = N / cfg->grow;
    if (N + nnew > cap) nnew = cap - N;
    if (nnew <= 0) { fl |= TWK_REF_FLAG_CAP; break; }
    /* tolerance-subtracted weights and their cumulative sum; an interval
     * narrower than THETA_FLOOR gets no new sample (READING: there the pair
     * merging on the critical curve is closer than its roots can be
     * resolved in binary64, and its pieces are rounding noise) */
    double avg = tol_r * fabs(A) / N;
    wcum[0] = 0.0;
    for (int i = 0; i < N; ++i) {
      double w = Wi[i] > THETA_FLOOR ? Ei[i] - avg : 0.0;
      wcum[i + 1] = wcum[i] + (w > 0.0 ? w : 0.0);
    }
    double W = wcum[N];
    if (!(W > 0.0)) break;
    /* invert the cumulative weight at nnew quantiles */
    int m = 0, iv = 0;
    for (int j = 0; j < nnew; ++j) {
      double u = (j + 0.5) / nnew * W;
      while (iv < N - 1 && wcum[iv + 1] <= u) ++iv;
      double wi = wcum[iv + 1] - wcum[iv];
      if (!(wi > 0.0)) continue;
      const sample_t *a = &sm[ord[iv]];
      double tb = iv + 1 < N ? sm[ord[iv + 1]].theta : 2.0 * PI_D;
      double th = a->theta + (u - wcum[iv]) / wi * (tb - a->theta);
      if (!(th > a->theta && th < tb)) continue;
      if (m > 0 && newiv[m - 1] == iv && !(th > newth[m - 1])) continue;
      newth[m] = th;
      newiv[m] = iv;
      ++m;
    }
    if (m == 0) { fl |= TWK_REF_FLAG_CAP; break; }
    /* solve the new samples and merge them into the sorted order */
    for (int j = 0; j < m; ++j) sample_at(L, yc, rho, newth[j], cfg->kgap, &sm[N + j]);
    int o = 0, j = 0;
    for (int i = 0; i < N; ++i) {
      ord2[o++] = ord[i];
      while (j < m && newiv[j] == i) { ord2[o++] = N + j; ++j; }
    }
    N += m;
    memcpy(ord, ord2, sizeof(int) * (size_t)N);
  }
  double area = PI_D * rho * rho;
  *mag = A / area;
  *err = E / area;
  *nsamp = N;
  *flags = fl;
  if (theta_out) {
    for (int i = 0; i < N && i < max_out; ++i) theta_out[i] = sm[ord[i]].theta;
  }
  free(sm); free(ord); free(ord2); free(wcum); free(Ei); free(Wi); free(newth); free(newiv);
  return TWK_REF_OK;
}

int twk_ref_finite_mag(double s, double q, int64_t n, const double *zx,
                       const double *zy, double rho, double tol,
                       const twk_ref_cfg *cfg_in, double *mag, double *err,
                       int32_t *nsamp, uint32_t *flags) {
  if (!lens_ok(s, q) || !(rho > 0.0) || !isfinite(rho) || !(tol > 0.0) ||
      n < 0 || (n > 0 && (!zx || !zy || !mag || !err || !nsamp || !flags)))
    return TWK_REF_EINVAL;
  twk_ref_cfg cfg;
  if (cfg_in) cfg = *cfg_in;
  else twk_ref_cfg_default(&cfg, tol);
  cfg.tol = tol;
  if (cfg.n0 < 4 || cfg.nnew < 1 || cfg.cap < cfg.n0 || cfg.cross_flip < 0 ||
      cfg.cross_flip > 3 || !(cfg.cross_tol > 0.0 && cfg.cross_tol <= 1.0))
    return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  for (int64_t i = 0; i < n; ++i) {
    if (!isfinite(zx[i]) || !isfinite(zy[i])) {
      mag[i] = NAN; err[i] = NAN; nsamp[i] = 0; flags[i] = TWK_REF_FLAG_NONFINITE;
      continue;
    }
    int rc = contour(&L, CMPLX(zx[i] - L.z2, zy[i]), rho, &cfg, &mag[i], &err[i],
                     &nsamp[i], &flags[i], NULL, 0);
    if (rc) return rc;
  }
  return TWK_REF_OK;
}

int twk_ref_finite_trace(double s, double q, double zx, double zy, double rho,
                         const twk_ref_cfg *cfg, double *mag, double *err,
                         int32_t *nsamp, uint32_t *flags, double *theta_out,
                         int32_t max_out) {
  if (!lens_ok(s, q) || !(rho > 0.0) || !cfg || !mag || !err || !nsamp || !flags)
    return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  return contour(&L, CMPLX(zx - L.z2, zy), rho, cfg, mag, err, nsamp, flags,
                 theta_out, max_out);
}

/* ------------------------------------------------------------------ */
/* Trajectory (not in the paper): straight line in the CM frame with    */
/* impact parameter u0 and angle alpha, tau = (t - t0)/tE.               */
/* ------------------------------------------------------------------ */
int twk_ref_trajectory(double u0, double alpha, int64_t n, const double *tau,
                       double *zx, double *zy) {
  if (n < 0 || (n > 0 && (!tau || !zx || !zy))) return TWK_REF_EINVAL;
  double ca = cos(alpha), sa = sin(alpha);
  for (int64_t i = 0; i < n; ++i) {
    zx[i] = tau[i] * ca - u0 * sa;
    zy[i] = tau[i] * sa + u0 * ca;
  }
  return TWK_REF_OK;
}

/* ------------------------------------------------------------------ */
/* Linear limb darkening (not in the paper; the paper only notes that    */
/* limb darkening is costly with contours).  Intensity relative to the    */
/* disk mean: I(r) = 1 - Gamma (1 - 1.5 sqrt(1 - r^2/rho^2)).  Annuli of   */
/* equal area: r_k = rho sqrt(k/na).  Annulus mean intensity I_k =        */
/* 1 - Gamma + Gamma * [(1-x_{k-1})^{3/2} - (1-x_k)^{3/2}] / (x_k - x_{k-1})*/
/* with x_k = r_k^2/rho^2.  mu_LD = sum_k I_k (x_k mu_k - x_{k-1} mu_{k-1}) */
/*                          / sum_k I_k (x_k - x_{k-1}).                   */
/* ------------------------------------------------------------------ */
int twk_ref_ld_combine(double gamma, int32_t na, const double *mu_k,
                       double *mu_ld) {
  if (na < 1 || !mu_k || !mu_ld) return TWK_REF_EINVAL;
  double num = 0.0, den = 0.0, xprev = 0.0, mprev = 0.0;
  for (int k = 1; k <= na; ++k) {
    double x = (double)k / na;
    double Ik = 1.0 - gamma +
                gamma * (pow(1.0 - xprev, 1.5) - pow(1.0 - x, 1.5)) / (x - xprev);
    num += Ik * (x * mu_k[k - 1] - xprev * mprev);
    den += Ik * (x - xprev);
    xprev = x;
    mprev = mu_k[k - 1];
  }
  *mu_ld = num / den;
  return TWK_REF_OK;
}

/* ------------------------------------------------------------------ */
/* Point-source adequacy (Sec. 2.3 names a quadrupole test and a ghost   */
/* image test without formulas).  READING:                               */
/*  - quadrupole: the four-point mean of mu at zeta_c +- rho, +- i rho   */
/*    exceeds mu(zeta_c) by (rho^2/4) Lap(mu) while the disk mean exceeds */
/*    it by (rho^2/8) Lap(mu); the finite-source correction is estimated  */
/*    as dQ = (mean4 - mu0)/2 and must satisfy CQ |dQ| < tol mu0;         */
/*  - every one of the five points has three images;                      */
/*  - ghost test: a ghost root g with residual R_g sits near the critical */
/*    curve when the source is near a fold; |R_g| grows like sqrt(d) with */
/*    the distance d to the caustic, with a scale set by f''.  The        */
/*    statistic |f''(g)| |R_g|^2 estimates d and must exceed CG rho for   */
/*    both ghosts of all five points.                                     */
/* ------------------------------------------------------------------ */
#define PS_CQ 20.0
#define PS_CG 8.0

/* The five point-source solves of the adequacy test: the centre zeta_c and
 * the four points zeta_c +- rho, zeta_c +- i rho, in that order. */
typedef struct {
  double mu[5];
  int adequate;
  int n0;          /* image count at the centre                         */
  double ghost0;   /* min over the centre's ghosts of |f''| |R|^2         */
  double pair0;    /* 5 images: min over opposite-parity real pairs of
                      |f''(midpoint)| |z+ - z-|^2 / 4                     */
} ps_probe_t;

static void ps_probe(const lens_t *L, cplx yc, double rho, double tol,
                     ps_probe_t *pp) {
  cplx pts[5] = {yc, yc + rho, yc + CMPLX(0.0, rho), yc - rho,
                 yc - CMPLX(0.0, rho)};
  int ok = 1;
  pp->ghost0 = INFINITY;
  pp->pair0 = INFINITY;
  for (int k = 0; k < 5; ++k) {
    images_t im;
    solve_point(L, pts[k], 100.0, &im);
    pp->mu[k] = mu_point(&im);
    if (im.n != 3) ok = 0;
    for (int g = im.n; g < 5; ++g) {
      double d = cabs(fsecond(L, im.z[g])) * creal(im.R[g] * conj(im.R[g]));
      if (!(d > PS_CG * rho)) ok = 0;
      if (k == 0 && d < pp->ghost0) pp->ghost0 = d;
    }
    if (k == 0) {
      pp->n0 = im.n;
      for (int a = 0; a < im.n; ++a)
        for (int b = 0; b < im.n; ++b) {
          if (!(im.par[a] > 0 && im.par[b] < 0)) continue;
          cplx dz = im.z[a] - im.z[b];
          double x = cabs(fsecond(L, 0.5 * (im.z[a] + im.z[b]))) *
                     creal(dz * conj(dz)) / 4.0;
          if (x < pp->pair0) pp->pair0 = x;
        }
    }
  }
  double dq = 0.5 * (0.25 * (pp->mu[1] + pp->mu[2] + pp->mu[3] + pp->mu[4]) -
                     pp->mu[0]);
  if (!(PS_CQ * fabs(dq) < tol * pp->mu[0])) ok = 0;
  pp->adequate = ok;
}

int twk_ref_ps_adequate(double s, double q, double zx, double zy, double rho,
                        double tol, int32_t *adequate, double *mu_ps) {
  if (!lens_ok(s, q) || !(rho > 0.0) || !(tol > 0.0) || !adequate || !mu_ps)
    return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  ps_probe_t pp;
  ps_probe(&L, CMPLX(zx - L.z2, zy), rho, tol, &pp);
  *adequate = pp.adequate;
  *mu_ps = pp.mu[0];
  return TWK_REF_OK;
}

/* ------------------------------------------------------------------ */
/* Features of one epoch for the learned sample budget and FS predictor  */
/* (not in the paper; inputs of the learned part).  READING, in order:   */
/*  f0 s, f1 log10 q, f2 Re zeta, f3 Im zeta (centre-of-mass frame),      */
/*  f4 log10 rho, f5 log10 mu_ps(zeta_c),                                 */
/*  f6 caustic proximity: +log10(1 + X/rho) with three images, X the     */
/*     centre's ghost statistic; -log10(1 + X/rho) with five, X the       */
/*     closest opposite-parity pair statistic (both estimate the source- */
/*     plane distance to the nearest fold),                               */
/*  f7 log10(rho |grad mu_ps| / mu_ps) from central differences over the  */
/*     four probe points, the argument floored at 1e-30.                  */
/* ------------------------------------------------------------------ */
int twk_ref_features(double s, double q, double zx, double zy, double rho,
                     double tol, float *feat, double *mu_ps,
                     int32_t *adequate) {
  if (!lens_ok(s, q) || !(rho > 0.0) || !(tol > 0.0) || !feat || !mu_ps ||
      !adequate)
    return TWK_REF_EINVAL;
  lens_t L = lens_make(s, q);
  ps_probe_t pp;
  ps_probe(&L, CMPLX(zx - L.z2, zy), rho, tol, &pp);
  double gx = pp.mu[1] - pp.mu[3], gy = pp.mu[2] - pp.mu[4];
  double grad = 0.5 * sqrt(gx * gx + gy * gy); /* rho |grad mu| */
  double prox = pp.n0 == 3 ? log10(1.0 + pp.ghost0 / rho)
                           : -log10(1.0 + pp.pair0 / rho);
  double f[8] = {s, log10(q), zx, zy, log10(rho), log10(pp.mu[0]), prox,
                 log10(fmax(grad / pp.mu[0], 1e-30))};
  for (int k = 0; k < 8; ++k) feat[k] = (float)f[k];
  *mu_ps = pp.mu[0];
  *adequate = pp.adequate;
  return TWK_REF_OK;
}
