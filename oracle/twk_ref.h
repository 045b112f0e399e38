/*
 * twk_ref.h -- plain FP64 CPU oracle for binary-lens point-source and
 * finite-source (uniform disk, contour integration) magnification.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, single-threaded
 * reference that the HIP path is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it and shares no code with it.
 *
 * Paper: Wang, Wang & Dong, "Twinkle: A GPU-based binary-lens microlensing
 * code with contour integration method" (arXiv 2501.03322).
 *
 * Conventions (paper Sec. 2.1, lens equation and binary positions):
 *   - lengths in units of the Einstein radius of the total mass;
 *   - origin at the centre of mass; lens 1 (mass m1 = 1/(1+q)) at
 *     z1 = -q s/(1+q), lens 2 (mass m2 = q/(1+q)) at z2 = s/(1+q);
 *   - source positions zeta are given in this centre-of-mass frame.
 * Internally the polynomial is written in the lens-2 frame of Sec. 2.2
 * (y = zeta - z2, eta = z - z2), where lens 1 sits at -s.
 *
 * All functions are synchronous, take host pointers, and return 0 on
 * success or a negative TWK_REF_E* code.  Nothing is allocated that outlives
 * a call.
 */
#ifndef TWK_REF_H
#define TWK_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TWK_REF_OK 0
#define TWK_REF_EINVAL (-1)
#define TWK_REF_ENOMEM (-3)

/* Per-result flag bits (same meaning as the GPU library's). */
#define TWK_REF_FLAG_POINT      (1u << 0) /* point-source value used            */
#define TWK_REF_FLAG_CAP        (1u << 1) /* sample cap reached, mu/err returned */
#define TWK_REF_FLAG_ANOMALY    (1u << 2) /* image count / parity anomaly        */
#define TWK_REF_FLAG_SLOPE      (1u << 3) /* slope detector reclassified a pair  */
#define TWK_REF_FLAG_NONFINITE  (1u << 4) /* non-finite input, output is NaN     */
#define TWK_REF_FLAG_NEARDEGEN  (1u << 5) /* ghost/real decision near threshold  */

/* Coefficients c0..c5 of the quintic sum_i c_i eta^i = 0 in the lens-2 frame,
 * by the cancellation-free refactoring of Sec. 2.2 (Eq. method-transformed).
 * zeta is in the centre-of-mass frame.  out[2k], out[2k+1] = Re, Im of c_k. */
int twk_ref_coeffs(double s, double q, double zeta_x, double zeta_y,
                   double *out12);

/* The conventional (VBBL-form) coefficients of Sec. 2.2 (Eq. lens-poly-orig),
 * with the printed symbol `a` in c3 read as -s.  Only for comparisons of
 * coefficient accuracy; never used for images. */
int twk_ref_coeffs_conventional(double s, double q, double zeta_x,
                                double zeta_y, double *out12);

/* All five roots of sum_k c_k x^k (c given as 12 doubles), by simultaneous
 * Aberth-Ehrlich iteration from a cold start followed by Newton polishing.
 * roots10[2k], roots10[2k+1] = Re, Im of root k.  Returns the number of
 * iterations used, or a negative error. */
int twk_ref_roots(const double *c12, double *roots10);

/* Images of a point source at zeta (centre-of-mass frame).
 *   img10:  the five polynomial roots, centre-of-mass frame, real images
 *           first (n_real of them), then the ghost pair;
 *   res10:  lens-equation residual R (Sec. 2.4.1) of each listed root;
 *   jac5:   Jacobian J = 1 - |f'|^2 of each listed root (Eq. jacobian);
 *   n_real: 3 or 5;  flags: TWK_REF_FLAG_* bits. */
int twk_ref_images(double s, double q, double zeta_x, double zeta_y,
                   double *img10, double *res10, double *jac5,
                   int32_t *n_real, uint32_t *flags);

/* Point-source magnification mu = sum over real images of 1/|J|. */
int twk_ref_point_mag(double s, double q, int64_t n, const double *zeta_x,
                      const double *zeta_y, double *mag, int32_t *n_images,
                      uint32_t *flags);

/* Derivatives along the limb at angle theta of a source of radius rho:
 * for each real image, z' = dz/dtheta and z' ^ z'' (Sec. 2.3, Eq. area_cal).
 * Images in the centre-of-mass frame, same order as twk_ref_images.
 * Computed by solving the differentiated lens equation directly. */
int twk_ref_limb_derivs(double s, double q, double zc_x, double zc_y,
                        double rho, double theta, double *img10,
                        double *dz10, double *wedge5, int32_t *n_real);

/* Finite-source (uniform disk) contour-integration configuration. */
typedef struct {
  double tol;    /* relative tolerance on the image area                  */
  int32_t n0;    /* initial uniform limb samples                           */
  int32_t nnew;  /* new samples per adaptive round (minimum)               */
  int32_t cap;   /* maximum samples per source                             */
  int32_t grow;  /* >0: new samples per round = max(nnew, N/grow)           */
  int32_t slope; /* 1: run the slope detector (Sec. 2.4.2)                  */
  double kgap;   /* residual-detector gap factor (default 100)              */
  int32_t cross_flip; /* diagnostic, default 0 (the reading used): bit 0
                         negates the cross-caustic correction of created
                         pairs, bit 1 that of destroyed pairs              */
  double cross_tol;   /* factor (0, 1] on tol for a contour whose samples
                         include both three- and five-image points (its
                         limb crosses a caustic), in the stop test and the
                         tolerance subtraction; default 1 (tol as stated)  */
} twk_ref_cfg;

/* Defaults as the paper describes its own sampler: tol as given, 64 initial
 * samples, 64 per round, cap 4096, slope detector on, gap factor 100. */
void twk_ref_cfg_default(twk_ref_cfg *cfg, double tol);

/* Uniform-disk magnification of n sources of radius rho at zeta (centre-of-
 * mass frame), by contour integration with adaptive limb sampling.
 *   mag = A / (pi rho^2), err = E / (pi rho^2); n_samples = limb samples used.
 * cfg may be NULL (defaults at the given tol). */
int twk_ref_finite_mag(double s, double q, int64_t n, const double *zeta_x,
                       const double *zeta_y, double rho, double tol,
                       const twk_ref_cfg *cfg, double *mag, double *err,
                       int32_t *n_samples, uint32_t *flags);

/* Diagnostic: run the contour integration of one source and report the
 * sorted limb angles used (theta_out, up to max_out entries). */
int twk_ref_finite_trace(double s, double q, double zeta_x, double zeta_y,
                         double rho, const twk_ref_cfg *cfg, double *mag,
                         double *err, int32_t *n_samples, uint32_t *flags,
                         double *theta_out, int32_t max_out);

/* Diagnostic: the piece of one interval in which an image pair is created
 * (kind > 0) or destroyed (kind < 0), from the pair's positions zp, zm
 * (+ and - parity), limb derivatives dp, dm (each as Re, Im) and
 * z' ^ z'' values wp, wm at the sample where the pair exists; dth is the
 * interval width.  Outputs: dA = chord + cross-caustic correction
 * (Sec. 2.3), E = E1 + E2 + E3 and E2 alone (Sec. 2.5, Eq. area_cross).
 * flip as in twk_ref_cfg.cross_flip. */
int twk_ref_cross_piece(const double *zp, const double *zm, const double *dp,
                        const double *dm, double wp, double wm, int32_t kind,
                        double dth, int32_t flip, double *dA, double *E,
                        double *E2);

/* Source centres along straight trajectories: zeta = (tau cos a - u0 sin a)
 * + i (tau sin a + u0 cos a), centre-of-mass frame. */
int twk_ref_trajectory(double u0, double alpha, int64_t n, const double *tau,
                       double *zeta_x, double *zeta_y);

/* Linear limb darkening by equal-area uniform annuli: combines the uniform-
 * disk magnifications mu_k of the nested disks of radius rho*sqrt(k/na),
 * k = 1..na, with annulus-mean intensities of the linear law. */
int twk_ref_ld_combine(double gamma, int32_t na, const double *mu_k,
                       double *mu_ld);

/* Point-source adequacy decision (quadrupole + ghost tests, Sec. 2.3):
 * returns 1 in *adequate if the point-source magnification may replace the
 * finite-source one at tolerance tol; mu_ps receives the point value. */
int twk_ref_ps_adequate(double s, double q, double zeta_x, double zeta_y,
                        double rho, double tol, int32_t *adequate,
                        double *mu_ps);

/* Eight features of one epoch for the learned budget / FS predictor, as
 * float32 (order: s, log10 q, Re zeta, Im zeta, log10 rho, log10 mu_ps,
 * signed caustic proximity, log10 of the relative gradient of mu_ps over
 * the probe radius), plus mu_ps and the adequacy decision. */
int twk_ref_features(double s, double q, double zeta_x, double zeta_y,
                     double rho, double tol, float *feat, double *mu_ps,
                     int32_t *adequate);

#ifdef __cplusplus
}
#endif

#endif /* TWK_REF_H */
