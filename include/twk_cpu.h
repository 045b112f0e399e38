/*
 * twk_cpu.h -- multi-core CPU backend of the finite-source binary-lens
 * magnification method (the CPU version of the paper's Sec. 4.5).
 *
 * Paper: S. Wang, L. Wang & S. Dong, "Twinkle: A GPU-based binary-lens
 * microlensing code with contour integration method", arXiv 2501.03322.
 *
 * The same method and readings as the GPU library (include/twk.h): refined
 * coefficients (Sec. 2.2), all five roots with a lens-equation polish,
 * residual ghost detection with parity from the parity sum (Secs. 2.3,
 * 2.4.1), least-distance linking, Stokes area with the parabolic and
 * cross-caustic corrections and the error estimate of Sec. 2.5, 64 initial
 * limb samples and 64 more per round placed by inverse transform sampling
 * of the tolerance-subtracted interval errors, at most 4096 samples
 * (Sec. 3), the point-source test before any contour work (Sec. 2.3), and
 * linear limb darkening by equal-area annuli.  One source per thread at a
 * time; `threads` worker threads share the sources (0 = all hardware
 * threads).  Differences from the GPU path: no slope detector (near-caustic
 * samples whose ghost/real decision is marginal are flagged), no learned
 * budget, FP64 throughout.
 *
 * All pointers are HOST memory owned by the caller; calls are synchronous
 * and return 0 or TWK_CPU_EINVAL (-1).  Flags as in twk.h (bit 0 point
 * value, 1 sample cap, 2 anomaly, 4 non-finite input, 5 near-degenerate).
 */
#ifndef TWK_CPU_H
#define TWK_CPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TWK_CPU_EINVAL (-1)

/* Uniform-disk magnification of n sources of radius rho centred at
 * (zeta_x[i], zeta_y[i]) (centre-of-mass frame, Einstein radii); all_fs != 0
 * skips the point-source test.  Outputs (length n): mag, err, n_samples,
 * flags.  TWK_CPU_EINVAL for s, q, rho, tol <= 0 or non-finite, n < 0, NULL
 * pointers (n > 0). */
int twk_cpu_finite_mag(double s, double q, int64_t n, const double *zeta_x, const double *zeta_y,
                       double rho, double tol, int32_t all_fs, int32_t threads, double *mag,
                       double *err, int32_t *n_samples, uint32_t *flags);

/* Light curves as twk_lightcurves (include/twk.h): nsets parameter sets
 * (s, q, u0, alpha, rho, gamma; gamma may be NULL for uniform sources, then
 * n_annuli must be 1) times nepochs epochs tau, straight trajectories
 * zeta = (tau cos a - u0 sin a) + i (tau sin a + u0 cos a).  Outputs
 * (length nsets * nepochs, set-major): mag, err, n_samples (summed over
 * annuli), flags.  TWK_CPU_EINVAL for bad sizes, tol <= 0, n_annuli outside
 * 1..64 or not 1 without gamma, NULL pointers. */
int twk_cpu_lightcurves(int64_t nsets, const double *s, const double *q, const double *u0,
                        const double *alpha, const double *rho, const double *gamma,
                        int64_t nepochs, const double *tau, int32_t n_annuli, double tol,
                        int32_t threads, double *mag, double *err, int32_t *n_samples,
                        uint32_t *flags);

#ifdef __cplusplus
}
#endif

#endif /* TWK_CPU_H */
