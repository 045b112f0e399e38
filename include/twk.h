/*
 * twk.h -- C ABI of the MI355X (gfx950) binary-lens magnification library.
 *
 * Paper: S. Wang, L. Wang & S. Dong, "Twinkle: A GPU-based binary-lens
 * microlensing code with contour integration method", arXiv 2501.03322.
 *
 * Problem statement (paper Sec. 2.1): a binary lens of separation s and mass
 * ratio q = m2/m1, lengths in Einstein radii of the total mass, origin at
 * the centre of mass, lens 1 at -q s/(1+q) and lens 2 at s/(1+q) on the real
 * axis.  A source at zeta has images z solving
 *     zeta = z + m1/(conj(z1) - conj(z)) + m2/(conj(z2) - conj(z)).
 * For a uniform source disk of radius rho the magnification is the total
 * image area divided by the source area (Sec. 1); it is computed by contour
 * integration of the limb images (Secs. 2.2-2.5) with a relative tolerance.
 *
 * Conventions for every call:
 *   - all array arguments are DEVICE pointers (memory of the context's
 *     device), owned by the caller, which must keep them alive until the
 *     work is complete (twk_sync or a later synchronisation of the stream);
 *   - all calls are asynchronous on the context's stream, except
 *     twk_create/twk_destroy/twk_sync;
 *   - return value: TWK_OK (0) or a negative TWK_E* status; no call aborts
 *     or throws.  After TWK_EDEVICE, twk_last_hip_error gives the HIP code;
 *   - one context per host thread; contexts own only their scratch memory.
 *
 * Per-element flags (uint32):
 *   bit 0  point-source value returned (finite-source test passed)
 *   bit 1  sample cap (4096 limb points) reached; mag and err still returned
 *   bit 2  image-count or parity anomaly seen on the limb
 *   bit 3  slope detector reclassified or deleted an image pair
 *   bit 4  non-finite input; outputs are NaN
 *   bit 5  a ghost/real decision lay near its threshold
 */
#ifndef TWK_H
#define TWK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TWK_OK 0
#define TWK_EINVAL (-1)  /* bad scalar argument, NULL pointer, bad mode bits */
#define TWK_EDEVICE (-2) /* a HIP call failed                              */
#define TWK_ENOMEM (-3)  /* device allocation failed                        */
#define TWK_ENOMLP (-4)  /* TWK_MODE_MLP requested without loaded weights   */

/* Mode bits for the finite-source calls. */
#define TWK_MODE_FP64 0u           /* FP64 root iterations                     */
#define TWK_MODE_MIXED (1u << 0)   /* FP32 bulk root iterations + FP64 polish  */
#define TWK_MODE_MLP (1u << 2)     /* learned sample budget / FS predictor      */
#define TWK_MODE_ALL_FS (1u << 3)  /* skip the point-source test: contour always */

#define TWK_FLAG_POINT (1u << 0)
#define TWK_FLAG_CAP (1u << 1)
#define TWK_FLAG_ANOMALY (1u << 2)
#define TWK_FLAG_SLOPE (1u << 3)
#define TWK_FLAG_NONFINITE (1u << 4)
#define TWK_FLAG_NEARDEGEN (1u << 5)

typedef struct twk_ctx twk_ctx;

/* Create a context on HIP device `device`, issuing work on `stream`
 * (a hipStream_t; NULL = the device's null stream).  The stream is borrowed,
 * not owned. */
int twk_create(twk_ctx **out, int device, void *stream);
int twk_destroy(twk_ctx *ctx);
/* Block until all work issued by the context has completed. */
int twk_sync(twk_ctx *ctx);
/* Last HIP error code seen by the context (0 if none). */
int twk_last_hip_error(const twk_ctx *ctx);
const char *twk_strerror(int status);

/* Point-source magnification (sum over real images of 1/|J|, Eq. jacobian)
 * of n sources at (zeta_x[i], zeta_y[i]), centre-of-mass frame.
 * Outputs (device, length n): mag; n_images (3 or 5); flags.
 * Errors: TWK_EINVAL if s <= 0, q <= 0, n < 0 or a pointer is NULL (n > 0). */
int twk_point_mag(twk_ctx *ctx, double s, double q, int64_t n, const double *zeta_x,
                  const double *zeta_y, double *mag, int32_t *n_images, uint32_t *flags);

/* Finite-source magnification of n uniform disks of radius rho centred at
 * (zeta_x[i], zeta_y[i]) by adaptive contour integration (Secs. 2.3-2.5, 3):
 * 64 initial limb samples, 64 new samples per round placed by inverse
 * transform sampling of the tolerance-subtracted interval errors, stop when
 * the summed error estimate is <= tol * |area|, at most 4096 samples.
 * Outputs (device, length n): mag = area/(pi rho^2); err = error estimate
 * in the same units; n_samples = limb samples used; flags.
 * mode: TWK_MODE_FP64 or TWK_MODE_MIXED; without TWK_MODE_ALL_FS the
 * point-source test may return the point value (flag bit 0).
 * Errors: TWK_EINVAL for s, q, rho, tol <= 0 or non-finite, n < 0, NULL
 * pointers or unknown mode bits; TWK_ENOMEM / TWK_EDEVICE. */
int twk_finite_mag(twk_ctx *ctx, double s, double q, int64_t n, const double *zeta_x,
                   const double *zeta_y, double rho, double tol, uint32_t mode, double *mag,
                   double *err, int32_t *n_samples, uint32_t *flags);

/* Batched light curves: nsets lenses/sources (device arrays s, q, u0,
 * alpha, rho, each of length nsets) times nepochs epochs tau (device array)
 * on straight trajectories zeta = (tau cos a - u0 sin a) + i (tau sin a +
 * u0 cos a), centre-of-mass frame.  gamma (length nsets, linear limb-
 * darkening coefficient of I(r)/<I> = 1 - gamma (1 - 1.5 sqrt(1 - r^2/rho^2)))
 * may be NULL for uniform sources (then n_annuli must be 1); with gamma the
 * source is split into n_annuli (1..64) equal-area annuli whose uniform-disk
 * magnifications are combined with the annulus mean intensities.
 * Outputs (device, length nsets*nepochs, set-major): mag, err, n_samples
 * (summed over annuli), flags.  Point-source-adequate epochs are answered
 * by the point value; all others by contour integration in one persistent
 * launch per chunk of parameter sets (a chunk holds at most 2^24 contour
 * tasks) fed by a device work queue. */
int twk_lightcurves(twk_ctx *ctx, int64_t nsets, const double *s, const double *q,
                    const double *u0, const double *alpha, const double *rho,
                    const double *gamma, int64_t nepochs, const double *tau, int32_t n_annuli,
                    double tol, uint32_t mode, double *mag, double *err, int32_t *n_samples,
                    uint32_t *flags);

/* Magnification map of one lens: uniform disks of radius rho centred on the
 * pixel centres of an nx x ny grid over the box [xc - width/2, xc + width/2]
 * x [yc - height/2, yc + height/2] (centre-of-mass frame).  Outputs (device,
 * length nx*ny, index iy*nx + ix): mag, err, n_samples, flags.  mode as for
 * twk_finite_mag. */
int twk_mag_map(twk_ctx *ctx, double s, double q, double rho, double xc, double yc, double width,
                double height, int32_t nx, int32_t ny, double tol, uint32_t mode, double *mag,
                double *err, int32_t *n_samples, uint32_t *flags);

/* Work counters of the last finite-source call (host pointer out[8]):
 * out[0] = contour tasks run, out[1] = tasks whose sorted limb arrays
 * outgrew LDS (continued in global memory), out[2] = limb samples of the
 * returned results, out[3] = persistent waves launched, out[4] = FP32 root
 * sweeps, out[5] = FP64 root sweeps (one sweep updates all five roots of one
 * limb point), out[6] = intervals linked, out[7] = contour runs.
 * Synchronises the context's stream. */
int twk_last_stats(twk_ctx *ctx, int64_t *out8);

/* Per-kernel timing with HIP events on the context's stream (on != 0 to
 * enable).  After a finite-source call, twk_kernel_times writes (host
 * pointer ms[4], milliseconds): point-source pass and contour kernel of the
 * first chunk, the rest of the call, whole call.  Waits for the call.
 * Errors: TWK_EINVAL if timing is off. */
int twk_enable_timing(twk_ctx *ctx, int on);
int twk_kernel_times(twk_ctx *ctx, double *ms4);

#ifdef __cplusplus
}
#endif

#endif /* TWK_H */
