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

/* Forms of the quintic's coefficients (twk_coefficients). */
#define TWK_COEF_REFINED 0      /* Sec. 2.2, Eq. method-transformed (the method's) */
#define TWK_COEF_CONVENTIONAL 1 /* Sec. 2.2, Eq. lens-poly-orig (comparator only)  */

/* Mode bits for the finite-source calls. */
#define TWK_MODE_FP64 0u           /* FP64 root iterations                     */
#define TWK_MODE_MIXED (1u << 0)   /* FP32 bulk root iterations + FP64 polish  */
#define TWK_MODE_MLP (1u << 2)     /* learned sample budget / FS predictor      */
#define TWK_MODE_ALL_FS (1u << 3)  /* skip the point-source test: contour always */
/* The paper's dispatch of the contour work (Secs. 3, 4.1) instead of the
 * persistent kernel: sources in batches of up to 32768, one kernel launch
 * per refinement round over the list of the batch's unfinished sources,
 * whose records stay in global memory between launches; the host reads the
 * list's length after every round (the call waits for the point-source
 * pass and for each round; it is never captured in a graph).  Results are
 * those of the persistent kernel (same rounds, same arithmetic). */
#define TWK_MODE_ROUNDS (1u << 4)
/* Comparator, for accuracy comparisons only (not the method): every limb
 * point solves the quintic with the conventional coefficients of Sec. 2.2
 * (Eq. lens-poly-orig, in which terms of order 1 and of order q cancel for
 * small q; Fig. 1) and classifies its roots as older codes do: real when
 * the lens-equation residual is below a fixed absolute 1e-6 (Einstein
 * radii), no lens-equation polish, no slope detector, parity from sign(J).
 * FP64 only (TWK_EINVAL with TWK_MODE_MIXED or TWK_MODE_MLP); every source
 * is integrated (as with TWK_MODE_ALL_FS) by the round-by-round dispatch. */
#define TWK_MODE_CONVENTIONAL (1u << 5)

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
 * Errors: TWK_EINVAL if s <= 0, q <= 0, n < 0 or n > 2^48, or a pointer is
 * NULL (n > 0). */
int twk_point_mag(twk_ctx *ctx, double s, double q, int64_t n, const double *zeta_x,
                  const double *zeta_y, double *mag, int32_t *n_images, uint32_t *flags);

/* Coefficients c0..c5 of the quintic sum_k c_k eta^k = 0 whose roots are
 * the image positions in the lens-2 frame (eta = z - s/(1+q)), for n source
 * positions (zeta_x[i], zeta_y[i]) in the centre-of-mass frame: form
 * TWK_COEF_REFINED (Sec. 2.2, Eq. method-transformed, as every limb point
 * of the method assembles them) or TWK_COEF_CONVENTIONAL (Eq.
 * lens-poly-orig, the comparator's).  Output (device, [n][12] doubles):
 * Re, Im of c0, ..., c5.  Errors: TWK_EINVAL for s, q <= 0 or
 * non-finite, n < 0 or > 2^48, an unknown form, NULL pointers (n > 0). */
int twk_coefficients(twk_ctx *ctx, double s, double q, int64_t n, const double *zeta_x,
                     const double *zeta_y, int32_t form, double *c12);

/* Finite-source magnification of n uniform disks of radius rho centred at
 * (zeta_x[i], zeta_y[i]) by adaptive contour integration (Secs. 2.3-2.5, 3):
 * 64 initial limb samples, 64 new samples per round placed by inverse
 * transform sampling of the tolerance-subtracted interval errors, stop when
 * the summed error estimate is <= tol * |area|, at most 4096 samples.
 * Outputs (device, length n): mag = area/(pi rho^2); err = error estimate
 * in the same units; n_samples = limb samples used; flags.
 * mode: TWK_MODE_FP64 or TWK_MODE_MIXED; without TWK_MODE_ALL_FS the
 * point-source test may return the point value (flag bit 0).  The
 * persistent contour kernel takes the queued contours in a dispersed order
 * (a golden-ratio stride over the queue, a limb-darkened epoch's annuli
 * together) rather than in source order.  With TWK_MODE_MLP the learned
 * budget (weights from twk_mlp_set/load/train) predicts each contour's
 * sample count and the contours predicted to need 256 samples or more
 * are spread over the first half of the queue (launch tails); the sampling
 * of a contour is unchanged (it starts from the 64 uniform samples of the
 * paper's schedule), so the results are bit-identical to those of the same
 * call without TWK_MODE_MLP.
 * Errors: TWK_EINVAL for s, q, rho, tol <= 0 or non-finite, n < 0 or > 2^48, NULL
 * pointers or unknown mode bits; TWK_ENOMLP for TWK_MODE_MLP without
 * weights; TWK_ENOMEM / TWK_EDEVICE. */
int twk_finite_mag(twk_ctx *ctx, double s, double q, int64_t n, const double *zeta_x,
                   const double *zeta_y, double rho, double tol, uint32_t mode, double *mag,
                   double *err, int32_t *n_samples, uint32_t *flags);

/* Finite-source magnification with a lens and source of its own per element
 * (Sec. 2's problem statement, one instance per element): device arrays s,
 * q, zeta_x, zeta_y, rho of length n.  This is the form for time-varying
 * lenses -- orbital motion (s and the trajectory angle changing with time)
 * or parallax (a displaced source trajectory): the caller evaluates s(t),
 * q and the source position at each epoch, in the centre-of-mass frame of
 * that epoch's lens.  Outputs, mode, tolerance and the adaptive refinement
 * as for twk_finite_mag; elements may mix lenses freely in one persistent
 * launch.  An element whose s, q or rho is not finite and positive is
 * answered as a non-finite input (NaN, TWK_FLAG_NONFINITE).
 * Errors: TWK_EINVAL for tol <= 0 or non-finite, n < 0 or > 2^48, NULL
 * pointers (n > 0) or unknown mode bits; TWK_ENOMLP for TWK_MODE_MLP
 * without weights; TWK_ENOMEM / TWK_EDEVICE. */
int twk_finite_mag_each(twk_ctx *ctx, int64_t n, const double *s, const double *q,
                        const double *zeta_x, const double *zeta_y, const double *rho, double tol,
                        uint32_t mode, double *mag, double *err, int32_t *n_samples,
                        uint32_t *flags);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * twk_finite_mag without any allocation.  Same arguments, results and
 * errors as twk_finite_mag, bit-identical results, for modes TWK_MODE_FP64
 * or TWK_MODE_MIXED, optionally with TWK_MODE_ALL_FS.  Its scratch (work
 * counters, the queue order, the task queue and the global slices of the
 * persistent waves)
 * is a fixed device array of 130 MB compiled into the library, of which
 * each device holds one copy until the process ends; its address on a
 * device is looked up when the first context is created there.  Limits:
 * n <= 65536 sources per call (TWK_EINVAL above), at most 128 persistent
 * waves; the learned budget (TWK_MODE_MLP) and TWK_MODE_ROUNDS are refused
 * with TWK_EINVAL.  Issues only kernel launches on the context's stream (no
 * memset, no synchronisation), so it may be captured.  Every call on one
 * device shares that device's array: calls that overlap on a device (other
 * streams, other contexts or threads) race and must be serialised by the
 * caller.  It does not update twk_last_stats or the stage timing. */
int twk_finite_mag_noalloc(twk_ctx *ctx, double s, double q, int64_t n, const double *zeta_x,
                           const double *zeta_y, double rho, double tol, uint32_t mode,
                           double *mag, double *err, int32_t *n_samples, uint32_t *flags);

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
 * launch per chunk of parameter sets (a chunk holds at most 2^28 contour
 * tasks) fed by a device work queue.  Queued on the context's stream without
 * waiting for it (except when the context's buffers must grow).
 * Errors: TWK_EINVAL for nsets or nepochs < 0, nepochs above 2^30,
 * nsets * nepochs * n_annuli above 2^48, tol <= 0 or non-finite, n_annuli outside 1..64 (or not 1
 * without gamma), NULL pointers (when there is work) or unknown mode bits;
 * TWK_ENOMLP for TWK_MODE_MLP without weights; TWK_ENOMEM / TWK_EDEVICE.
 * Per-element parameters are not checked on the host: a non-finite source
 * position returns NaN with TWK_FLAG_NONFINITE. */
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
 * limb point), out[6] = intervals linked, out[7] = contour-kernel launches
 * of the call (one per chunk; a call is split into chunks of at most 2^28
 * contour tasks).  Synchronises the context's stream. */
int twk_last_stats(twk_ctx *ctx, int64_t *out8);

/* Per-kernel timing with HIP events on the context's stream (on != 0 to
 * enable).  After a finite-source call, twk_kernel_times writes (host
 * pointer ms[5], milliseconds), each summed over the call's chunks: the
 * point-source pass, the learned stage (0 without TWK_MODE_MLP) and the
 * contour kernel; then the rest of the call and the whole call.  A call
 * replayed from a captured graph is timed as a whole: the three stage
 * entries read 0 and the rest and whole-call entries both hold the whole
 * call.  Waits for the call.  Errors: TWK_EINVAL if timing is off. */
int twk_enable_timing(twk_ctx *ctx, int on);
int twk_kernel_times(twk_ctx *ctx, double *ms5);

/* ------------------------------------------------------------------------
 * Launch tuning of the contour stage and graph replay.  None of these
 * change the arithmetic of a source: results are bit-identical under any
 * tuning.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t waves_per_cu; /* resident contour waves per CU: the persistent grid is
                           waves_per_cu x CUs; 1 .. the occupancy limit of lds_cap
                           for the mixed path (whose sample records are smaller);
                           an FP64-path launch uses at most its own limit */
  int32_t lds_cap;      /* limb samples a source keeps in LDS (sorted arrays and
                           sample records) before continuing in global memory:
                           64, 128 or 256 */
  float budget_shift;   /* in [-2, 4]; no effect (the learned budget no longer
                           sets a starting grid; kept for the layout) */
  int32_t graphs;       /* 1: capture each call's launch sequence in a hipGraph and
                           replay it when an identical call (same arguments and
                           pointers) repeats; needs a created (non-null) stream */
} twk_tuning;

/* Current tuning (defaults: the occupancy limit at lds_cap 128, shift 1, no
 * graphs). */
int twk_get_tuning(twk_ctx *ctx, twk_tuning *out);
/* Set the tuning; synchronises the stream and drops captured graphs.
 * TWK_EINVAL for values out of range (graphs on a null stream included). */
int twk_set_tuning(twk_ctx *ctx, const twk_tuning *t);
/* Autotuner: times twk_lightcurves on this batch (a representative sample
 * of the workload; arguments as for twk_lightcurves) for every LDS capacity
 * and four persistent grid sizes each, taking the fastest of `trials`
 * (1..100) calls per candidate; the best tuning is left in the context
 * (graphs setting unchanged) and copied to *best (may be NULL).
 * Synchronous; allocates its own output buffers. */
int twk_autotune(twk_ctx *ctx, int64_t nsets, const double *s, const double *q,
                 const double *u0, const double *alpha, const double *rho,
                 const double *gamma, int64_t nepochs, const double *tau, int32_t n_annuli,
                 double tol, uint32_t mode, int32_t trials, twk_tuning *best);

/* ------------------------------------------------------------------------
 * Learned sample budget and finite-source predictor.  Not part of the
 * paper's method; an addition that only chooses where contour integration
 * starts.  Model: perceptron 8 -> 128 -> 128 -> 128 -> 2 with erf-GELU
 * activations x Phi(x), bf16 matrix-core products with float32
 * accumulation.  Parameters: one float32 vector of TWK_MLP_NPARAM entries,
 *   mean[8], std[8]   (features are standardised as (f - mean) / std),
 *   W0[8][128], b0[128], W1[128][128], b1[128], W2[128][128], b2[128],
 *   W3[128][2], b3[2]   (row-major, input index first).
 * Outputs per row: [0] log2 of the limb-sample count the contour needs,
 * [1] logit of "the point-source value misses the tolerance".
 * ---------------------------------------------------------------------- */
#define TWK_MLP_NPARAM 34450
#define TWK_MLP_GRAD_MAX_ROWS 65536

/* Per-epoch features of light-curve batches (same arguments as
 * twk_lightcurves for the geometry): feat (device, [nsets*nepochs][8]
 * float32) = s, log10 q, Re zeta, Im zeta, log10 rho, log10 mu_ps, signed
 * caustic proximity (+log10(1 + X/rho) with 3 images, X = min over ghosts of
 * |f''| |R|^2; -log10(1 + X/rho) with 5, X = min over opposite-parity real
 * pairs of |f''(midpoint)| |z+ - z-|^2 / 4), log10 of rho |grad mu_ps| / mu_ps
 * (central differences at zeta +- rho, zeta +- i rho, floored at 1e-30);
 * mu_ps (device, f64) the point value; adequate (device, i32) the
 * point-source test's decision at tolerance tol.  Non-finite centres give
 * NaN features.  Errors: TWK_EINVAL for negative sizes, nepochs above 2^30,
 * nsets * nepochs above 2^48, tol <= 0, NULL. */
int twk_features(twk_ctx *ctx, int64_t nsets, const double *s, const double *q,
                 const double *u0, const double *alpha, const double *rho, int64_t nepochs,
                 const double *tau, double tol, float *feat, double *mu_ps, int32_t *adequate);

/* Install parameters from a host vector of n = TWK_MLP_NPARAM floats
 * (copied; synchronous).  TWK_EINVAL for a wrong n, non-finite entries or
 * std <= 0. */
int twk_mlp_set(twk_ctx *ctx, const float *host_params, int64_t n);
/* Copy the current parameters to a host vector (synchronous); TWK_ENOMLP if none. */
int twk_mlp_get(twk_ctx *ctx, float *host_params, int64_t n);
/* Weight file: 8 bytes "TWKMLP01", int32 count (= TWK_MLP_NPARAM), then the
 * float32 parameter vector, little-endian.  TWK_EINVAL for unreadable or
 * malformed files (the context keeps its previous weights). */
int twk_mlp_save(twk_ctx *ctx, const char *path);
int twk_mlp_load(twk_ctx *ctx, const char *path);

/* Inference on n rows: feat (device, [n][8] raw features) -> out (device,
 * [n][2] float32).  Asynchronous.  TWK_ENOMLP without weights; TWK_EINVAL
 * for n < 0 or > 2^48 or NULL pointers (n > 0). */
int twk_mlp_infer(twk_ctx *ctx, int64_t n, const float *feat, float *out);

/* Loss and gradient on one batch of n (1..TWK_MLP_GRAD_MAX_ROWS) rows:
 * loss = mean Huber(out0 - y_budget; delta) + mean BCE-with-logits(out1,
 * y_fs).  grad (device, TWK_MLP_NPARAM floats, same layout as the
 * parameters; the 16 standardisation entries are set to 0); *loss (host).
 * Synchronous.  The device work area is shared with twk_mlp_train. */
int twk_mlp_grad(twk_ctx *ctx, int64_t n, const float *feat, const float *y_budget,
                 const float *y_fs, float huber_delta, float *grad, double *loss);

typedef struct {
  int32_t epochs;      /* passes over the rows                              */
  int32_t batch;       /* rows per Adam step, 32 .. TWK_MLP_GRAD_MAX_ROWS    */
  float lr, lr_end;    /* Adam step size, decayed linearly to lr_end         */
  float beta1, beta2, eps;
  float huber_delta;
  int32_t init;        /* 1: standardise from these rows and draw fresh       */
                       /*    He-normal weights; 0: continue from the current  */
  uint64_t seed;       /* initialisation and shuffles (splitmix64)           */
} twk_train_cfg;

/* Minibatch Adam training on n rows (device: feat [n][8], y_budget [n],
 * y_fs [n] in {0,1}); every epoch visits the rows in a fresh shuffled order
 * and drops the last n mod batch.  loss_hist (host, may be NULL) receives
 * the mean loss of each epoch.  Synchronous; deterministic for a seed. */
int twk_mlp_train(twk_ctx *ctx, int64_t n, const float *feat, const float *y_budget,
                  const float *y_fs, const twk_train_cfg *cfg, float *loss_hist);

#ifdef __cplusplus
}
#endif

#endif /* TWK_H */
