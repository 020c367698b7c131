/*
 * dsnlm.h -- C ABI of the MI355X (gfx950) library for the doubly stochastic
 * NLM denoiser (DSG-NLM) and linearized plug-and-play ADMM.
 *
 * Paper: Unni, Ghosh, Chaudhury, "Linearized ADMM and Fast Nonlocal Denoising
 * for Efficient Plug-and-Play Restoration" (arXiv 1901.06110).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Images are single-channel FP32, row-major, contiguous, n1 rows by n2
 * columns, in DEVICE memory owned by the caller (for example torch tensors'
 * data pointers).  No call copies between host and device unless it says so.
 * `stream` is a hipStream_t (NULL = the default stream); all work is enqueued
 * on it and calls return without synchronising, except the few documented as
 * synchronous.  Only the opaque `dsnlm_weights` handle is owned by the
 * library (created by a build call, released by dsnlm_weights_destroy).
 *
 * Every call returns a dsnlm_status.  Arguments are validated on the host
 * before anything is launched; a rejected call returns DSNLM_EINVAL and leaves
 * all outputs untouched.  A failure reported by the HIP runtime is returned
 * as DSNLM_EDEVICE.  dsnlm_last_error() returns a per-thread message for the
 * last non-OK status.  No C++ exception crosses this interface.
 *
 * Denoiser parameters (Section 3, eq. NLM and steps S1-S3):
 *   S  search half-width: the window of pixel s holds the pixels r of the
 *      image with max(|r1-s1|, |r2-s2|) <= S (the window is cut at the image
 *      border and includes s itself);
 *   P  patch half-width: patches are (2P+1) x (2P+1); patch pixels outside
 *      the image take the half-sample symmetric mirror of the guide
 *      (index -1 -> 0, n -> n-1), which needs P < min(n1, n2);
 *   h  bandwidth: k_{s,r} = exp(-||P_s - P_r||^2 / (2 (2P+1)^2 h^2));
 *      must be finite and > 0.
 *   Supported: 0 <= S <= 24, 0 <= P <= 5; dsnlm_build_weights, dsnlm_apply,
 *   dsnlm_forward and dsnlm_forward_brute also take 5 < P <= 15 (patch sides
 *   up to 31, Table 1's range: the half-window forward sweeps, or the
 *   full-window wide-patch passes when the tuning table selects a full-window
 *   schedule); the other entry points return DSNLM_EUNSUPPORTED for P > 5.  Images are limited
 *   to 2^28 pixels, and so is the image padded by S + P on every side
 *   (the kernels index elements with 32-bit offsets): larger ones return
 *   DSNLM_EUNSUPPORTED before anything is launched.
 * The weights are Lambda_{s,r} k_{s,r} with the separable hat
 * Lambda = (1 - |r1-s1|/(S+1)) (1 - |r2-s2|/(S+1)) (step S1), normalised
 * symmetrically by the row sums (step S2) and scaled by the largest
 * resulting row sum m with the diagonal completed to row sum one (step S3).
 * W is symmetric and doubly stochastic.  W is never stored: a handle keeps
 * the guide, the per-pixel factors c_s = (row sum of step S1)^(-1/2), the
 * step-S2 row sums delta_s, and m with the first pixel attaining it.
 */
#ifndef DSNLM_H
#define DSNLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DSNLM_OK = 0,
    DSNLM_EINVAL = -1,      /* bad argument; nothing was launched            */
    DSNLM_ENOMEM = -2,      /* device allocation failed                      */
    DSNLM_EDEVICE = -3,     /* the HIP runtime reported an error             */
    DSNLM_ENONFINITE = -4,  /* a solver produced a non-finite residual       */
    DSNLM_EUNSUPPORTED = -5 /* valid per the paper but outside this library  */
} dsnlm_status;

typedef struct dsnlm_weights dsnlm_weights;

/* Build the weights of W(guide) (Algorithm 2, first and second aggregation:
 * row sums of step S1, then the step-S2 row sums and their maximum m).
 * guide: device, n1*n2 floats.  If *out is NULL a new handle is created;
 * if *out is an existing handle of the same n1, n2 it is rebuilt in place
 * (no allocation).  The handle copies the guide, so the caller may reuse the
 * guide buffer once the stream has passed this call. */
int dsnlm_build_weights(const float* guide, int n1, int n2, int S, int P, float h,
                        void* stream, dsnlm_weights** out);

/* y = W x for built weights (Algorithm 2, third aggregation, computed as
 * y_s = x_s + (1/m) c_s sum_r Lambda k c_r (x_r - x_s), which equals the
 * loop's sum of w x_r plus (1 - sum w) x_s).  x, y: device, n1*n2 floats;
 * y must not overlap x.  The handle records the intermediate needed by
 * dsnlm_apply_backward for this x. */
int dsnlm_apply(const dsnlm_weights* w, const float* x, float* y, void* stream);

/* Build and apply in one go: y = W(guide) x, two sweeps over the window
 * instead of three.  out: NULL, or as in dsnlm_build_weights (the handle then
 * holds everything dsnlm_apply_backward needs).  guide may equal x. */
int dsnlm_forward(const float* guide, const float* x, float* y, int n1, int n2,
                  int S, int P, float h, void* stream, dsnlm_weights** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as dsnlm_forward with out = NULL -- y = W(guide) x, the same
 * kernels, bit-identical results while the scratch below holds the partial
 * regions of dsnlm_forward's shift split for the image (for larger images
 * the split is reduced to fit, and the result differs only by the order of
 * FP32 additions) -- but it allocates nothing (no hipMalloc,
 * no hipFree, no allocating library call) and does not synchronise.  Its
 * intermediates (c, delta, B', m, the partial regions, the mirrored guide)
 * live in a fixed scratch array of dsnlm_forward_noalloc_limit() bytes
 * (48 MiB) that each device holds from its first call until the process ends.
 * Arguments as for dsnlm_forward; P <= 5.  An image whose intermediates
 * (dsnlm_forward_noalloc_bytes) exceed the limit returns DSNLM_EUNSUPPORTED
 * before anything is launched (1024 x 1024 at S = 10, P = 3 needs 31 MiB
 * without a shift split, 44 MiB with the 2-way split it then uses).
 * Every call on a device shares that device's scratch, which keeps the last
 * call's contents: calls that overlap in time on one device (different
 * streams, or host threads) race and give wrong results; calls ordered on
 * one stream are safe. */
int dsnlm_forward_noalloc(const float* guide, const float* x, float* y, int n1, int n2, int S, int P,
                          float h, void* stream);
/* Scratch bytes of the array above, and bytes an n1 x n2 image at S, P
 * would use of it (0 for arguments outside the supported range).  Host-only. */
size_t dsnlm_forward_noalloc_limit(void);
size_t dsnlm_forward_noalloc_bytes(int n1, int n2, int S, int P);

/* Plain NLM, eq. NLM of Section 3 (the row-stochastic filter DSG-NLM is
 * derived from): y_s = sum_r k_{s,r} x_r / sum_r k_{s,r}, k the same kernel of
 * the guide's patches (no hat), r over the border-cut window, r = s included.
 * Arguments as for dsnlm_forward; out (NULL or a handle, created if *out is
 * NULL) only lends its workspace: the handle then holds no DSG-NLM weights
 * (dsnlm_apply_backward rejects it until the next DSG-NLM forward). */
int dsnlm_nlm(const float* guide, const float* x, float* y, int n1, int n2, int S, int P, float h,
              void* stream, dsnlm_weights** out);

/* The brute-force comparator of Table 1: y = W(guide) x with every patch
 * distance summed directly over its N_p^2 offsets (no box sums), one GPU
 * thread per pixel.  Same arguments, outputs and handle state as
 * dsnlm_forward; for timing comparisons, not the fast path. */
int dsnlm_forward_brute(const float* guide, const float* x, float* y, int n1, int n2, int S, int P, float h,
                        void* stream, dsnlm_weights** out);

/* Vector-Jacobian product of y = W(guide, h) x at the x of the last apply or
 * forward on this handle (x must be passed again, unchanged).
 * dy: cotangent of y.  Outputs (each may be NULL to skip it):
 *   dx     = W dy (W is symmetric), n1*n2 floats;
 *   dguide = gradient with respect to the guide, n1*n2 floats;
 *   dh     = gradient with respect to h, one float on the device.
 * The derivative of the maximum m is routed to the first pixel attaining it.
 * Outputs are overwritten, not accumulated.  Not defined in the paper: the
 * chain rule through eq. NLM and steps S1-S3. */
int dsnlm_apply_backward(const dsnlm_weights* w, const float* x, const float* dy,
                         float* dx, float* dguide, float* dh, void* stream);

void dsnlm_weights_destroy(dsnlm_weights* w);

/* Copy the handle's scalars to the host (synchronises the stream):
 * m (largest step-S2 row sum) and the flat index of the first pixel
 * attaining it.  Either pointer may be NULL. */
int dsnlm_weights_scalars(const dsnlm_weights* w, float* m, int* argmax, void* stream);

/* Device pointers to the handle's per-pixel arrays (valid until destroy):
 * which = 0: c (row sums of step S1 to the power -1/2), 1: delta (row sums
 * after step S2), 2: the guide copy.  Returns NULL for a bad argument. */
const float* dsnlm_weights_array(const dsnlm_weights* w, int which);

/* ----------------------------------------------------------------------- */
/* Many images of uneven sizes denoised together: one launch per sweep for  */
/* the whole batch, each image with its own m.                              */
typedef struct {
    const float* guide; /* device, n1*n2 */
    const float* x;     /* device, n1*n2 (may equal guide) */
    float* y;           /* device, n1*n2, must not overlap x */
    int n1, n2;
    float h;            /* per-image bandwidth, > 0 */
} dsnlm_image;

/* imgs: HOST array of `count` descriptors (count = 0 is a no-op).  The
 * per-image intermediates live in a grow-only device workspace owned by the
 * library and reused by later calls; the descriptor list is uploaded only
 * when it changes.  Calls on different streams must not overlap in time
 * (they share the workspace). */
int dsnlm_forward_batched(const dsnlm_image* imgs, int count, int S, int P, void* stream);

/* State of image `image` (0-based) of the LAST dsnlm_forward_batched call:
 * device pointers to its c (row sums of step S1 to the power -1/2) and delta
 * (row sums after step S2) inside the library's batch workspace (valid until
 * the next batched call), and, copied to the host, its m and the flat index
 * of the first pixel attaining it (this copy synchronises the stream).  Any
 * output may be NULL.  DSNLM_EINVAL if there is no such image. */
int dsnlm_batched_state(int image, float* m, int* argmax, const float** c, const float** delta,
                        void* stream);

/* Vector-Jacobian products of the LAST dsnlm_forward_batched call (same
 * images, same order; its inputs must be unchanged): per image, dy is the
 * cotangent of y and dx = W dy, dguide, dh (device scalar) are written; each
 * output may be NULL.  One launch per backward sweep for the whole batch.
 * Guide and bandwidth gradients cover every supported S (LDS permitting:
 * DSNLM_EUNSUPPORTED otherwise). */
typedef struct {
    const float* dy;
    float* dx;
    float* dguide;
    float* dh;
} dsnlm_image_grad;
int dsnlm_backward_batched(const dsnlm_image_grad* grads, int count, void* stream);

/* ----------------------------------------------------------------------- */
/* Linearized plug-and-play ADMM (Section 2, Algorithm 1).                   */
/* Problem: min_x f(x) + lambda g(x), x in C = [lo, hi]^n.  f is defined by  */
/* the forward operator below; g is implicit in the DSG-NLM denoiser, whose  */
/* bandwidth is sigma = sqrt(lambda / rho) unless h > 0 overrides it.       */
typedef enum { LADMM_OP_SR = 1, LADMM_OP_SPI = 2 } ladmm_op_kind;

typedef struct {
    ladmm_op_kind kind;
    int n1, n2;               /* high-resolution image size */
    /* Super-resolution (Section 4.1, eq. dataterm): f = 1/2 ||A x - y||^2,
     * A = keep every `factor`-th sample (phase 0) of the blur of x by the
     * separable kernel taps (x) taps; blur pixels outside the image take the
     * half-sample symmetric mirror (boundary = 0) or wrap (boundary = 1).
     * taps: HOST array of blur_size floats (odd size <= 31, normalised by the
     * caller); y: device, ceil(n1/factor) x ceil(n2/factor) floats. */
    const float* taps;
    int blur_size;
    int factor;               /* 1..8 */
    int boundary;             /* 0 symmetric, 1 periodic */
    const float* y;
    /* Single-photon imaging (Section 4.2, eqs. obj and photongrad): per pixel
     * K1 = ones[i] of K binary measurements are 1; f = sum phi(x_i) with
     * phi(t) = (K-K1) eta t / K - K1 log(1 - exp(-eta t/K)), evaluated at
     * max(t, t_min).  ones: device, n1*n2 bytes. */
    const unsigned char* ones;
    int K;
    float eta;
    float t_min;
} ladmm_operator;

typedef struct {
    float lambda, rho;        /* Algorithm 1's lambda and rho (> 0) */
    float gamma;              /* 1/alpha: alpha = 1/gamma must exceed the
                                 Lipschitz constant of grad f for the
                                 convergence result of Section 2 */
    int S, P;                 /* denoiser window and patch half-widths */
    float h;                  /* > 0: bandwidth; <= 0: sqrt(lambda / rho) */
    int iters;                /* iterations for ladmm_solve */
    int freeze_after;         /* k0 >= 1: weights rebuilt from the denoiser's
                                 input x + u while k <= k0, then frozen */
    float lo, hi;             /* box C = [lo, hi]^n (lo < hi) */
    int denoiser;             /* 0: DSG-NLM (Section 3); 1: plain NLM (eq. NLM),
                                 rebuilt every iteration (freeze_after is not
                                 used; no backward) */
} ladmm_params;

/* One iteration k (1-based) of Algorithm 1 in place on x, v, u (device,
 * n1*n2 each): x <- Pi_C(mu (alpha x + rho (v - u) - grad f(x))),
 * v <- W (x + u) with W rebuilt from x + u when k <= freeze_after (into *w,
 * created if NULL) and reused otherwise, u <- u + x - v. */
int ladmm_step(const ladmm_operator* op, const ladmm_params* p, int k, dsnlm_weights** w,
               float* x, float* v, float* u, void* stream);

/* Run p->iters iterations from (x, v, u) (device, in place).  residuals:
 * NULL or device [iters][2]: RMS of x - v and of rho (v_k - v_{k-1}) per
 * iteration.  checkpoints: NULL or device [iters][4][n1*n2]: x, v, u and the
 * denoiser input x + u after each iteration.
 * All iterations (adaptive and frozen) are captured into one HIP graph the
 * first time a combination of image size, operator kind, scalars and taps,
 * params, and whether residuals and checkpoints are requested is seen on the
 * current device, and the graph is replayed by later calls with the same
 * combination (other buffers included).  The graph works on copies the
 * library keeps for that combination -- x, v, u, the observation (y or
 * ones), residuals, checkpoints -- which are copied from the caller's buffers
 * before each replay and back after it (device-to-device copies).  Up to 4
 * combinations are kept, each with its own weights and buffers (about 27 MiB
 * at 512 x 512, S = 10, without checkpoints), least recently used dropped
 * first.  The work runs on a library stream of the device that waits for the
 * work already on `stream`, and `stream` waits for it, so ordering is as if it
 * ran on `stream`.  Returns without synchronising when residuals is NULL; with
 * residuals it synchronises and returns DSNLM_ENONFINITE if one is not
 * finite.  `stream` must not be under
 * capture (DSNLM_EINVAL): the call captures its own graph. */
int ladmm_solve(const ladmm_operator* op, const ladmm_params* p, float* x, float* v, float* u,
                float* residuals, float* checkpoints, void* stream);

/* Standard plug-and-play ADMM, the comparator of Fig. 2 (super-resolution
 * only): each iteration solves the inversion step exactly,
 * (A^T A + rho I) x = A^T y + rho (v - u), by cg_iters conjugate-gradient
 * steps warm-started at the current x (no box projection; lo, hi and gamma
 * are not used), then v = W(x + u) with the same weight schedule as
 * ladmm_solve and u <- u + x - v.  residuals: device [iters][2] or NULL.
 * Synchronises the stream before returning. */
int admm_cg_solve(const ladmm_operator* op, const ladmm_params* p, int cg_iters, float* x, float* v,
                  float* u, float* residuals, void* stream);

/* Reverse mode through iteration k of Algorithm 1 (unrolled differentiation;
 * not in the paper: the chain rule through the x-step, the projection, the
 * denoiser and the dual update).  Inputs: the iteration's guide (z_k while
 * k <= freeze_after, else z_{freeze_after}), the state before the iteration
 * (x_prev, v_prev, u_prev) and x_k, z_k = x_k + u_prev after it -- all device
 * n1*n2.  In/out: xbar, vbar, ubar hold the adjoints of (x_k, v_k, u_k) on
 * entry and of (x_prev, v_prev, u_prev) on return.  gacc: device n1*n2
 * accumulator of the frozen guide's adjoint (required when k > freeze_after;
 * it is added into z's adjoint at k = freeze_after).  dparams: device
 * float[2], incremented by the explicit derivative with respect to rho and by
 * the derivative with respect to the bandwidth h.  The weights are rebuilt
 * from the guide (checkpointing: nothing per iteration is kept besides the
 * states).  Returns without synchronising.  The library's reverse-pass
 * workspace of the device (grow-only; allocated on first use and when a
 * larger image arrives) is shared with ladmm_solve_backward, so calls of the
 * two on one device must not overlap in time. */
int ladmm_step_backward(const ladmm_operator* op, const ladmm_params* p, int k, const float* guide,
                        const float* x_prev, const float* v_prev, const float* u_prev,
                        const float* x_k, const float* z_k, float* xbar, float* vbar, float* ubar,
                        float* gacc, float* dparams, void* stream);

/* All iterations in reverse from the checkpoints written by ladmm_solve
 * ([iters][4][n1*n2]: x, v, u, z after each iteration) and the initial state
 * (x0, v0, u0).  xbar, vbar, ubar: adjoints of the final (x, v, u) on entry,
 * of (x0, v0, u0) on return.  dinit: NULL or device n1*n2, set to
 * xbar + vbar, the adjoint of the initial image when the iterations start from
 * x0 = v0 (u0 fixed), as Algorithm 1 does.  dparams: device float[4],
 * overwritten: [0] the explicit derivative with respect to rho (x-steps),
 * [1] the derivative with respect to the bandwidth h, [2] dL/dlambda,
 * [3] dL/drho.  With h <= 0 in the params (h = sqrt(lambda / rho)),
 * [2] = [1] h / (2 lambda) and [3] = [0] - [1] h / (2 rho); with h > 0,
 * [2] = 0 and [3] = [0].  The weights of the frozen iterations are built once
 * from z_{freeze_after}; each reverse step re-applies them to its z_k.
 * Returns without synchronising; workspace as for ladmm_step_backward. */
int ladmm_solve_backward(const ladmm_operator* op, const ladmm_params* p, const float* x0,
                         const float* v0, const float* u0, const float* checkpoints, float* xbar,
                         float* vbar, float* ubar, float* dinit, float* dparams, void* stream);

/* out = A x (super-resolution operator only; out is the low-resolution
 * grid) -- used to synthesise observations and by tests. */
int ladmm_apply_forward(const ladmm_operator* op, const float* x, float* out, void* stream);

/* g = grad f(x) for either operator (device, n1*n2). */
int ladmm_gradient(const ladmm_operator* op, const float* x, float* g, void* stream);

/* Largest eigenvalue of A^T A by `iters` power iterations from a fixed
 * start (super-resolution only).  Synchronous; *out is a host float. */
int ladmm_operator_norm2(const ladmm_operator* op, int iters, float* out, void* stream);

const char* dsnlm_last_error(void);

/* ----------------------------------------------------------------------- */
/* Instrumentation.  While enabled, every kernel launch of the library is    */
/* bracketed by HIP events recorded on its launch stream (not inside a graph */
/* capture), so callers can read per-kernel device time without a profiler.  */
typedef enum {
    DSNLM_K_PASS_A = 0,     /* sweep: row sums of step S1 -> c              */
    DSNLM_K_PASS_B = 1,     /* sweep: step-S2 row sums, B', max m           */
    DSNLM_K_APPLY = 2,      /* sweep: B' with built weights                 */
    DSNLM_K_EPILOGUE = 3,   /* y = x + B'/m                                 */
    DSNLM_K_BWD_PREP = 4,   /* backward: reductions before the sweeps       */
    DSNLM_K_PASS_C = 5,     /* backward sweep: input-gradient sums          */
    DSNLM_K_PASS_D = 6,     /* backward sweep: guide and bandwidth sums     */
    DSNLM_K_BWD_TAIL = 7,   /* backward: fold and final reductions          */
    DSNLM_K_LADMM = 8,      /* forward-model, gradient and update kernels   */
    DSNLM_K_HALF_AUX = 9,   /* half-window sweeps: factor prep and gather   */
    DSNLM_K_COUNT = 10
} dsnlm_kernel_kind;

int dsnlm_profile_enable(int on);
/* Total device milliseconds and number of launches of `kind` since the last
 * reset (waits for the recorded events). */
int dsnlm_profile_query(int kind, double* total_ms, int* launches);
int dsnlm_profile_reset(void);

/* ----------------------------------------------------------------------- */
/* Autotuning of the window sweeps (not in the paper: launch configuration).
 * Two tables steer the launches.  (1) Every sweep kind has several compiled
 * schedules ("variants"); a table keyed by (kind, S <= 12 or not, P) picks
 * the one launched.  kind: 0 = pass A, 1 = pass B (build and fused forward),
 * 2 = apply with built weights, 3 = backward input-gradient sweep; variant
 * 0-2 = full-window schedules, 3 = half window (the default).  (2) A
 * single-image half-window sweep splits each 32 x 64 tile's shifts into
 * `groups` equal contiguous ranges, one block each, so that a small image
 * fills the GPU; a table keyed by (S <= 12 or not, P, image size class by
 * its number of 32 x 64 tiles: <= 16, 32, 64, 128, 256, 512, more) gives the
 * count (0 = the default: 8 groups up to 64 tiles, 4 up to 256, 3 up to
 * 512, then none).
 * Batched launches never split.  Changing an entry changes the order of the
 * FP32 additions, not the result beyond rounding.
 * If the environment variable DSNLM_TUNE_CACHE names a file, the tables are
 * read from it on first use and written back by dsnlm_tune. */
int dsnlm_tune_set(int kind, int S, int P, int variant);
int dsnlm_tune_get(int kind, int S, int P, int* variant);
/* Set the shift groups (0..8; 0 = the rule) for images of the size class of
 * n1 x n2 at S, P; get the count an n1 x n2 image at S, P is launched with. */
int dsnlm_tune_set_groups(int n1, int n2, int S, int P, int groups);
int dsnlm_tune_get_groups(int n1, int n2, int S, int P, int* groups);
/* Time, on an n1 x n2 image (guide: device, the image used for timing),
 * `reps` launches of every variant of every kind and keep the fastest; then,
 * when the forward runs on the half window, time the single-image forward
 * plus one frozen apply for each shift-group count in {1, 2, 3, 4, 5, 6, 8}
 * and keep the fastest for this size class.  Synchronous; allocates a
 * temporary handle. */
int dsnlm_tune(const float* guide, int n1, int n2, int S, int P, float h, int reps, void* stream);

/* Measured peak of one rate on the current device, used as a roofline
 * denominator: kind 0 = FP32 FMA throughput in FLOP/s (2 per FMA, non-packed
 * VALU), 1 = v_exp_f32 throughput in exp/s, 2 = HBM copy bandwidth in bytes/s
 * (1 GiB read + 1 GiB written per launch), 3 = LDS read bandwidth in bytes/s
 * summed over the chip (conflict-free 16-byte reads).  Synchronous; allocates 2 GiB for
 * kind 2. */
int dsnlm_peak_probe(int kind, double* rate, void* stream);

/* Library version string. */
const char* dsnlm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DSNLM_H */
