/*
 * sadmm.h -- C ABI of the MI355X sharing-ADMM radar imaging engine.
 *
 * Problem (Sec. II, eq. (1); Sec. III, eq. (2)).  Q radar sensors observe one
 * scene of N pixels.  Sensor q measures y_q = A_q x_q + w_q in C^{KM}, with
 * A_q in C^{KM x N} (K fast-time samples times M receive antennas) and x_q the
 * scene's reflectivity as seen by sensor q.  The engine solves
 *
 *   min  sum_q [ mu/2 ||y_q - A_q x_q||^2 + gamma/2 ||x_q||^2 ]
 *        + lambda ||sum_q x_q||_1
 *
 * by sharing ADMM (eq. (3)): per-sensor ridge x-updates through a cached
 * factor of (c/mu) I + Ahat_q Ahat_q^H (Woodbury form, c = beta + gamma), a
 * global soft-threshold update of the image z, and a dual update.  With
 * `prune` set, the selector update of eq. (3) (subroutine SSC, Alg. 1)
 * removes pixels whose mean change over the last Kp iterations falls below
 * eps_p, once the primal residual meets its tolerance; removed pixels are
 * frozen at their last value.  The returned image is z, the global image at
 * the scale of the average sub-image (1/Q) sum_q x_q.
 *
 * Conventions
 *   - Every call returns an sadmm_status (0 = success).  No exception or
 *     abort crosses the ABI; sadmm_last_error() gives a message for the last
 *     failing call on a handle.
 *   - Complex buffers are interleaved (re, im) in the sadmm_dtype given.
 *     Operators are column-major: column n (pixel n) holds KM contiguous
 *     entries, row index m*K + k; consecutive columns are `ld` entries apart.
 *   - Pointers flagged `on_device` are HIP device pointers on the handle's
 *     device; others are host pointers.  The caller owns every buffer it
 *     passes; the engine copies inputs (converting to its storage precision)
 *     before the call returns, and writes outputs into caller buffers.
 *   - A handle is used by one host thread at a time and issues all work on
 *     params.stream (a hipStream_t, 0 = the null stream).  Calls return after
 *     their work on that stream has completed.
 */
#ifndef SADMM_H
#define SADMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sadmm_s* sadmm_t;
typedef struct sadmm_cnn_s* sadmm_cnn_t;

typedef enum {
  SADMM_OK = 0,
  SADMM_E_ARG = -1,      /* null pointer, out-of-range value */
  SADMM_E_SHAPE = -2,    /* sizes inconsistent with the handle */
  SADMM_E_STATE = -3,    /* call order (e.g. solve before every operator is set) */
  SADMM_E_HIP = -4,      /* a HIP runtime call failed */
  SADMM_E_NOMEM = -5,    /* device allocation failed */
  SADMM_E_NUMERIC = -6   /* non-finite value, or a factor lost positive definiteness */
} sadmm_status;

typedef enum { SADMM_C128 = 0, SADMM_C64 = 1 } sadmm_dtype;

/* Storage and arithmetic of the operator.  FP64: complex128 storage and FP64
 * arithmetic throughout.  FP32: complex64 storage, FP32 arithmetic, FP64 factor
 * build.  FP16P / BF16P: operator stored as separate real and imaginary half /
 * bfloat16 planes per column, FP32 arithmetic, FP64 factor build.
 * MATRIX_FREE: no operator entries are stored; every product regenerates the
 * LFM steering entries of eq. (1) from per-pixel phase records (an FP64 phase
 * fraction and FP32 complex exponential every 8 rows, FP32 rotation by the
 * per-sample phase step in between); operators must be given by
 * sadmm_set_operator_geometry. */
typedef enum {
  SADMM_ST_FP64 = 0,
  SADMM_ST_FP32 = 1,
  SADMM_ST_FP16P = 2,
  SADMM_ST_BF16P = 3,
  SADMM_ST_MATRIX_FREE = 4
} sadmm_storage;

typedef struct {
  int32_t Q, K, M, N;         /* sensors, fast-time samples, Rx antennas, pixels */
  double mu, beta, gamma;     /* data weight, ADMM penalty, per-sensor ridge (> 0) */
  double lambda;              /* absolute l1 weight on sum_q x_q */
  double eps_abs, eps_rel;    /* residual tolerances (Boyd Sec. 3.3.1 form) */
  int32_t max_iter;           /* iteration cap (>= 1) */
  int32_t stop;               /* 1: stop at convergence; 0: run exactly max_iter */
  int32_t check_every;        /* iterations queued between host status reads (>= 1) */
  int32_t prune;              /* 0: plain SADMM; 1: accelerated (SSC, Alg. 1) */
  int32_t Kp;                 /* SSC window (iterations), 1..64 */
  double eps_p;               /* SSC tolerance on the mean |change| */
  int32_t prune_mode;         /* 0: freeze eliminated pixels; 1: zero them */
  int32_t kkt;                /* 1: a solve that starts from a selector with
                                 eliminated pixels (caller mask or CNN) re-checks,
                                 after convergence, every eliminated pixel (the
                                 selector's and SSC's) against the optimality
                                 condition and reinstates violators; at most 8
                                 rounds, after which remaining violations end the
                                 solve with status 3.  SSC's eliminations in a
                                 solve that starts from the full image are Alg. 1
                                 as the paper gives it and are not judged */
  double kkt_tol;             /* reinstate eliminated pixel n of sensor q when
                                 |g_qn| > kkt_tol * lambda (lambda = 0: kkt_tol),
                                 g_q = mu A_q^H (A_q x_q - y_q) + gamma x_q + beta u
                                 (0 at the optimum); default 1e-2 */
  int32_t storage;            /* sadmm_storage */
  int32_t reuse_factor;       /* 1: a later solve reuses a factor built for the same
                                 starting selector; 0: every solve rebuilds it */
  int32_t gram;               /* Gram Ahat Ahat^H of a factor build.  0 (default): for
                                 FP32 / FP16P / BF16P / MATRIX_FREE storage, an exact
                                 integer product on the int8 16x16x64 matrix
                                 instruction of the operator rounded to 30 bits below
                                 each row's largest magnitude (FP64 storage always
                                 takes path 1); 1: FP64 matrix instructions on the
                                 stored values; 2: the same integer product as 0 on
                                 the int8 32x32x32 instruction (identical results,
                                 slower; a cross-check) */
  int32_t direct;             /* x-update form of a sensor whose active set N_q falls
                                 below the per-iteration bytes crossover (2.41 KM for
                                 FP64 storage, 1.62 KM for FP32, 1.28 KM for 16-bit,
                                 KM matrix-free): 0 (default) switches to the direct
                                 (mu Ahat^H Ahat + cI)^{-1} of order N_q, 1 keeps the
                                 Woodbury form (Sec. III solves the N_q system) */
  int32_t refine_every;       /* FP16P / BF16P storage only, operator set from the
                                 geometry: at iterations 2, 4, 8, ... (the spacing
                                 doubling up to refine_every, then every
                                 refine_every iterations; a scene of a batch that
                                 halted in between corrects at the first status
                                 read at or after that) the
                                 correction g = mu (A^H (y - A x) - Ahat^H (y' - Ahat x))
                                 of the stored operator Ahat toward the accurate A
                                 (FP32 entries regenerated as in MATRIX_FREE) enters
                                 the x-update, whose fixed point becomes that of A.
                                 When the stop test passes on a correction taken at
                                 an earlier x, g is retaken at the converged x and
                                 the solve stops only if the x-update moves by at
                                 most eps_pri under the new g (the change of
                                 (mu Ahat^H Ahat + cI)^{-1} g over the active
                                 pixels), else it iterates on.  With pruning, SSC
                                 judges only iterates of a settled corrected
                                 problem: it eliminates nothing until a correction
                                 has moved the x-update by at most eps_pri (or by
                                 at most 1e-5 of the iterate norm in eps_pri, the
                                 FP32 floor of the correction), and its
                                 K_p-window starts after the last correction that
                                 moved it by more.  0 (default): off */
  int32_t nonneg;             /* 1: the image is a non-negative magnitude (Sec. II):
                                 z = max(Re(xbar + u) - lambda / beta, 0) instead
                                 of the complex soft threshold.  With a real
                                 stacked operator (sadmm_stack_real) and real
                                 stacked measurements, every x_q stays real.
                                 0 (default): complex image */
  int32_t balance_every;      /* residual balancing (Boyd et al. 2011, Sec. 3.4.1):
                                 after every balance_every-th iteration that has not
                                 converged, beta is multiplied by balance_tau when
                                 r > balance_mu s and divided by it when
                                 s > balance_mu r; the scaled dual u is divided by
                                 the same factor (beta u unchanged) and every factor
                                 is rebuilt for c = beta + gamma (gamma, which fixes
                                 the problem, stays).  Each later solve starts from
                                 the beta given here.  0 (default): off */
  double balance_mu;          /* > 1 (default 10) */
  double balance_tau;         /* > 1 (default 2) */
  void* stream;               /* hipStream_t */
} sadmm_params;

typedef struct {
  int32_t iters;              /* iterations run */
  int32_t status;             /* 0 converged, 1 max_iter reached, 2 NMSE target reached,
                                 3 converged on the restricted problem but the
                                 optimality re-check's round cap left violations */
  int32_t prune_events;       /* iterations at which SSC removed pixels */
  int32_t reinstated;         /* pixels put back by the optimality re-check */
  int32_t refactors;          /* full factor rebuilds after the start (Woodbury factor
                                 or direct-form inverse) */
  int32_t updates;            /* low-rank factor up/down-dates */
  double r, s, eps_pri, eps_dual;   /* residuals of the last iteration */
  double max_active_frac;     /* max_q N_q / N at the end */
  double nmse;                /* NMSE of z vs the reference image, if one is set */
  int32_t direct_sensors;     /* sensors whose x-update is in the direct form at the end */
  int32_t pad;
} sadmm_info;

/* Fills *p with defaults: mu = beta = gamma = 1, eps_rel = 1e-4, Kp = 5,
 * eps_p = 1e-5, storage FP32, stop = 1, check_every = 8, kkt_tol = 1e-2,
 * reuse_factor = 1. */
void sadmm_default_params(sadmm_params* p);

/* Creates a handle on the current HIP device.  Allocates all per-problem
 * device memory sized for Q, K*M and N.  Errors: E_ARG on invalid params. */
int sadmm_create(const sadmm_params* p, sadmm_t* out);

/* Creates a handle that borrows the operators A_q and factors W_q of src
 * (frames of one array geometry: the same eq. (1) operator, different
 * measurements).  It allocates only its own state (x_q, z, u, y, data terms).
 * Requirements: same Q, K, M, N, storage, mu, beta, gamma as src; plain SADMM
 * (prune = 0, kkt = 0 on both handles); src has no pixel selector and borrows
 * from no one.  set_operator* and set_active_mask on the new handle return
 * E_STATE.  src must outlive every handle created from it; a later
 * set_operator on src changes the operator of all of them.  A solve_batch
 * whose handles all use one FP32 operator (src and/or its borrowers, 2..64
 * scenes) runs the forward and adjoint products of all scenes as
 * multi-right-hand-side products on FP32 matrix instructions.
 * Errors: E_ARG (message from sadmm_last_error(NULL)). */
int sadmm_create_shared(const sadmm_params* p, sadmm_t src, sadmm_t* out);

/* Operator of sensor q (eq. (1)): A, KM x N column-major with leading
 * dimension ld >= KM, complex128 or complex64.  Copied and converted to the
 * storage precision.  Invalidates the factor of sensor q. */
int sadmm_set_operator(sadmm_t h, int32_t q, const void* A, int32_t dtype,
                       int64_t ld, int32_t on_device);

/* Operator of sensor q generated on the device from the LFM geometry of
 * eq. (1): A[m*K+k, n] = exp(-j 2 pi f_k tau_{m,n}), f_k = f0 + bw*k/K,
 * tau_{m,n} = (|tx - p_n| + |rx_m - p_n|)/c.  tx_xy: 2 doubles; rx_xy: 2*M
 * doubles; pix_xy: 2*N doubles (host pointers).  The phase f_k*tau is reduced
 * modulo one cycle in FP64 before the complex exponential. */
int sadmm_set_operator_geometry(sadmm_t h, int32_t q, const double* tx_xy,
                                const double* rx_xy, const double* pix_xy,
                                double f0, double bw);

/* Initial selector of sensor q (eq. (3), P_q at the first iteration):
 * mask[n] = 1 keeps pixel n active, 0 eliminates it from the start (frozen at
 * x = 0).  Host pointer, N bytes.  Persists for later solves until reset by
 * passing mask = NULL (all active). */
int sadmm_set_active_mask(sadmm_t h, int32_t q, const uint8_t* mask);

/* Optional reference image x_ref (N complex): the NMSE ||z - x_ref||^2 /
 * ||x_ref||^2 is recorded each iteration, and when nmse_target > 0 the solve
 * stops at the first iteration with NMSE <= nmse_target (info.status = 2).
 * Pass x_ref = NULL to clear. */
int sadmm_set_reference(sadmm_t h, const void* x_ref, int32_t dtype,
                        int32_t on_device, double nmse_target);

/* Solves for measurements y (Q x KM complex, sensor-major).  Runs from X = 0,
 * z = 0, u = 0 with the selectors set by sadmm_set_active_mask.  Builds or
 * reuses the per-sensor factors.  info may be NULL.  Errors: E_STATE when an
 * operator is missing, E_NUMERIC on a non-finite residual. */
int sadmm_solve(sadmm_t h, const void* y, int32_t dtype, int32_t on_device,
                sadmm_info* info);

/* Solves S independent problems (handles hs[0..S-1], all with the same
 * storage; any sizes, sensor counts, parameters and selectors) in one
 * iteration loop: each per-iteration kernel is launched once for every scene
 * of the batch, one iteration is captured as a hipGraph and replayed, and each
 * scene halts on its own (converged, max_iter, NMSE target, numeric error);
 * pixel eliminations and re-checks are applied per scene.  ys[i] is the
 * measurement buffer of scene i (as for sadmm_solve); infos may be NULL or
 * hold S entries.  Results are read per handle afterwards. */
int sadmm_solve_batch(sadmm_t* hs, int32_t S, const void* const* ys, int32_t dtype,
                      int32_t on_device, sadmm_info* infos);

/* Global image z (N complex) of the last solve. */
int sadmm_get_image(sadmm_t h, void* xG, int32_t dtype, int32_t on_device);

/* Sub-image x_q (N complex) of sensor q, eliminated pixels included. */
int sadmm_get_sensor_image(sadmm_t h, int32_t q, void* xq, int32_t dtype,
                           int32_t on_device);

/* Scaled dual u (N complex) of the last solve; beta*u is the multiplier of the
 * sharing constraint (eq. (3), row 3) and satisfies |beta*u_j| <= lambda at
 * the optimum. */
int sadmm_get_dual(sadmm_t h, void* u, int32_t dtype, int32_t on_device);

/* Factor W_q = ((c/mu) I + Ahat_q Ahat_q^H)^{-1} of sensor q as last built or
 * updated (complex128, KM x KM column-major, host buffer of KM*KM entries);
 * *n receives KM.  For a sensor in the direct form (params.direct) it is built
 * here for the current active set.  Diagnostic: lets callers check the factor
 * directly. */
int sadmm_get_factor(sadmm_t h, int32_t q, void* W, int32_t* n);

/* Final selector of sensor q: mask[n] = 1 if pixel n is active (host, N bytes). */
int sadmm_get_active_mask(sadmm_t h, int32_t q, uint8_t* mask);

/* Active pixel indices of sensor q in ascending order (host, capacity N
 * int32); *count receives N_q. */
int sadmm_get_active_indices(sadmm_t h, int32_t q, int32_t* idx, int32_t* count);

/* Per-iteration history of the last solve (host buffers of capacity cap):
 * which = 0 r, 1 s, 2 eps_pri, 3 eps_dual, 4 nmse, 5 max_q N_q / N,
 * 6 change of the x-update when a stale 16-bit correction was retaken at a
 * passed stop test (0 at other iterations; compared with eps_pri),
 * 7 beta in force after the iteration (residual balancing),
 * 8 move of the x-update caused by each 16-bit correction, at the iteration
 * that took it (0 at other iterations).
 * *count receives the number of iterations recorded. */
int sadmm_get_history(sadmm_t h, int32_t which, double* out, int32_t cap,
                      int32_t* count);

/* Matched-filter images |A_q^H y_q| (Q x N doubles, host) of the given
 * measurements, over all pixels (the CNN input and the back-projection image). */
int sadmm_matched_filter(sadmm_t h, const void* y, int32_t dtype, int32_t on_device,
                         double* out);

/* Tile autotuner of the forward product (columns per work-group, from
 * 64, 128, 256, 512, 1024; images of 4096 pixels or more from 256 up; not
 * part of the method, only of its speed).  For each
 * width it runs min(iters, params.max_iter) plain iterations of this
 * handle's problem on the measurements y twice (as sadmm_solve, with
 * stopping, elimination, re-check, refinement and balancing off; the factor
 * is built once), times the second run with device events, keeps the
 * fastest width for the handle and records it for the key (storage, rows,
 * power-of-two bucket of N): handles created later in this process with the
 * same key start from it.  *chunk receives the width; iters = 0 only
 * reports the handle's current width.  The parameters are unchanged
 * afterwards and the next solve starts afresh; results of later solves
 * differ from the untuned width's only by summation order.  SADMM_E_ARG for
 * iters = 1 or < 0 and for handles that share an operator. */
int sadmm_autotune(sadmm_t h, const void* y, int32_t dtype, int32_t on_device, int32_t iters,
                   int32_t* chunk);

/* Back-projection image of Sec. IV (Fig. 1): |sum_q A_q^H y_q| per pixel,
 * the coherent sum over the sensors of each sensor's adjoint applied to its
 * measurements (y: Q x KM complex, sensor-major, in dtype; on_device selects
 * a device pointer).  out: N doubles, host.  Allocates a Q x N complex128
 * scratch for the call (and a staging copy of host measurements). */
int sadmm_back_projection(sadmm_t h, const void* y, int32_t dtype, int32_t on_device, double* out);

/* Rendering of an image on a range_db dynamic range (Sec. IV shows every
 * image on 30 dB): with r = |x_n| / max_m |x_m|, level
 * floor(255 (1 + 20 log10(r) / range_db)) clipped to [0, 255], 0 where
 * r < 10^(-range_db / 20) or the image is all zero; decided as the number of
 * thresholds 10^((L/255 - 1) range_db / 20) * max |x|, L = 1..255, at or
 * below |x_n|.  img: n doubles (is_complex = 0, magnitudes or real values)
 * or n interleaved complex128 (is_complex = 1); levels: n bytes; both host
 * or both device (on_device) pointers owned by the caller.  Runs on the given
 * hipStream_t and returns after it; allocates small buffers (and staging for
 * host pointers). */
int sadmm_render_db(const void* img, int32_t is_complex, int64_t n, double range_db, int32_t on_device,
                    uint8_t* levels, void* stream);

/* Wall time of the last solve on its stream (HIP events), milliseconds:
 * which = 0 whole solve, 1 factor builds/updates, 2 iterations. */
int sadmm_get_timing(sadmm_t h, int32_t which, double* ms);

/* ---------------------------------------------------------------------------
 * Learned pixel elimination.  A small CNN maps the Q matched-filter images
 * |A_q^H y_q| (each H x W, pixel n = i*W + j, scaled by their common maximum)
 * to a per-pixel probability that the pixel can be eliminated from every
 * sensor's sub-problem before the solve (an initial selector P_q of eq. (3)).
 * Layers: four 3x3 zero-padded convolutions Q -> C -> C -> C -> 1 with ReLU
 * after the first three and a sigmoid output; FP32.  Parameters are one flat
 * FP32 vector: W1 (C x Q x 3 x 3), b1 (C), W2 (C x C x 3 x 3), b2, W3, b3,
 * W4 (1 x C x 3 x 3), b4 (1).  Training minimises the pixel-averaged weighted
 * binary cross-entropy (positive pixels weighted by pos_weight) with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  Training runs in FP32; inference
 * (sadmm_cnn_forward and the solver's selector) runs by default on the FP16
 * matrix instructions with FP32 accumulation (sadmm_cnn_set_half).  The CNN only proposes eliminations: the
 * solver's optimality re-check (params.kkt) reinstates false ones.
 * ------------------------------------------------------------------------- */

/* Creates a CNN for Q input channels, C hidden channels (C, Q <= 32) and H x W
 * images on the given hipStream_t.  Parameters start at zero. */
int sadmm_cnn_create(int32_t Q, int32_t C, int32_t H, int32_t W, void* stream,
                     sadmm_cnn_t* out);
/* Number of FP32 parameters. */
int64_t sadmm_cnn_param_count(sadmm_cnn_t c);
/* Copy parameters in / out (host buffers of param_count floats); setting them
 * resets the Adam state. */
int sadmm_cnn_set_params(sadmm_cnn_t c, const float* params, int64_t count);
int sadmm_cnn_get_params(sadmm_cnn_t c, float* params, int64_t count);
/* Probability map (H*W floats) of the input x (Q x H x W floats). */
int sadmm_cnn_forward(sadmm_cnn_t c, const float* x, int32_t x_on_device, float* prob,
                      int32_t prob_on_device);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the probability
 * map of sadmm_cnn_forward for an H x W input of any size up to 512 x 512
 * pixels (H * W <= 262144, else SADMM_E_SHAPE), with the handle's parameters
 * and arithmetic (sadmm_cnn_set_half).  x (Q x H x W floats) and prob (H * W
 * floats) are device pointers owned by the caller.  The activations live in
 * a fixed 65 MiB array of the library, one per GPU, held until the process
 * ends; the call allocates and frees nothing, enqueues its kernels on the
 * handle's stream and returns without synchronising (prob is ready when the
 * stream reaches that point).  Every call on one GPU uses that GPU's array:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must be serialised by the caller. */
int sadmm_cnn_forward_noalloc(sadmm_cnn_t c, const float* x, int32_t H, int32_t W, float* prob);
/* Inference arithmetic: on = 1 (default) FP16 operands (activations and
 * weights rounded to binary16) on the 16x16x16 matrix instruction with FP32
 * accumulation; 0 = FP32 direct convolutions (the training forward). */
int sadmm_cnn_set_half(sadmm_cnn_t c, int32_t on);
/* Loss and gradient (host buffer of param_count floats) for input x and
 * target map (H*W floats, 1 = eliminate). */
int sadmm_cnn_gradients(sadmm_cnn_t c, const float* x, const float* target, int32_t on_device,
                        float pos_weight, float* grads, double* loss);
/* One Adam step on (x, target); *loss receives the loss before the step. */
int sadmm_cnn_train_step(sadmm_cnn_t c, const float* x, const float* target, int32_t on_device,
                         float pos_weight, float lr, double* loss);
void sadmm_cnn_destroy(sadmm_cnn_t c);
const char* sadmm_cnn_last_error(sadmm_cnn_t c);

/* Attach a CNN to a solver (NULL detaches).  Each later solve computes the
 * matched-filter images of its y, runs the CNN, and eliminates from every
 * sensor, before the factor build, the pixels whose probability is >=
 * threshold (combined with any mask set by sadmm_set_active_mask).  The CNN's
 * image size must be N pixels and its input channels Q; it must use the
 * solver's stream.  Eliminated pixels are frozen at x = 0.  The solver must
 * have kkt = 1 (else SADMM_E_ARG): the optimality re-check judges every
 * learned elimination after convergence and reinstates false ones. */
int sadmm_set_pruning_cnn(sadmm_t h, sadmm_cnn_t cnn, double threshold);

/* Kernel classes timed when profiling is on. */
enum {
  SADMM_KC_GRAM = 0,     /* Gram Ahat Ahat^H of a factor build (matrix-instruction kernel;
                            one launch per 8192-column chunk on the integer path) */
  SADMM_KC_INVERSE = 1,  /* Cholesky, triangular inverse and W = X^H X */
  SADMM_KC_FWD = 2,      /* forward product Ahat v (+ partial-sum reduction) */
  SADMM_KC_WPROD = 3,    /* W t */
  SADMM_KC_XUPD = 4,     /* adjoint product Ahat^H w with the fused x-update */
  SADMM_KC_PIXEL = 5,    /* image/dual update, residuals, SSC check */
  SADMM_KC_CNN = 6,      /* matched filter + CNN inference before a solve */
  SADMM_KC_SLICE = 7,    /* integer Gram: row scales and digit planes of the operator */
  SADMM_KC_COUNT = 8
};

/* level 0: off.  level 1: HIP events around the factor build and update
 * launches (GRAM, INVERSE, CNN); iterations still run as a replayed hipGraph.
 * level 2: also events around every iteration stage (FWD, WPROD, XUPD, PIXEL),
 * launched directly instead of from the graph.  Resets the accumulated times. */
int sadmm_set_profiling(sadmm_t h, int32_t level);

/* Launch count, summed event time (ms) and algorithmic work of a kernel class
 * since the last sadmm_set_profiling call.  Work is in flops for GRAM and
 * INVERSE (complex multiply-add = 8 flops; Hermitian product counts one
 * triangle; the integer Gram reports the same FP64-equivalent count) and in
 * bytes for the others (operator, factor and state bytes each launch must move
 * at least once). */
int sadmm_get_kernel_stats(sadmm_t h, int32_t kclass, int32_t* launches, double* total_ms,
                           double* work);

/* Real form of the model for a real unknown (Sec. II, x_q the magnitude):
 * |y - A x|^2 = |[Re y; Im y] - [Re A; Im A] x|^2.  Writes the stacked real
 * matrix [Re S; Im S] of the complex rows x cols column-major matrix S (dtype,
 * leading dimension ld >= rows) as complex128 with zero imaginary parts,
 * (2 rows) x cols column-major, leading dimension 2 rows, into dst.  Both are
 * caller-owned device pointers; the work runs on the given hipStream_t and
 * the call returns after it.  An operator A_q (KM x N) becomes one of 2 KM
 * rows; the measurements (Q x KM, sensor-major) are the KM x Q matrix with
 * ld = KM.  A handle for the stacked problem is created with K * M = 2 KM
 * (for example K doubled). */
int sadmm_stack_real(const void* src, int32_t dtype, int64_t rows, int64_t cols, int64_t ld, void* dst,
                     void* stream);

/* ---------------------------------------------------------------------------
 * Roofline probes (no part of the method): the device's own bandwidth and
 * matrix throughput, the denominators measured beside the published peaks.
 * ------------------------------------------------------------------------- */

/* Bandwidth over `bytes` (a multiple of 16) of device memory, `reps` passes
 * after one untimed pass on the given hipStream_t; *ms receives the mean time
 * of one pass (HIP events).  kind 0: copy src -> dst with non-temporal 16-byte
 * loads and stores (bandwidth = 2 * bytes / time); kind 1: read src only
 * (bandwidth = bytes / time; dst unused, may be NULL).  src and dst are
 * caller-owned device pointers, 16-byte aligned; kind 1 allocates and frees a
 * small result buffer. */
int sadmm_probe_bandwidth(int32_t kind, const void* src, void* dst, int64_t bytes, int32_t reps,
                          void* stream, double* ms);

/* Register-only matrix-instruction loop over every compute unit, `iters`
 * rounds of independent accumulators: kind 0 = int8 16x16x64 (8 waves per
 * SIMD), 1 = FP64 16x16x4 (8 waves per SIMD), 2 = int8 32x32x32 (4 waves per
 * SIMD).  *ops_per_s receives the achieved operations per second (multiply
 * and add counted separately).  Allocates and frees a small result buffer. */
int sadmm_probe_mfma(int32_t kind, int32_t iters, void* stream, double* ops_per_s);

void sadmm_destroy(sadmm_t h);
/* Message of the last failing call on h; with h = NULL, of the last failed
 * sadmm_create on this thread. */
const char* sadmm_last_error(sadmm_t h);

#ifdef __cplusplus
}
#endif

#endif /* SADMM_H */
