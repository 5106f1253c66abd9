// Per-iteration kernels of sharing ADMM (eq. (3)) and the SSC check (Alg. 1).
#pragma once
#include <functional>

#include "common.h"

// Per-sensor view used by the iteration kernels (device array, one per sensor).
struct SensorDesc {
  const void* A;       // active columns Ahat_q (compacted, ascending pixel order)
  const void* Afull;   // full operator A_q
  const int* J;        // active pixel indices, nq entries (ascending)
  const void* xy;      // Ahat^H W y'_q, nq complex (compute precision): the
                       // data part of the x-update, (mu Ahat^H Ahat + cI)^{-1} mu Ahat^H y'
  const void* W;       // KMp x KMp factor, compute precision, ld = KMp
  const cd* W64;       // the same factor in complex128
  int64_t lda;         // column stride of A and Afull (storage slots)
  int nq;
  int direct;          // 1: x-update in the direct form x = F (b0 + beta v)
  const cd* F;         // direct form: (mu Ahat^H Ahat + cI)^{-1}, nq x nq, ld = fld
  const cd* b0;        // direct form: mu Ahat^H y', nq complex128
  cd* rdir;            // direct form: b0 + beta v of the current iteration (fld)
  int fld;             // leading dimension of F (multiple of 32)
  int wtri;            // 1: W is not formed; W64 holds U = X^H and X = L^{-1} (lower
                       // triangular, W = X^H X), so W v = X^H (X v)
  const cd* X;         // with wtri: X = L^{-1}, KMp x KMp, ld = KMp, zeros above the diagonal
};

// Everything the per-iteration kernels need; passed by value.
struct IterArgs {
  int Q, KMp, N, Kp;
  int chunk, nchunk;   // forward kernel: columns per work-group, chunks per sensor
  int prune, stop, nonneg;
  int bal_every;       // residual balancing period (0: off)
  double bal_mu;       // imbalance ratio
  double beta, c, tau, eps_abs, eps_rel, eps_p, inv_Q;
  double bc;           // beta / c
  double nmse_target, xref_norm2;
  const SensorDesc* sens;
  void* X;             // Q x N complex
  void* dX;            // Q x N complex, x^(k) - x^(k-1) (0 on eliminated pixels)
  void* xbar;          // N complex
  void* z;             // N complex
  void* u;             // N complex
  void* D;             // Kp x Q x N real: |x^(i) - x^(i-1)| ring
  void* tpart;         // Q x nchunk x KMp complex partial forward products
  void* t;             // Q x KMp complex
  void* w;             // Q x KMp complex
  const void* xref;    // N complex or null
  const double* yp;    // Q x KMp complex128: y'_q (measurement minus frozen pixels)
  double* wy;          // Q x KMp complex128 scratch: W_q y'_q
  double* red;         // pixel-kernel block partials (nblk x 8)
  int nblk;
  int max_iter;
  int ssc_from;        // first iteration at which SSC may eliminate (its window
                       // then lies after the latest operator correction)
  Ctl* ctl;
  double* hist;        // 6 x max_iter
  uint8_t* keep;       // Q x N: SSC keep flag per active position
  int* gone;           // Q: pixels to eliminate per sensor
  // Correction of a stored 16-bit operator toward the accurate one (null when
  // off): gfix = mu (A^H (y - A x) - Ahat^H (y' - Ahat x)) at a recent x, and
  // xfix = (mu Ahat^H Ahat + cI)^{-1} gfix, both Q x N by pixel.
  const double* gfix;  // complex128
  const void* xfix;    // compute precision
  double* ws;          // Q x KMp complex128: X v of the triangular W products
  // 1: the passes over the operator (stream_op) or over the W factors
  // (stream_w) read more than the caches keep between iterations, so their
  // loads are non-temporal
  int stream_op, stream_w;
};

// A batch of independent problems ("scenes") iterated by one launch per
// kernel: per-scene arguments in device memory, and a slot table mapping each
// work slot to (scene, sensor).  A single solve is a batch of one.
struct BatchView {
  const IterArgs* args;   // nscene entries (device)
  const int2* slots;      // nslot entries (device): x = scene, y = sensor
};
struct BatchDims {
  int nscene, nslot;
  int KMp_max, nchunk_max, N_max, nblk_max;
  int fld_max;          // largest order a sensor may take in the direct form (0: none can)
};

constexpr int FWD_THREADS = 256;
// most columns one forward work-group takes (its coefficient tile in LDS)
constexpr int MAX_CHUNK = 1024;
// Columns per wavefront of the column-dot kernels: two for stored FP32 / FP64
// entries (more waves in flight), four for 16-bit and generated entries (one
// LDS read of the staged vector serves more columns).
// Entries of the LDS copy of the vector of a column-dot kernel: stores with 8
// rows per lane keep it lane-interleaved in blocks of 512 (see sv_slot), so
// its length is KMp rounded up to 512.
template <int ST> inline int sv_len(int KMp) {
  return Store<ST>::RPT == 8 ? (KMp + 511) / 512 * 512 : KMp;
}
template <int ST> constexpr int dot_cols() {
  return (ST == ST_FP16P || ST == ST_BF16P || ST == ST_MF) ? 4 : 2;
}
// Direct-form right-hand side entries staged in LDS per pass (16 KB: within
// the share of one of eight 256-thread work-groups on a CU).
constexpr int XDIR_SEG = 1024;

// Launchers.  `st` is the operator storage (sadmm_storage), `dbl` selects FP64
// compute (only with ST_FP64).
// One iteration of every scene of a batch (all scenes share the storage st).
// The optional hook is called before (begin = true) and after each stage:
// 0 forward + partial reduce, 1 W product, 2 adjoint + x-update,
// 3 pixel update + finalize + SSC check.
constexpr int IT_NSTAGE = 4;
void launch_iteration_batch(const BatchView& b, const BatchDims& d, int st, hipStream_t s,
                            const std::function<void(int, bool)>* hook);

// Stage 3 alone (pixel update, finalize, SSC check) for every scene.
void launch_pixel_stage(const BatchView& b, const BatchDims& d, bool dbl, hipStream_t s);

// Scenes that share one FP32 operator (and so one factor, no pixel
// elimination): the forward and adjoint products of all scenes run as
// multi-right-hand-side products on the FP32 matrix instructions.
struct SharedBatch {
  int S;              // scenes (right-hand sides)
  int nch;            // pixel chunks of the forward product
  float* Vb;          // Q x N x S complex: v_q of every scene (pixel-major)
  float* Tp;          // nch x Q x KMp x S complex: forward partial sums
  cd* T64;            // Q x S x KMp: Ahat v per scene (column-major per sensor)
  cd* Wt64;           // Q x S x KMp: W (Ahat v)
  float* Wt32;        // the same as complex64 (adjoint operands)
  const void* wdesc;  // Q MmDesc products Wt = W T (device)
};
constexpr int MRHS_CHUNK = 1024;   // pixels per forward work-group
void launch_iteration_shared(const BatchView& b, const BatchDims& d, const SharedBatch& sb,
                             hipStream_t s, const std::function<void(int, bool)>* hook);

// Copies the control blocks of a batch (ptrs: nscene device pointers) into out.
void gather_ctl(Ctl* const* ptrs, Ctl* out, int nscene, hipStream_t s);
int fwd_row_tile(int st);   // rows covered by one forward work-group

// xy_q = Ahat_q^H (W_q y'_q) for the sensors in [q0, q1), FP64 arithmetic
// (rounded to the compute precision on store).
void launch_xy(const IterArgs& a, int st, bool dbl, int q0, int q1, hipStream_t s);

// Generic gathered forward product for one sensor q:
//   out += sign * sum_j coef_j * Afull[:, idx_j],   coef_j = X[q, idx_j]
// with idx = null meaning all N columns; out is complex128 KMp (e.g. y'_q).
// `tmp` holds nchunk x KMp compute-precision partials.
void launch_gather_fwd(const IterArgs& a, int st, bool dbl, int q, const int* idx, int count,
                       double sign, double* out, void* tmp, hipStream_t s);

// Optimality re-check of eliminated pixels of sensor q (idx, count):
// g = mu A[:,n]^H e + gamma X[q,n] + beta u[n] with e = A_q x_q - y_q
// (complex128, KMp); flag[j] = |g| > thr.
// g_p = mu a_p^H e + gamma x_q[idx_p] + beta u[idx_p] (e = A_q x_q - y_q) for
// the listed pixels (complex128, by list slot)
void launch_kkt_grad(const IterArgs& a, int st, bool dbl, int q, const int* idx, int count,
                     const double* e, double mu, double gamma, double* g, hipStream_t s);

// |A_q^H y_q| over all pixels for every sensor, into out (Q x N doubles).
// Correction products over every sensor (one launch per step):
//   launch_refine_fwd:  out_q += sign * A_q x_q over the active pixels J_q
//                       (active) or all N pixels, x from xsrc (Q x N compute
//                       precision) or X; tpart is the scratch; out Q x KMp c128;
//   launch_factor_vec:  out_q = W_q v_q (W Hermitian, FP64; held as W64_q, or
//                       as the triangular pair X_q^H X_q, using ws as scratch);
//   launch_refine_grad: g[q, J_q[p]] = scale (A_q^H e_q)_p, or with accumulate
//                       += it, also writing the sum in compute precision to g32;
//   launch_refine_fix:  xfix[q, J_q[p]] = cinv (g - A_q^H w_q)_p.
// e, w: Q x KMp complex128; g: Q x N complex128; g32, xfix: Q x N compute
// precision; max_nq: the largest N_q.  Sensors in the direct form are skipped
// by the W and fix steps.
void launch_refine_fwd(const IterArgs& a, int st, bool active, const void* xsrc, double sign, double* out,
                       hipStream_t s);
void launch_factor_vec(const IterArgs& a, const double* v, double* out, hipStream_t s);
void launch_refine_grad(const IterArgs& a, int st, int max_nq, const double* e, double scale,
                        bool accumulate, double* g, void* g32, hipStream_t s);
void launch_refine_fix(const IterArgs& a, int st, int max_nq, const double* w, const double* g,
                       double cinv, void* xfix, hipStream_t s);
void launch_matched_filter(const IterArgs& a, int st, bool dbl, const double* y, double* out,
                           hipStream_t s, bool cplx = false);
