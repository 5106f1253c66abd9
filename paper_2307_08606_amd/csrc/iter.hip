// Per-iteration kernels of sharing ADMM (eq. (3)) with the SSC check of Alg. 1.
//
// The x-update of eq. (3), x = (mu Ahat^H Ahat + cI)^{-1} (mu Ahat^H y' + beta v),
// is applied as
//     x = Ahat^H W y'  +  (beta/c) (v - Ahat^H W Ahat v),   W = ((c/mu) I + Ahat Ahat^H)^{-1},
// (push-through and Woodbury identities; exact in exact arithmetic).  The
// data part Ahat^H W y' is fixed between selector changes and is computed once
// in FP64; only the v-part goes through W every iteration.  Applying W to the
// whole right-hand side instead would cancel catastrophically in FP32, since
// mu Ahat^H y' lies in the row space of Ahat where W is tiny.
//
// One iteration = seven launches, each covering all Q sensors:
//   fwd      t_q = Ahat_q v_q, v_q = (x_q - xbar + z - u)[J_q]
//            (column chunks per work-group -> partial sums, no atomics)
//   reduce   t_q = sum of the chunk partials, fixed order
//   wdot     w_q = W_q t_q  (W_q Hermitian: one wavefront dot per column)
//   xupd     x_q[J_q] = xy_q + (beta/c)(v_q - Ahat_q^H w_q), fused epilogue writes
//            x_q, dx_q and |dx_q| into the SSC history ring
//   pixel    xbar, z = S_{lambda/beta}(xbar + u), u += xbar - z, and block
//            partial sums of the residual norms
//   finalize residuals r, s, eps_pri, eps_dual, stop / gate flags, history
//   ssc      zeta = mean |dx| over the ring; pixels with zeta < eps_p flagged
// Every kernel reads the device control block first and does nothing once
// the solve has halted (converged, max_iter, NMSE target, numeric error, or a
// pending pixel elimination the host must apply), so the host can queue many
// iterations ahead and synchronise rarely.
#include <algorithm>

#include "iter.h"

namespace {

template <class T> __device__ inline C2<T> ldc(const void* p, int64_t i) {
  return reinterpret_cast<const C2<T>*>(p)[i];
}
template <class T> __device__ inline void stc(void* p, int64_t i, C2<T> v) {
  reinterpret_cast<C2<T>*>(p)[i] = v;
}
template <class T> __device__ inline T habs(C2<T> v) { return hypot(v.re, v.im); }

// v_q[n] = x_q - xbar + z - u at pixel n (eq. (3), row 1, sharing form)
template <class T>
__device__ inline C2<T> shared_v(const IterArgs& a, int q, int n) {
  const C2<T> x = ldc<T>(a.X, (int64_t)q * a.N + n);
  const C2<T> xb = ldc<T>(a.xbar, n);
  const C2<T> zz = ldc<T>(a.z, n);
  const C2<T> uu = ldc<T>(a.u, n);
  return csub(cadd(csub(x, xb), zz), uu);
}

// ------------------------------------------------------------------ forward
template <int ST, bool NT = false>
__device__ inline void fwd_accumulate(const void* A, int64_t lda, const int* colidx, int p0, int np,
                                      const C2<typename Store<ST>::T>* coef, int row, int KMp,
                                      C2<typename Store<ST>::T>* acc) {
  using T = typename Store<ST>::T;
  constexpr int R = Store<ST>::RPT;
  auto step = [&](int e) {
    const int col = colidx ? colidx[p0 + e] : p0 + e;
    T re[R], im[R];
    Store<ST>::template load<NT>(col_ptr<ST>(A, lda, col), row, KMp, re, im);
    const C2<T> cf = coef[e];
#pragma unroll
    for (int r = 0; r < R; ++r) cfma(acc[r], C2<T>{re[r], im[r]}, cf);
  };
  if constexpr (ST == ST_MF) {
    // generated entries: few columns in flight keep registers (and waves) for
    // the generation arithmetic
    const double* rec0 = reinterpret_cast<const double*>(col_ptr<ST>(A, lda, colidx ? colidx[p0] : p0));
    const int K = (int)rec0[0], M = (int)rec0[1];
    if ((K & (R - 1)) == 0) {
      // the thread's 8 rows lie in one receiver: the term coef * a0 of the
      // anchor entry a0 is rotated row by row (one complex rotation and one
      // complex add per entry, against a rotation of the entry and a
      // complex multiply-add)
      const int m = row / K, k = row - m * K;
      if (m >= M) return;                     // padding rows: zero entries
#pragma unroll 2
      for (int e = 0; e < np; ++e) {
        const int col = colidx ? colidx[p0 + e] : p0 + e;
        float ar, ai, rc, rs;
        Store<ST_MF>::anchor(col_ptr<ST>(A, lda, col), m, k, M, &ar, &ai, &rc, &rs);
        const C2<T> cf = coef[e];
        T wr = fmaf(ar, cf.re, -(ai * cf.im));
        T wi = fmaf(ar, cf.im, ai * cf.re);
        acc[0].re += wr;
        acc[0].im += wi;
#pragma unroll
        for (int r = 1; r < R; ++r) {   // w <- w (rc - j rs)
          const T nr = fmaf(wr, rc, wi * rs);
          const T ni = fmaf(wi, rc, -(wr * rs));
          wr = nr;
          wi = ni;
          acc[r].re += wr;
          acc[r].im += wi;
        }
      }
      return;
    }
#pragma unroll 2
    for (int e = 0; e < np; ++e) step(e);
  } else {
#pragma unroll 8
    for (int e = 0; e < np; ++e) step(e);
  }
}

// use(i, load(i)) for i = 0 .. n-1 in index order, with the loads of G
// consecutive indices issued before their uses: a short dynamic loop of
// dependent adds otherwise waits out one memory latency per index.
template <int G, class L, class U>
__device__ inline void in_order(int n, L load, U use) {
  for (int i0 = 0; i0 < n; i0 += G) {
    decltype(load(0)) v[G];
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (i0 + j < n) v[j] = load(i0 + j);
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (i0 + j < n) use(i0 + j, v[j]);
  }
}

template <int ST>
__global__ __launch_bounds__(FWD_THREADS) void fwd_iter_kernel(BatchView bv) {
  using T = typename Store<ST>::T;
  constexpr int R = Store<ST>::RPT;
  const int2 sl = bv.slots[blockIdx.z];
  const IterArgs& a = bv.args[sl.x];
  if (a.ctl->halt) return;
  const int q = sl.y, ch = blockIdx.y;
  const SensorDesc sd = a.sens[q];
  if (sd.direct) return;   // the direct form needs no forward product
  const int p0 = ch * a.chunk;
  if (p0 >= sd.nq) return;
  const int np = min(a.chunk, sd.nq - p0);
  __shared__ C2<T> coef[MAX_CHUNK];
  for (int e = threadIdx.x; e < np; e += FWD_THREADS) {
    const int p = p0 + e;
    coef[e] = shared_v<T>(a, q, sd.J[p]);
  }
  __syncthreads();
  const int row = (blockIdx.x * FWD_THREADS + threadIdx.x) * R;
  if (row >= a.KMp) return;
  C2<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = {(T)0, (T)0};
  if (a.stream_op) fwd_accumulate<ST, true>(sd.A, sd.lda, nullptr, p0, np, coef, row, a.KMp, acc);
  else fwd_accumulate<ST, false>(sd.A, sd.lda, nullptr, p0, np, coef, row, a.KMp, acc);
  C2<T>* out = reinterpret_cast<C2<T>*>(a.tpart) + ((int64_t)q * a.nchunk + ch) * a.KMp + row;
#pragma unroll
  for (int r = 0; r < R; ++r) out[r] = acc[r];
}

template <class T>
__global__ __launch_bounds__(256) void fwd_reduce_kernel(BatchView bv) {
  const int2 sl = bv.slots[blockIdx.y];
  const IterArgs& a = bv.args[sl.x];
  if (a.ctl->halt) return;
  const int q = sl.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (a.sens[q].direct) {
    // direct form: right-hand side b0 + beta v of this iteration (all of it
    // before any x_q of the iteration is written)
    const SensorDesc sd = a.sens[q];
    if (i < sd.fld) {
      cd r = {0.0, 0.0};
      if (i < sd.nq) {
        const C2<T> v = shared_v<T>(a, q, sd.J[i]);
        r = {sd.b0[i].re + a.beta * (double)v.re, sd.b0[i].im + a.beta * (double)v.im};
        if (a.gfix) {
          const double* g = a.gfix + 2 * ((int64_t)q * a.N + sd.J[i]);
          r.re += g[0];
          r.im += g[1];
        }
      }
      sd.rdir[i] = r;
    }
    return;
  }
  if (i >= a.KMp) return;
  const int nq = a.sens[q].nq;
  const int nch = (nq + a.chunk - 1) / a.chunk;
  const C2<T>* tp = reinterpret_cast<const C2<T>*>(a.tpart) + (int64_t)q * a.nchunk * a.KMp + i;
  C2<T> s = {(T)0, (T)0};
  in_order<8>(nch, [&](int c) { return tp[(int64_t)c * a.KMp]; }, [&](int, C2<T> v) { s = cadd(s, v); });
  stc<T>(a.t, (int64_t)q * a.KMp + i, s);
}

// Gathered forward product (host-orchestrated, no halt check):
// partials of sum_j X[q, idx_j] * A[:, idx_j]
template <int ST>
__global__ __launch_bounds__(FWD_THREADS) void fwd_gather_kernel(IterArgs a, int q, const int* idx,
                                                                 int count, void* tmp) {
  using T = typename Store<ST>::T;
  constexpr int R = Store<ST>::RPT;
  const SensorDesc sd = a.sens[q];
  const int ch = blockIdx.y;
  const int p0 = ch * a.chunk;
  if (p0 >= count) return;
  const int np = min(a.chunk, count - p0);
  __shared__ C2<T> coef[MAX_CHUNK];
  for (int e = threadIdx.x; e < np; e += FWD_THREADS) {
    const int n = idx ? idx[p0 + e] : p0 + e;
    coef[e] = ldc<T>(a.X, (int64_t)q * a.N + n);
  }
  __syncthreads();
  const int row = (blockIdx.x * FWD_THREADS + threadIdx.x) * R;
  if (row >= a.KMp) return;
  C2<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = {(T)0, (T)0};
  if (a.stream_op) fwd_accumulate<ST, true>(sd.Afull, sd.lda, idx, p0, np, coef, row, a.KMp, acc);
  else fwd_accumulate<ST, false>(sd.Afull, sd.lda, idx, p0, np, coef, row, a.KMp, acc);
  C2<T>* out = reinterpret_cast<C2<T>*>(tmp) + (int64_t)ch * a.KMp + row;
#pragma unroll
  for (int r = 0; r < R; ++r) out[r] = acc[r];
}

template <class T>
__global__ __launch_bounds__(256) void gather_reduce_kernel(int KMp, int nch, const void* tmp,
                                                            double sign, double* out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= KMp) return;
  const C2<T>* tp = reinterpret_cast<const C2<T>*>(tmp) + i;
  C2<T> s = {(T)0, (T)0};
  in_order<8>(nch, [&](int c) { return tp[(int64_t)c * KMp]; }, [&](int, C2<T> v) { s = cadd(s, v); });
  out[2 * i] += sign * (double)s.re;
  out[2 * i + 1] += sign * (double)s.im;
}

// Forward products of every sensor for the correction (blockIdx.z = sensor):
// over its active pixels J_q (active = 1) or over all N pixels (active = 0),
// coefficients from xsrc (Q x N, compute precision) or from X; partial sums
// per column chunk into tpart (Q x nchunk x KMp).
template <int ST>
__global__ __launch_bounds__(FWD_THREADS) void fwd_all_kernel(IterArgs a, int active, const void* xsrc) {
  using T = typename Store<ST>::T;
  constexpr int R = Store<ST>::RPT;
  const int q = blockIdx.z, ch = blockIdx.y;
  const SensorDesc sd = a.sens[q];
  const int count = active ? sd.nq : a.N;
  const int* idx = active ? sd.J : nullptr;
  const int p0 = ch * a.chunk;
  if (p0 >= count) return;
  const int np = min(a.chunk, count - p0);
  const void* xs = xsrc ? xsrc : a.X;
  __shared__ C2<T> coef[MAX_CHUNK];
  for (int e = threadIdx.x; e < np; e += FWD_THREADS) {
    const int n = idx ? idx[p0 + e] : p0 + e;
    coef[e] = ldc<T>(xs, (int64_t)q * a.N + n);
  }
  __syncthreads();
  const int row = (blockIdx.x * FWD_THREADS + threadIdx.x) * R;
  if (row >= a.KMp) return;
  C2<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = {(T)0, (T)0};
  if (a.stream_op) fwd_accumulate<ST, true>(sd.Afull, sd.lda, idx, p0, np, coef, row, a.KMp, acc);
  else fwd_accumulate<ST, false>(sd.Afull, sd.lda, idx, p0, np, coef, row, a.KMp, acc);
  C2<T>* out = reinterpret_cast<C2<T>*>(a.tpart) + ((int64_t)q * a.nchunk + ch) * a.KMp + row;
#pragma unroll
  for (int r = 0; r < R; ++r) out[r] = acc[r];
}

// out_q += sign * (sum of sensor q's chunk partials), complex128 Q x KMp.
template <class T>
__global__ __launch_bounds__(256) void fwd_all_reduce_kernel(IterArgs a, int active, double sign,
                                                             double* out) {
  const int q = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.KMp) return;
  const int count = active ? a.sens[q].nq : a.N;
  const int nch = (count + a.chunk - 1) / a.chunk;
  const C2<T>* tp = reinterpret_cast<const C2<T>*>(a.tpart) + (int64_t)q * a.nchunk * a.KMp + i;
  C2<T> sm = {(T)0, (T)0};
  in_order<8>(nch, [&](int c) { return tp[(int64_t)c * a.KMp]; }, [&](int, C2<T> v) { sm = cadd(sm, v); });
  double* o = out + 2 * ((int64_t)q * a.KMp + i);
  o[0] += sign * (double)sm.re;
  o[1] += sign * (double)sm.im;
}

// ------------------------------------------------------------------ column dots
enum : int { EPI_W = 0, EPI_XUPD = 1, EPI_WY = 2, EPI_XY = 3, EPI_KKT = 4, EPI_MF = 5,
              EPI_GRAD = 6, EPI_FIX = 7, EPI_WVEC = 8, EPI_W1 = 9, EPI_WY1 = 10,
              EPI_WVEC1 = 11 };
// W products of a sensor with wtri: EPI_W1 / EPI_WY1 / EPI_WVEC1 form
// ws = X t / X y' / X v by column dots of U = X^H (column p nonzero in rows
// 0..p), then EPI_W / EPI_WY / EPI_WVEC take X^H ws by column dots of X
// (column p nonzero in rows p..KMp-1).
// Column dots over a caller's pixel list of one sensor (x.q, x.idx, x.count)
template <int EPI> constexpr bool listed_cols() { return EPI == EPI_KKT; }
// Column dots over the active pixels J_q of every sensor (blockIdx.y = sensor)
template <int EPI> constexpr bool active_cols() { return EPI == EPI_GRAD || EPI == EPI_FIX; }

struct DotExtra {
  const int* idx;       // KKT: eliminated pixel list
  int count;
  int q;                // KKT: sensor
  const double* vec;    // WY / XY / KKT / MF: complex128 source vector(s)
  int64_t vec_stride;   // per-sensor stride (complex entries)
  double mu, gamma, thr;
  uint8_t* flag;        // KKT
  double* out;          // MF (|.|), WY (complex); GRAD / FIX: g (complex128, by pixel)
  int q0;               // WY / XY: first sensor of the launch
  int accumulate;       // GRAD: add to out
  void* out32;          // GRAD (accumulate): g in compute precision; FIX: xfix
  int cplx;             // MF: write A^H y itself (complex128) instead of |A^H y|
  double cinv;          // FIX: 1 / c
};

// Dot of one operator column with the LDS vector sv, accumulated in TA.
template <int ST, class TA>
__device__ inline C2<TA> coldot_core(const void* col, const C2<TA>* sv, int KMp, int lane) {
  using T = typename Store<ST>::T;
  constexpr int R = Store<ST>::RPT;
  C2<TA> acc = {(TA)0, (TA)0};
#pragma unroll 4
  for (int i0 = lane * R; i0 < KMp; i0 += SADMM_WAVE * R) {
    T re[R], im[R];
    Store<ST>::load(col, i0, KMp, re, im);
#pragma unroll
    for (int r = 0; r < R; ++r) cfmac(acc, C2<TA>{(TA)re[r], (TA)im[r]}, sv[i0 + r]);
  }
  acc.re = wave_sum(acc.re);
  acc.im = wave_sum(acc.im);
  return acc;
}

// Slot of vector entry i in the LDS copy.  With 8 rows per lane, lane l of a
// row step reads entries base + 8 l + r, r < 8: entry i is kept at
// (i / 512) * 512 + (i % 8) * 64 + (i % 512) / 8, so the 64 lanes read 64
// consecutive slots for each r (entries 64 bytes apart would share banks).
template <int ST> __device__ inline int sv_slot(int i) {
  if constexpr (Store<ST>::RPT == 8) return (i & ~511) | ((i & 7) << 6) | ((i >> 3) & 63);
  else return i;
}

// Dots of C operator columns with the LDS vector sv in one sweep over the
// rows: every LDS read of the vector serves all C columns, and the C column
// loads of a row step are in flight together.
template <int ST, class TA, int C, bool NT = false>
__device__ inline void coldot_multi(const void* const (&col)[C], const C2<TA>* sv, int KMp, int lane,
                                    C2<TA> (&acc)[C], int rbeg = 0, int rend = -1) {
  using T = typename Store<ST>::T;
  constexpr int R = Store<ST>::RPT;
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = {(TA)0, (TA)0};
  // rows [rbeg, rend): rbeg a multiple of the sweep width or 0
  const int re_ = rend < 0 ? KMp : rend;
  if constexpr (ST == ST_MF) {
    const double* rec0 = reinterpret_cast<const double*>(col[0]);
    const int K = (int)rec0[0], M = (int)rec0[1];
    if ((K & (R - 1)) == 0) {
      // a lane's 8 rows lie in one receiver: sum_r conj(a0 rho^r) v_r =
      // conj(a0) * sum_r conj(rho)^r v_r, the sum by Horner's rule (one
      // complex multiply-add per entry, against a rotation of the entry and
      // a complex multiply-add)
      for (int i0 = rbeg + lane * R; i0 < re_; i0 += SADMM_WAVE * R) {
        const int m = i0 / K;
        if (m >= M) break;                    // padding rows: zero entries
        const int k = i0 - m * K;
        C2<TA> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = sv[sv_slot<ST>(i0 + r)];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          float ar, ai, rc, rs;
          Store<ST_MF>::anchor(col[c], m, k, M, &ar, &ai, &rc, &rs);
          const TA cr = (TA)rc, ci = (TA)rs;  // conj(rho) = rc + j rs
          TA hr = v[R - 1].re, hi = v[R - 1].im;
#pragma unroll
          for (int r = R - 2; r >= 0; --r) {
            const TA nr = fma(cr, hr, fma(-ci, hi, v[r].re));
            const TA ni = fma(cr, hi, fma(ci, hr, v[r].im));
            hr = nr;
            hi = ni;
          }
          cfmac(acc[c], C2<TA>{(TA)ar, (TA)ai}, C2<TA>{hr, hi});
        }
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        acc[c].re = wave_sum(acc[c].re);
        acc[c].im = wave_sum(acc[c].im);
      }
      return;
    }
  }
  // general case: generated entries cost registers, so the matrix-free
  // operator takes its columns two per sweep
  constexpr int CS = (ST == ST_MF && C > 2) ? 2 : C;
  static_assert(C % CS == 0, "column groups");
#pragma unroll
  for (int c0 = 0; c0 < C; c0 += CS) {
    // stored entries of at most 8 bytes per lane and column: four row steps
    // in flight, so that each lane keeps 64-128 bytes of loads outstanding
#pragma unroll(R <= 2 ? 4 : 1)
    for (int i0 = rbeg + lane * R; i0 < re_; i0 += SADMM_WAVE * R) {
      C2<TA> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = sv[sv_slot<ST>(i0 + r)];
#pragma unroll
      for (int c = c0; c < c0 + CS; ++c) {
        T re[R], im[R];
        Store<ST>::template load<NT>(col[c], i0, KMp, re, im);
#pragma unroll
        for (int r = 0; r < R; ++r) cfmac(acc[c], C2<TA>{(TA)re[r], (TA)im[r]}, v[r]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    acc[c].re = wave_sum(acc[c].re);
    acc[c].im = wave_sum(acc[c].im);
  }
}

// Accumulation precision: the per-iteration products run in the compute
// precision; the once-per-factor data term (WY, XY) and the certificate
// products (KKT, MF) accumulate in FP64.
template <int ST, int EPI> struct DotAcc {
  using type = typename std::conditional<(EPI == EPI_XUPD), typename Store<ST>::T, double>::type;
};

// The W product always reads the FP64 factor and accumulates in FP64: W_q has
// condition number (c/mu + s_max^2)/(c/mu) and rounding it to FP32 would put a
// relative error of about 6e-8 * s_max^2 / (c/mu) on every x-update.
template <int ST, int EPI, class TS>
__device__ inline void coldot_body(const IterArgs& a, const DotExtra& x, int q) {
  using T = TS;                               // compute precision of the state
  using TA = typename DotAcc<ST, EPI>::type;  // accumulation precision
  constexpr int DC = dot_cols<ST>();
  if ((EPI == EPI_W || EPI == EPI_W1 || EPI == EPI_XUPD) && a.ctl->halt) return;
  const SensorDesc sd = a.sens[q];
  if ((EPI == EPI_W || EPI == EPI_FIX || EPI == EPI_WVEC || EPI == EPI_W1 || EPI == EPI_WVEC1) && sd.direct)
    return;
  if ((EPI == EPI_W1 || EPI == EPI_WY1 || EPI == EPI_WVEC1) && !sd.wtri) return;
  int ncols;
  if constexpr (EPI == EPI_W || EPI == EPI_WY || EPI == EPI_WVEC || EPI == EPI_W1 || EPI == EPI_WY1 ||
                EPI == EPI_WVEC1)
    ncols = a.KMp;
  else if constexpr (EPI == EPI_XUPD || EPI == EPI_XY || active_cols<EPI>()) ncols = sd.nq;
  else if constexpr (listed_cols<EPI>()) ncols = x.count;
  else ncols = a.N;
  const int cols_per_block = 4 * DC;
  // U's column p holds rows 0..p: its triangle pass takes the longest
  // columns first, so the last work-groups of the grid are the short ones
  // (X's pass, rows p..KMp-1, is longest first in the plain order)
  const int bx = (EPI == EPI_W1 || EPI == EPI_WY1 || EPI == EPI_WVEC1)
                     ? (int)gridDim.x - 1 - (int)blockIdx.x : (int)blockIdx.x;
  const int col0 = bx * cols_per_block;
  if (col0 >= ncols) return;
  extern __shared__ unsigned char smem_raw[];
  C2<TA>* sv = reinterpret_cast<C2<TA>*>(smem_raw);
  // stage the vector operand
#pragma unroll 4
  for (int i = threadIdx.x; i < a.KMp; i += 256) {
    C2<TA> v;
    if constexpr ((EPI == EPI_W || EPI == EPI_WY || EPI == EPI_WVEC) && std::is_same<TA, double>::value) {
      if (sd.wtri) {   // second half of X^H (X v)
        v = {(TA)a.ws[2 * ((int64_t)q * a.KMp + i)], (TA)a.ws[2 * ((int64_t)q * a.KMp + i) + 1]};
        sv[sv_slot<ST>(i)] = v;
        continue;
      }
    }
    if constexpr (EPI == EPI_W || EPI == EPI_W1) {
      const C2<T> tv = ldc<T>(a.t, (int64_t)q * a.KMp + i);
      v = {(TA)tv.re, (TA)tv.im};
    }
    else if constexpr (EPI == EPI_XUPD) v = ldc<TA>(a.w, (int64_t)q * a.KMp + i);
    else if constexpr (EPI == EPI_XY) v = {a.wy[2 * ((int64_t)q * a.KMp + i)], a.wy[2 * ((int64_t)q * a.KMp + i) + 1]};
    else {
      const double* src = x.vec + 2 * ((listed_cols<EPI>() ? 0 : (int64_t)q * x.vec_stride) + i);
      v = {(TA)src[0], (TA)src[1]};
    }
    sv[sv_slot<ST>(i)] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int pw = col0 + wv * DC;   // this wave's first column
  if (pw >= ncols) return;
  const void* cols[DC];
#pragma unroll
  for (int c = 0; c < DC; ++c) {
    const int p = min(pw + c, ncols - 1);   // past the end: repeat the last column
    if constexpr (EPI == EPI_W || EPI == EPI_WY || EPI == EPI_WVEC || EPI == EPI_W1 || EPI == EPI_WY1 ||
                  EPI == EPI_WVEC1)
      cols[c] = col_ptr<ST>(sd.W64, a.KMp, p);
    else if constexpr (EPI == EPI_XUPD || EPI == EPI_XY) cols[c] = col_ptr<ST>(sd.A, sd.lda, p);
    else if constexpr (listed_cols<EPI>()) cols[c] = col_ptr<ST>(sd.Afull, sd.lda, x.idx[p]);
    else if constexpr (active_cols<EPI>()) cols[c] = col_ptr<ST>(sd.Afull, sd.lda, sd.J[p]);
    else cols[c] = col_ptr<ST>(sd.Afull, sd.lda, p);
  }
  C2<TA> dots[DC];
  if constexpr (EPI == EPI_W || EPI == EPI_WY || EPI == EPI_W1 || EPI == EPI_WY1 || EPI == EPI_WVEC ||
                EPI == EPI_WVEC1) {
    int rbeg = 0, rend = -1;
    if (sd.wtri) {
      if constexpr (EPI == EPI_W1 || EPI == EPI_WY1 || EPI == EPI_WVEC1) {
        rend = min(a.KMp, (pw + DC + 63) & ~63);   // U: rows <= p
      } else {
#pragma unroll
        for (int c = 0; c < DC; ++c)                // X: rows >= p
          cols[c] = col_ptr<ST_FP64>(sd.X, a.KMp, min(pw + c, ncols - 1));
        rbeg = pw & ~63;
      }
    }
    if (a.stream_w) coldot_multi<ST, TA, DC, true>(cols, sv, a.KMp, lane, dots, rbeg, rend);
    else coldot_multi<ST, TA, DC, false>(cols, sv, a.KMp, lane, dots, rbeg, rend);
  } else {
    if (a.stream_op) coldot_multi<ST, TA, DC, true>(cols, sv, a.KMp, lane, dots);
    else coldot_multi<ST, TA, DC, false>(cols, sv, a.KMp, lane, dots);
  }
  // The butterfly reduction leaves the same sums in every lane: lane c
  // finishes column pw + c, so a wave's columns complete together.
  if (lane >= DC) return;
  const int p = pw + lane;
  if (p >= ncols) return;
  C2<TA> d = dots[0];
#pragma unroll
  for (int c = 1; c < DC; ++c)
    if (lane == c) d = dots[c];
  {
    if constexpr (EPI == EPI_W) {
      stc<T>(a.w, (int64_t)q * a.KMp + p, C2<T>{(T)d.re, (T)d.im});
    } else if constexpr (EPI == EPI_XUPD) {
      const int n = sd.J[p];
      const C2<T> v = shared_v<T>(a, q, n);
      const C2<T> xy = ldc<T>(sd.xy, p);
      const T bc = (T)a.bc;
      C2<T> xn = {xy.re + bc * (v.re - d.re), xy.im + bc * (v.im - d.im)};
      if (a.xfix) xn = cadd(xn, ldc<T>(a.xfix, (int64_t)q * a.N + n));
      const int64_t o = (int64_t)q * a.N + n;
      const C2<T> xo = ldc<T>(a.X, o);
      const C2<T> dx = csub(xn, xo);
      stc<T>(a.X, o, xn);
      stc<T>(a.dX, o, dx);
      const int slot = a.ctl->k % a.Kp;
      reinterpret_cast<T*>(a.D)[((int64_t)slot * a.Q + q) * a.N + n] = habs(dx);
    } else if constexpr (EPI == EPI_WY) {
      a.wy[2 * ((int64_t)q * a.KMp + p)] = d.re;
      a.wy[2 * ((int64_t)q * a.KMp + p) + 1] = d.im;
    } else if constexpr (EPI == EPI_XY) {
      stc<T>(const_cast<void*>(sd.xy), p, C2<T>{(T)d.re, (T)d.im});
    } else if constexpr (EPI == EPI_KKT) {
      const int n = x.idx[p];
      const C2<T> xv = ldc<T>(a.X, (int64_t)q * a.N + n);
      const C2<T> uv = ldc<T>(a.u, n);
      const double gre = x.mu * d.re + x.gamma * (double)xv.re + a.beta * (double)uv.re;
      const double gim = x.mu * d.im + x.gamma * (double)xv.im + a.beta * (double)uv.im;
      x.out[2 * p] = gre;
      x.out[2 * p + 1] = gim;
    } else if constexpr (EPI == EPI_W1 || EPI == EPI_WY1 || EPI == EPI_WVEC1) {
      a.ws[2 * ((int64_t)q * a.KMp + p)] = d.re;
      a.ws[2 * ((int64_t)q * a.KMp + p) + 1] = d.im;
    } else if constexpr (EPI == EPI_WVEC) {
      x.out[2 * ((int64_t)q * a.KMp + p)] = d.re;        // (W v)_p: W Hermitian
      x.out[2 * ((int64_t)q * a.KMp + p) + 1] = d.im;
    } else if constexpr (EPI == EPI_GRAD) {
      const int64_t o = (int64_t)q * a.N + sd.J[p];
      double gr = x.mu * d.re, gi = x.mu * d.im;
      if (x.accumulate) {
        gr += x.out[2 * o];
        gi += x.out[2 * o + 1];
        stc<T>(x.out32, o, C2<T>{(T)gr, (T)gi});
      }
      x.out[2 * o] = gr;
      x.out[2 * o + 1] = gi;
    } else if constexpr (EPI == EPI_FIX) {
      const int64_t o = (int64_t)q * a.N + sd.J[p];
      stc<T>(x.out32, o, C2<T>{(T)(x.cinv * (x.out[2 * o] - d.re)), (T)(x.cinv * (x.out[2 * o + 1] - d.im))});
    } else if (x.cplx) {
      x.out[2 * ((int64_t)q * a.N + p)] = d.re;
      x.out[2 * ((int64_t)q * a.N + p) + 1] = d.im;
    } else {
      x.out[(int64_t)q * a.N + p] = hypot(d.re, d.im);
    }
  }
}

template <int ST, int EPI, class TS = typename Store<ST>::T>
__global__ __launch_bounds__(256) void coldot_kernel(IterArgs a, DotExtra x) {
  const int q = listed_cols<EPI>() ? x.q
              : ((EPI == EPI_WY || EPI == EPI_XY || EPI == EPI_WY1) ? x.q0 + (int)blockIdx.y
                                                                      : (int)blockIdx.y);
  coldot_body<ST, EPI, TS>(a, x, q);
}

// Per-iteration column dots over a batch: blockIdx.y is the work slot.
// x-update of a sensor in the direct form, x_q = F (b0 + beta v) with
// F = (mu Ahat^H Ahat + cI)^{-1}: F is Hermitian, so column p of F,
// conjugated and dotted with the right-hand side, gives x at the p-th active
// pixel.  FP64 throughout; the right-hand side (prepared by the forward
// reduction, zero-padded to fld) passes through LDS in XDIR_SEG segments.
template <int ST, class T>
__device__ inline void xdir_body(const IterArgs& a, int q) {
  constexpr int DC = dot_cols<ST>();   // the x-update launch's columns per wave
  if (a.ctl->halt) return;
  const SensorDesc sd = a.sens[q];
  const int col0 = blockIdx.x * 4 * DC;
  if (col0 >= sd.nq) return;
  extern __shared__ unsigned char smem_raw[];
  cd* sv = reinterpret_cast<cd*>(smem_raw);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cd acc[DC];
#pragma unroll
  for (int c = 0; c < DC; ++c) acc[c] = {0.0, 0.0};
  for (int s0 = 0; s0 < sd.fld; s0 += XDIR_SEG) {
    const int len = min(XDIR_SEG, sd.fld - s0);
    __syncthreads();   // the previous segment is consumed
#pragma unroll 4
    for (int i = threadIdx.x; i < len; i += 256) sv[i] = sd.rdir[s0 + i];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      const int p = col0 + wv * DC + c;
      if (p < sd.nq) {   // uniform across the wave
        const cd d = coldot_core<ST_FP64, double>(sd.F + (int64_t)p * sd.fld + s0, sv, len, lane);
        acc[c].re += d.re;
        acc[c].im += d.im;
      }
    }
  }
  // every lane holds the sums: lane c finishes column c of the wave
  if (lane >= DC) return;
  const int slot = a.ctl->k % a.Kp;
  {
    const int p = col0 + wv * DC + lane;
    if (p >= sd.nq) return;
    cd ac = acc[0];
#pragma unroll
    for (int c = 1; c < DC; ++c)
      if (lane == c) ac = acc[c];
    const int n = sd.J[p];
    const C2<T> xn = {(T)ac.re, (T)ac.im};
    const int64_t o = (int64_t)q * a.N + n;
    const C2<T> dx = csub(xn, ldc<T>(a.X, o));
    stc<T>(a.X, o, xn);
    stc<T>(a.dX, o, dx);
    reinterpret_cast<T*>(a.D)[((int64_t)slot * a.Q + q) * a.N + n] = habs(dx);
  }
}

template <int ST, int EPI, class TS = typename Store<ST>::T>
__global__ __launch_bounds__(256) void coldot_batch_kernel(BatchView bv) {
  const int2 sl = bv.slots[blockIdx.y];
  DotExtra x{};
  if constexpr (EPI == EPI_XUPD) {
    if (bv.args[sl.x].sens[sl.y].direct) {
      xdir_body<ST, TS>(bv.args[sl.x], sl.y);
      return;
    }
  }
  coldot_body<ST, EPI, TS>(bv.args[sl.x], x, sl.y);
}

// ------------------------------------------------------------------ pixel update
// Residuals, stop test, balancing decision and history of one iteration of a
// scene from the pixel blocks' partial sums, by one work-group of 256.
__device__ __forceinline__ void finalize_scene(const IterArgs& a, double* sm) {
  Ctl* ctl = a.ctl;
  double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < a.nblk; b += 256) {
#pragma unroll
    for (int j = 0; j < 8; ++j) part[j] += a.red[(int64_t)b * 8 + j];
  }
  block_sum256<double, 8>(part, sm);
  if (threadIdx.x != 0) return;
  const double Q = a.Q;
  const int k = ctl->k + 1;
  const double r = sqrt(Q) * sqrt(part[0]);
  const double s = a.beta * sqrt(part[1]);
  const double sqQN = sqrt(Q * (double)a.N);
  const double eps_pri = sqQN * a.eps_abs + a.eps_rel * fmax(sqrt(part[2]), sqrt(part[3]));
  const double eps_dual = sqQN * a.eps_abs + a.eps_rel * a.beta * sqrt(Q) * sqrt(part[4]);
  const double nmse = a.xref ? part[5] / a.xref_norm2 : 0.0;
  int halt = 0;
  bool finite = true;
  for (int j = 0; j < 6; ++j) finite = finite && isfinite(part[j]);
  if (!finite) halt |= HALT_NAN;
  if (a.stop && r <= eps_pri && s <= eps_dual) halt |= HALT_CONV;
  if (a.xref && a.nmse_target > 0.0 && nmse <= a.nmse_target) halt |= HALT_NMSE;
  if (k >= a.max_iter) halt |= HALT_MAXIT;
  // residual balancing (Boyd et al. 2011, Sec. 3.4.1), decided here and
  // applied by the host after this iteration's SSC check
  int bal = 0;
  if (a.bal_every > 0 && !(halt & (HALT_CONV | HALT_NAN | HALT_NMSE | HALT_MAXIT)) && k % a.bal_every == 0) {
    if (r > a.bal_mu * s) bal = 1;
    else if (s > a.bal_mu * r) bal = -1;
    if (bal) halt |= HALT_BAL;
  }
  ctl->bal = bal;
  double* h = a.hist;
  const int mi = a.max_iter;
  h[0 * mi + k - 1] = r;
  h[1 * mi + k - 1] = s;
  h[2 * mi + k - 1] = eps_pri;
  h[3 * mi + k - 1] = eps_dual;
  h[4 * mi + k - 1] = nmse;
  ctl->r = r; ctl->s = s; ctl->eps_pri = eps_pri; ctl->eps_dual = eps_dual; ctl->nmse = nmse;
  ctl->gate = (r <= eps_pri) ? 1 : 0;
  ctl->nan = finite ? 0 : 1;
  ctl->k = k;
  ctl->halt = halt;
}

template <class T>
__global__ __launch_bounds__(256) void pixel_kernel(BatchView bv) {
  const IterArgs& a = bv.args[blockIdx.y];
  if (a.ctl->halt || (int)blockIdx.x >= a.nblk) return;
  __shared__ double sm[4 * 8];
  double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n < a.N) {
    C2<T> sum = {(T)0, (T)0};
    in_order<8>(a.Q, [&](int q) { return ldc<T>(a.X, (int64_t)q * a.N + n); },
                [&](int, C2<T> v) { sum = cadd(sum, v); });
    const T Qt = (T)a.Q;
    const C2<T> xb = {sum.re / Qt, sum.im / Qt};
    const C2<T> zo = ldc<T>(a.z, n), xbo = ldc<T>(a.xbar, n), uo = ldc<T>(a.u, n);
    const C2<T> v = cadd(xb, uo);
    const T mag = habs(v);
    const T tau = (T)a.tau;
    C2<T> zn = {(T)0, (T)0};
    if (a.nonneg) {             // projection on the non-negative reals
      if (v.re > tau) zn.re = v.re - tau;
    } else if (mag > tau) {
      const T sc = (T)1 - tau / mag;
      zn = {v.re * sc, v.im * sc};
    }
    const C2<T> un = csub(cadd(uo, xb), zn);
    const C2<T> dz = csub(csub(zn, xb), csub(zo, xbo));
    // replicated shared variable Z[q] = x_q + z - xbar: s from its change,
    // its norm for the primal tolerance
    const C2<T> zx = csub(zn, xb);
    double s2 = 0.0, nx2 = 0.0, nz2 = 0.0;
    struct DX { C2<T> dx, x; };
    in_order<8>(a.Q, [&](int q) {
      const int64_t o = (int64_t)q * a.N + n;
      return DX{ldc<T>(a.dX, o), ldc<T>(a.X, o)};
    }, [&](int, DX v) {
      const C2<T> d = cadd(v.dx, dz);
      s2 += (double)cabs2(d);
      nx2 += (double)cabs2(v.x);
      nz2 += (double)cabs2(cadd(v.x, zx));
    });
    part[0] = (double)cabs2(csub(xb, zn));
    part[1] = s2;
    part[2] = nx2;
    part[3] = nz2;
    part[4] = (double)cabs2(un);
    if (a.xref) {
      const C2<T> r = ldc<T>(a.xref, n);
      part[5] = (double)cabs2(csub(zn, r));
    }
    stc<T>(a.xbar, n, xb);
    stc<T>(a.z, n, zn);
    stc<T>(a.u, n, un);
  }
  block_sum256<double, 8>(part, sm);
  // The scene's last block to finish (counted on the control block) finds
  // every partial written and ends the iteration; it also clears the count
  // for the next iteration, so replays need no reset.
  __shared__ int last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a.red[(int64_t)blockIdx.x * 8 + j] = part[j];
    __threadfence();   // the partials are visible before the count
    last = atomicAdd(&a.ctl->pix_done, 1u) == (unsigned)a.nblk - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) a.ctl->pix_done = 0;
  finalize_scene(a, sm);
}


// SSC check (Alg. 1, steps 1-2): runs when the gate is open and K_p
// differences exist.  Runs at the last permitted iteration too (max_iter),
// but not once converged.
template <class T>
__global__ __launch_bounds__(256) void ssc_kernel(BatchView bv) {
  const int2 sl = bv.slots[blockIdx.y];
  const IterArgs& a = bv.args[sl.x];
  Ctl* ctl = a.ctl;
  if (!a.prune) return;
  if (ctl->halt & (HALT_CONV | HALT_NAN | HALT_NMSE | HALT_PRUNE)) return;
  const int k = ctl->k;
  if (k < a.Kp || k < a.ssc_from || !ctl->gate) return;
  const int q = sl.y;
  const SensorDesc sd = a.sens[q];
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < sd.nq) {
    const int n = sd.J[p];
    const T* D = reinterpret_cast<const T*>(a.D);
    T zs = (T)0;
    in_order<8>(a.Kp, [&](int sl) { return D[((int64_t)sl * a.Q + q) * a.N + n]; }, [&](int, T v) { zs += v; });
    const T zeta = zs / (T)a.Kp;
    const bool keep = zeta >= (T)a.eps_p;
    a.keep[(int64_t)q * a.N + p] = keep ? 1 : 0;
    if (!keep) atomicAdd(&a.gone[q], 1);
  }
  // The scene's last block (of gridDim.x per sensor, Q sensors) raises the
  // prune halt bit when the check removed anything, and clears the count.
  __shared__ int last;
  __threadfence();   // this thread's eliminations are counted before the block is
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&ctl->ssc_done, 1u) == gridDim.x * (unsigned)a.Q - 1;
  __syncthreads();
  if (!last || threadIdx.x != 0) return;
  __threadfence();
  ctl->ssc_done = 0;
  int tot = 0;
  for (int qq = 0; qq < a.Q; ++qq) tot += atomicAdd(&a.gone[qq], 0);
  if (tot > 0) {
    ctl->gone_total = tot;
    ctl->halt |= HALT_PRUNE;
  }
}

__global__ void gather_ctl_kernel(Ctl* const* ptrs, Ctl* out, int n) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i < n) out[i] = *ptrs[i];
}

template <class T>
void launch_pixel_stage_t(const BatchView& b, const BatchDims& d, hipStream_t s) {
  pixel_kernel<T><<<dim3(d.nblk_max, d.nscene), 256, 0, s>>>(b);   // ends with the scene's residuals
  ssc_kernel<T><<<dim3((d.N_max + 255) / 256, d.nslot), 256, 0, s>>>(b);
}

template <int ST>
void run_iteration_batch(const BatchView& b, const BatchDims& d, hipStream_t s,
                         const std::function<void(int, bool)>* hook) {
  using T = typename Store<ST>::T;
  auto mark = [&](int stage, bool begin) { if (hook) (*hook)(stage, begin); };
  const int rows = FWD_THREADS * Store<ST>::RPT;
  const int cpb64 = 4 * dot_cols<ST_FP64>(), cpb = 4 * dot_cols<ST>();
  mark(0, true);
  fwd_iter_kernel<ST><<<dim3((d.KMp_max + rows - 1) / rows, d.nchunk_max, d.nslot), FWD_THREADS, 0, s>>>(b);
  fwd_reduce_kernel<T><<<dim3((std::max(d.KMp_max, d.fld_max) + 255) / 256, d.nslot), 256, 0, s>>>(b);
  mark(0, false);
  mark(1, true);
  coldot_batch_kernel<ST_FP64, EPI_W1, T><<<dim3((d.KMp_max + cpb64 - 1) / cpb64, d.nslot), 256,
                                            (size_t)d.KMp_max * sizeof(cd), s>>>(b);
  coldot_batch_kernel<ST_FP64, EPI_W, T><<<dim3((d.KMp_max + cpb64 - 1) / cpb64, d.nslot), 256,
                                           (size_t)d.KMp_max * sizeof(cd), s>>>(b);
  mark(1, false);
  mark(2, true);
  coldot_batch_kernel<ST, EPI_XUPD><<<dim3((d.N_max + cpb - 1) / cpb, d.nslot), 256,
                                      std::max((size_t)sv_len<ST>(d.KMp_max) * sizeof(C2<T>),
                                               (size_t)std::min(d.fld_max, XDIR_SEG) * sizeof(cd)),
                                      s>>>(b);
  mark(2, false);
  mark(3, true);
  launch_pixel_stage_t<T>(b, d, s);
  mark(3, false);
}

}  // namespace

void launch_pixel_stage(const BatchView& b, const BatchDims& d, bool dbl, hipStream_t s) {
  if (dbl) launch_pixel_stage_t<double>(b, d, s);
  else launch_pixel_stage_t<float>(b, d, s);
}

int fwd_row_tile(int st) {
  switch (st) {
    case ST_FP64: return FWD_THREADS * Store<ST_FP64>::RPT;
    case ST_FP32: return FWD_THREADS * Store<ST_FP32>::RPT;
    case ST_MF: return FWD_THREADS * Store<ST_MF>::RPT;
    default: return FWD_THREADS * Store<ST_FP16P>::RPT;
  }
}

void launch_iteration_batch(const BatchView& b, const BatchDims& d, int st, hipStream_t s,
                            const std::function<void(int, bool)>* hook) {
  switch (st) {
    case ST_FP64: run_iteration_batch<ST_FP64>(b, d, s, hook); break;
    case ST_FP32: run_iteration_batch<ST_FP32>(b, d, s, hook); break;
    case ST_FP16P: run_iteration_batch<ST_FP16P>(b, d, s, hook); break;
    case ST_BF16P: run_iteration_batch<ST_BF16P>(b, d, s, hook); break;
    case ST_MF: run_iteration_batch<ST_MF>(b, d, s, hook); break;
  }
}

void gather_ctl(Ctl* const* ptrs, Ctl* out, int nscene, hipStream_t s) {
  gather_ctl_kernel<<<(nscene + 63) / 64, 64, 0, s>>>(ptrs, out, nscene);
}

template <int ST>
static void xy_impl(const IterArgs& a, int q0, int q1, hipStream_t s) {
  DotExtra x{};
  x.q0 = q0;
  const int cpb64 = 4 * dot_cols<ST_FP64>(), cpb = 4 * dot_cols<ST>();
  const size_t smem = (size_t)a.KMp * sizeof(cd);
  // W_q y'_q in FP64, then Ahat_q^H (W_q y'_q) accumulated in FP64
  x.vec = a.yp;
  x.vec_stride = a.KMp;
  coldot_kernel<ST_FP64, EPI_WY1><<<dim3((a.KMp + cpb64 - 1) / cpb64, q1 - q0), 256, smem, s>>>(a, x);
  coldot_kernel<ST_FP64, EPI_WY><<<dim3((a.KMp + cpb64 - 1) / cpb64, q1 - q0), 256, smem, s>>>(a, x);
  coldot_kernel<ST, EPI_XY><<<dim3((a.N + cpb - 1) / cpb, q1 - q0), 256,
                             (size_t)sv_len<ST>(a.KMp) * sizeof(cd), s>>>(a, x);
}

void launch_xy(const IterArgs& a, int st, bool dbl, int q0, int q1, hipStream_t s) {
  (void)dbl;
  if (q1 <= q0) return;
  switch (st) {
    case ST_FP64: xy_impl<ST_FP64>(a, q0, q1, s); break;
    case ST_FP32: xy_impl<ST_FP32>(a, q0, q1, s); break;
    case ST_FP16P: xy_impl<ST_FP16P>(a, q0, q1, s); break;
    case ST_BF16P: xy_impl<ST_BF16P>(a, q0, q1, s); break;
    case ST_MF: xy_impl<ST_MF>(a, q0, q1, s); break;
  }
}

template <int ST>
static void gather_impl(const IterArgs& a, int q, const int* idx, int count, double sign,
                        double* out, void* tmp, hipStream_t s) {
  using T = typename Store<ST>::T;
  if (count <= 0) return;
  const int rows = FWD_THREADS * Store<ST>::RPT;
  const int nch = (count + a.chunk - 1) / a.chunk;
  fwd_gather_kernel<ST><<<dim3((a.KMp + rows - 1) / rows, nch, 1), FWD_THREADS, 0, s>>>(a, q, idx, count, tmp);
  gather_reduce_kernel<T><<<(a.KMp + 255) / 256, 256, 0, s>>>(a.KMp, nch, tmp, sign, out);
}

void launch_gather_fwd(const IterArgs& a, int st, bool dbl, int q, const int* idx, int count,
                       double sign, double* out, void* tmp, hipStream_t s) {
  (void)dbl;
  switch (st) {
    case ST_FP64: gather_impl<ST_FP64>(a, q, idx, count, sign, out, tmp, s); break;
    case ST_FP32: gather_impl<ST_FP32>(a, q, idx, count, sign, out, tmp, s); break;
    case ST_FP16P: gather_impl<ST_FP16P>(a, q, idx, count, sign, out, tmp, s); break;
    case ST_BF16P: gather_impl<ST_BF16P>(a, q, idx, count, sign, out, tmp, s); break;
    case ST_MF: gather_impl<ST_MF>(a, q, idx, count, sign, out, tmp, s); break;
  }
}

template <int ST>
static void kkt_impl(const IterArgs& a, int q, const int* idx, int count, const double* e,
                     double mu, double gamma, double* g, hipStream_t s) {
  using T = typename Store<ST>::T;
  if (count <= 0) return;
  DotExtra x{};
  x.idx = idx;
  x.count = count;
  x.q = q;
  x.vec = e;
  x.mu = mu;
  x.gamma = gamma;
  x.out = g;
  const int cpb = 4 * dot_cols<ST>();
  const size_t smem = (size_t)sv_len<ST>(a.KMp) * sizeof(cd);
  coldot_kernel<ST, EPI_KKT><<<dim3((count + cpb - 1) / cpb, 1), 256, smem, s>>>(a, x);
}

void launch_kkt_grad(const IterArgs& a, int st, bool dbl, int q, const int* idx, int count,
                     const double* e, double mu, double gamma, double* g, hipStream_t s) {
  (void)dbl;
  switch (st) {
    case ST_FP64: kkt_impl<ST_FP64>(a, q, idx, count, e, mu, gamma, g, s); break;
    case ST_FP32: kkt_impl<ST_FP32>(a, q, idx, count, e, mu, gamma, g, s); break;
    case ST_FP16P: kkt_impl<ST_FP16P>(a, q, idx, count, e, mu, gamma, g, s); break;
    case ST_BF16P: kkt_impl<ST_BF16P>(a, q, idx, count, e, mu, gamma, g, s); break;
    case ST_MF: kkt_impl<ST_MF>(a, q, idx, count, e, mu, gamma, g, s); break;
  }
}

template <int ST>
static void refine_fwd_impl(const IterArgs& a, bool active, const void* xsrc, double sign, double* out,
                            hipStream_t s) {
  using T = typename Store<ST>::T;
  const int rows = FWD_THREADS * Store<ST>::RPT;
  fwd_all_kernel<ST><<<dim3((a.KMp + rows - 1) / rows, a.nchunk, a.Q), FWD_THREADS, 0, s>>>(
      a, active ? 1 : 0, xsrc);
  fwd_all_reduce_kernel<T><<<dim3((a.KMp + 255) / 256, a.Q), 256, 0, s>>>(a, active ? 1 : 0, sign, out);
}

void launch_refine_fwd(const IterArgs& a, int st, bool active, const void* xsrc, double sign, double* out,
                       hipStream_t s) {
  switch (st) {
    case ST_FP16P: refine_fwd_impl<ST_FP16P>(a, active, xsrc, sign, out, s); break;
    case ST_BF16P: refine_fwd_impl<ST_BF16P>(a, active, xsrc, sign, out, s); break;
    case ST_MF: refine_fwd_impl<ST_MF>(a, active, xsrc, sign, out, s); break;
    default: break;   // the correction applies to 16-bit storage (checked by the caller)
  }
}

void launch_factor_vec(const IterArgs& a, const double* v, double* out, hipStream_t s) {
  DotExtra x{};
  x.vec = v;
  x.vec_stride = a.KMp;
  x.out = out;
  const int cpb = 4 * dot_cols<ST_FP64>();
  const dim3 grid((a.KMp + cpb - 1) / cpb, a.Q);
  // sensors holding the triangular pair: ws = X v first (into the iteration's
  // scratch, free between iterations), then X^H ws
  coldot_kernel<ST_FP64, EPI_WVEC1, float><<<grid, 256, (size_t)a.KMp * sizeof(cd), s>>>(a, x);
  coldot_kernel<ST_FP64, EPI_WVEC, float><<<grid, 256, (size_t)a.KMp * sizeof(cd), s>>>(a, x);
}

template <int ST>
static void refine_impl(const IterArgs& a, int epi, int max_nq, const double* v, double scale,
                        bool accumulate, double* g, void* out32, double cinv, hipStream_t s) {
  if (max_nq <= 0) return;
  DotExtra x{};
  x.vec = v;
  x.vec_stride = a.KMp;
  x.mu = scale;
  x.accumulate = accumulate ? 1 : 0;
  x.out = g;
  x.out32 = out32;
  x.cinv = cinv;
  const int cpb = 4 * dot_cols<ST>();
  const size_t smem = (size_t)sv_len<ST>(a.KMp) * sizeof(cd);
  const dim3 grid((max_nq + cpb - 1) / cpb, a.Q);
  if (epi == EPI_GRAD) coldot_kernel<ST, EPI_GRAD><<<grid, 256, smem, s>>>(a, x);
  else coldot_kernel<ST, EPI_FIX><<<grid, 256, smem, s>>>(a, x);
}

static void refine_dispatch(const IterArgs& a, int st, int epi, int max_nq, const double* v, double scale,
                            bool accumulate, double* g, void* out32, double cinv, hipStream_t s) {
  switch (st) {
    case ST_FP16P: refine_impl<ST_FP16P>(a, epi, max_nq, v, scale, accumulate, g, out32, cinv, s); break;
    case ST_BF16P: refine_impl<ST_BF16P>(a, epi, max_nq, v, scale, accumulate, g, out32, cinv, s); break;
    case ST_MF: refine_impl<ST_MF>(a, epi, max_nq, v, scale, accumulate, g, out32, cinv, s); break;
    default: break;
  }
}

void launch_refine_grad(const IterArgs& a, int st, int max_nq, const double* e, double scale,
                        bool accumulate, double* g, void* g32, hipStream_t s) {
  refine_dispatch(a, st, EPI_GRAD, max_nq, e, scale, accumulate, g, g32, 0.0, s);
}

void launch_refine_fix(const IterArgs& a, int st, int max_nq, const double* w, const double* g,
                       double cinv, void* xfix, hipStream_t s) {
  refine_dispatch(a, st, EPI_FIX, max_nq, w, 1.0, false, const_cast<double*>(g), xfix, cinv, s);
}

template <int ST>
static void mf_impl(const IterArgs& a, const double* y, double* out, bool cplx, hipStream_t s) {
  using T = typename Store<ST>::T;
  DotExtra x{};
  x.vec = y;
  x.vec_stride = a.KMp;
  x.out = out;
  x.cplx = cplx ? 1 : 0;
  const int cpb = 4 * dot_cols<ST>();
  const size_t smem = (size_t)sv_len<ST>(a.KMp) * sizeof(cd);
  coldot_kernel<ST, EPI_MF><<<dim3((a.N + cpb - 1) / cpb, a.Q), 256, smem, s>>>(a, x);
}

void launch_matched_filter(const IterArgs& a, int st, bool dbl, const double* y, double* out,
                           hipStream_t s, bool cplx) {
  (void)dbl;
  switch (st) {
    case ST_FP64: mf_impl<ST_FP64>(a, y, out, cplx, s); break;
    case ST_FP32: mf_impl<ST_FP32>(a, y, out, cplx, s); break;
    case ST_FP16P: mf_impl<ST_FP16P>(a, y, out, cplx, s); break;
    case ST_BF16P: mf_impl<ST_BF16P>(a, y, out, cplx, s); break;
    case ST_MF: mf_impl<ST_MF>(a, y, out, cplx, s); break;
  }
}
