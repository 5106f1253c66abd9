// Shared device helpers: complex arithmetic, operator storage formats,
// wavefront reductions.  gfx950 (CDNA4): 64-lane wavefronts.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#define SADMM_WAVE 64

template <class T> struct C2 { T re, im; };
using cf = C2<float>;
using cd = C2<double>;

template <class T> __host__ __device__ inline C2<T> cmk(T r, T i) { return C2<T>{r, i}; }
template <class T> __device__ inline C2<T> cadd(C2<T> a, C2<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ inline C2<T> csub(C2<T> a, C2<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ inline C2<T> cscale(C2<T> a, T s) { return {a.re * s, a.im * s}; }
// a*b
template <class T> __device__ inline C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc += a*b
template <class T> __device__ inline void cfma(C2<T>& acc, C2<T> a, C2<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a)*b
template <class T> __device__ inline void cfmac(C2<T>& acc, C2<T> a, C2<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
template <class T> __device__ inline T cabs2(C2<T> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------- storage formats
// Storage ids match sadmm_storage.
enum : int { ST_FP64 = 0, ST_FP32 = 1, ST_FP16P = 2, ST_BF16P = 3, ST_MF = 4 };

// Column layout per storage (ld counts storage "slots" per column):
//   ST_FP64 : KM complex128 entries               (ld >= KM, slot = 16 B)
//   ST_FP32 : KM complex64 entries                (ld >= KM, slot = 8 B)
//   ST_FP16P/ST_BF16P : KM real halves then KM imaginary halves
//                       (ld >= 2*KM slots of 2 B; real plane at +0, imag at +KM)
// RPT = rows covered by one 16-byte vector load (per plane for planar).
template <int ST> struct Store;
template <> struct Store<ST_FP64> {
  using T = double;
  static constexpr int RPT = 1;
  static constexpr int BYTES = 16;   // per complex entry
  // NT: a non-temporal load, for passes over more data than the caches hold
  template <bool NT = false>
  __device__ static inline void load(const void* col, int i, int KM, T* re, T* im) {
    (void)KM;
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* p = reinterpret_cast<const d2*>(col) + i;
    d2 v;
    if constexpr (NT) v = __builtin_nontemporal_load(p);
    else v = *p;
    re[0] = v.x; im[0] = v.y;
  }
  __device__ static inline cd get(const void* col, int i, int KM) {
    (void)KM;
    const double2 v = reinterpret_cast<const double2*>(col)[i];
    return {v.x, v.y};
  }
  // get() for a pass that reads each entry once (non-temporal load)
  __device__ static inline cd get_stream(const void* col, int i, int KM) {
    (void)KM;
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(col) + i);
    return {v.x, v.y};
  }
};
template <> struct Store<ST_FP32> {
  using T = float;
  static constexpr int RPT = 2;
  static constexpr int BYTES = 8;
  template <bool NT = false>
  __device__ static inline void load(const void* col, int i, int KM, T* re, T* im) {
    (void)KM;
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4* p = reinterpret_cast<const f4*>(reinterpret_cast<const float2*>(col) + i);
    f4 v;
    if constexpr (NT) v = __builtin_nontemporal_load(p);
    else v = *p;
    re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w;
  }
  __device__ static inline cd get(const void* col, int i, int KM) {
    (void)KM;
    const float2 v = reinterpret_cast<const float2*>(col)[i];
    return {(double)v.x, (double)v.y};
  }
  __device__ static inline cd get_stream(const void* col, int i, int KM) {
    (void)KM;
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = __builtin_nontemporal_load(reinterpret_cast<const f2*>(col) + i);
    return {(double)v.x, (double)v.y};
  }
};
__device__ inline float h2f(uint16_t b) { return __half2float(__ushort_as_half(b)); }
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
template <int ST> __device__ inline float p16_to_f(uint16_t b) {
  if constexpr (ST == ST_FP16P) return h2f(b); else return bf2f(b);
}
template <int STP> struct StoreP16 {
  using T = float;
  static constexpr int RPT = 8;
  static constexpr int BYTES = 4;
  template <bool NT = false>
  __device__ static inline void load(const void* col, int i, int KM, T* re, T* im) {
    const uint16_t* c = reinterpret_cast<const uint16_t*>(col);
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4* pr = reinterpret_cast<const u4*>(c + i);
    const u4* pi = reinterpret_cast<const u4*>(c + KM + i);
    u4 vr, vi;
    if constexpr (NT) {
      vr = __builtin_nontemporal_load(pr);
      vi = __builtin_nontemporal_load(pi);
    } else {
      vr = *pr;
      vi = *pi;
    }
    const uint32_t r4[4] = {vr.x, vr.y, vr.z, vr.w};
    const uint32_t i4[4] = {vi.x, vi.y, vi.z, vi.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      re[2 * t] = p16_to_f<STP>((uint16_t)(r4[t] & 0xffffu));
      re[2 * t + 1] = p16_to_f<STP>((uint16_t)(r4[t] >> 16));
      im[2 * t] = p16_to_f<STP>((uint16_t)(i4[t] & 0xffffu));
      im[2 * t + 1] = p16_to_f<STP>((uint16_t)(i4[t] >> 16));
    }
  }
  __device__ static inline cd get(const void* col, int i, int KM) {
    const uint16_t* c = reinterpret_cast<const uint16_t*>(col);
    return {(double)p16_to_f<STP>(c[i]), (double)p16_to_f<STP>(c[KM + i])};
  }
  __device__ static inline cd get_stream(const void* col, int i, int KM) {
    const uint16_t* c = reinterpret_cast<const uint16_t*>(col);
    return {(double)p16_to_f<STP>(__builtin_nontemporal_load(c + i)),
            (double)p16_to_f<STP>(__builtin_nontemporal_load(c + KM + i))};
  }
};
template <> struct Store<ST_FP16P> : StoreP16<ST_FP16P> {};
template <> struct Store<ST_BF16P> : StoreP16<ST_BF16P> {};

// Matrix-free LFM operator (eq. (1)): instead of stored entries, each pixel has
// a record of 2 + 4M doubles [K, M, then per receiver m: c0_m, d_m,
// cos(2 pi d_m), sin(2 pi d_m)] with c0_m = frac(f0 tau_m) and
// d_m = frac(bw tau_m / K) (cycles), and entry (m*K + k) =
// exp(-j 2 pi frac(c0_m + k d_m)).
// Entries are generated in groups of 8 consecutive rows starting at a multiple
// of 8.  The first row of a group (and the first row of a receiver inside it)
// is anchored: phase fraction in FP64 (f0 tau is thousands of cycles), the
// exponential by the FP32 hardware sine and cosine of that fraction.  The
// following rows are the previous entry times exp(-j 2 pi d_m) in FP32 (at
// most 7 steps, each a few units of 2^-24).  The arithmetic is written with
// explicit round-to-nearest operations and get() replays its row's group, so
// the Gram and the entry-wise uses see identical entries; the per-iteration
// products rotate their running terms from the same anchors instead (the
// same entries up to FP32 rounding).
constexpr int MF_REC_BASE = 2, MF_REC_PER_RX = 4;
__device__ inline void mf_entry(double c0, double d, int k, float* re, float* im) {
  const double cyc = fma((double)k, d, c0);
  const float fr = (float)(cyc - floor(cyc));
  // the hardware sine and cosine take the angle in turns: sin(2 pi fr) and
  // cos(2 pi fr) for fr in [0, 1), within 1.3e-7 (measured over 4M
  // fractions against FP64; sincospif: 5.1e-8)
  *re = __builtin_amdgcn_cosf(fr);
  *im = -__builtin_amdgcn_sinf(fr);
}
template <> struct Store<ST_MF> {
  using T = float;
  static constexpr int RPT = 8;
  static constexpr int BYTES = 0;   // nothing stored per entry
  // rows i .. i+7, i a multiple of 8
  template <bool NT = false>   // (nothing is loaded per entry)
  __device__ static inline void load(const void* col, int i, int KM, T* re, T* im) {
    (void)KM;
    const double* rec = reinterpret_cast<const double*>(col);
    const int K = (int)rec[0], M = (int)rec[1];
    int m = i / K, k = i - m * K;
    float er = 0.f, ei = 0.f, rc = 0.f, rs = 0.f;
    if ((K & (RPT - 1)) == 0) {   // the group stays within one receiver
      if (m < M) {
        const double* p = rec + MF_REC_BASE + MF_REC_PER_RX * m;
        mf_entry(p[0], p[1], k, &er, &ei);
        rc = (float)p[2];
        rs = (float)p[3];
      }
      re[0] = er;
      im[0] = ei;
#pragma unroll
      for (int r = 1; r < RPT; ++r) {
        const float nr = __fmaf_rn(er, rc, __fmul_rn(ei, rs));
        const float ni = __fmaf_rn(ei, rc, -__fmul_rn(er, rs));
        er = nr;
        ei = ni;
        re[r] = er;
        im[r] = ei;
      }
      return;
    }
    bool anchored = false;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (m < M) {
        if (!anchored) {
          const double* p = rec + MF_REC_BASE + MF_REC_PER_RX * m;
          mf_entry(p[0], p[1], k, &er, &ei);
          rc = (float)p[2];
          rs = (float)p[3];
          anchored = true;
        } else {
          // (er + j ei) * (rc - j rs)
          const float nr = __fmaf_rn(er, rc, __fmul_rn(ei, rs));
          const float ni = __fmaf_rn(ei, rc, -__fmul_rn(er, rs));
          er = nr;
          ei = ni;
        }
        re[r] = er;
        im[r] = ei;
      } else {
        re[r] = 0.f;
        im[r] = 0.f;
      }
      if (++k == K) { k = 0; ++m; anchored = false; }
    }
  }
  // Anchor of the group of rows m*K + k .. m*K + k + 7 (K and k multiples
  // of 8, so the group lies within receiver m): its first entry and the
  // per-row rotation exp(-j 2 pi d_m) = rc - j rs; zero for padding rows
  // (m >= M).  The products that take it rotate their own running term
  // instead of the entry (same entries up to FP32 rounding).
  __device__ static inline void anchor(const void* col, int m, int k, int M, float* ar, float* ai,
                                       float* rc, float* rs) {
    if (m < M) {
      const double* p = reinterpret_cast<const double*>(col) + MF_REC_BASE + MF_REC_PER_RX * m;
      mf_entry(p[0], p[1], k, ar, ai);
      *rc = (float)p[2];
      *rs = (float)p[3];
    } else {
      *ar = 0.f; *ai = 0.f; *rc = 0.f; *rs = 0.f;
    }
  }
  __device__ static inline cd get(const void* col, int i, int KM) {
    const int g = i & ~(RPT - 1);
    float re[RPT], im[RPT];
    load(col, g, KM, re, im);
    float vr = re[0], vi = im[0];
#pragma unroll
    for (int r = 1; r < RPT; ++r)
      if (i - g == r) { vr = re[r]; vi = im[r]; }
    return {(double)vr, (double)vi};
  }
  __device__ static inline cd get_stream(const void* col, int i, int KM) { return get(col, i, KM); }
};

// Address of column `n` for a storage with leading dimension ld (in slots).
template <int ST> __device__ inline const void* col_ptr(const void* base, int64_t ld, int64_t n) {
  if constexpr (ST == ST_FP64) return reinterpret_cast<const double2*>(base) + ld * n;
  else if constexpr (ST == ST_FP32) return reinterpret_cast<const float2*>(base) + ld * n;
  else if constexpr (ST == ST_MF) return reinterpret_cast<const double*>(base) + ld * n;
  else return reinterpret_cast<const uint16_t*>(base) + ld * n;
}

// ---------------------------------------------------------------- reductions
template <class T> __device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, SADMM_WAVE);
  return v;
}

// Deterministic block sum of NV values per thread (blockDim.x = 256).
// Result valid in thread 0.  `sm` must hold 4*NV values.
template <class T, int NV> __device__ inline void block_sum256(T (&v)[NV], T* sm) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) sm[w * NV + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = ((sm[j] + sm[NV + j]) + sm[2 * NV + j]) + sm[3 * NV + j];
  }
  __syncthreads();
}

// Device control block shared by all per-iteration kernels.
struct Ctl {
  int k;            // completed iterations
  int halt;         // bit mask of HALT_* : set => per-iteration kernels do nothing
  int gate;         // r <= eps_pri at the last iteration
  int nan;          // non-finite value seen
  int gone_total;   // pixels SSC decided to eliminate at the last iteration
  int max_iter;
  int bal;          // residual balancing at the last iteration: +1 beta up, -1 down, 0 none
  unsigned pix_done;   // pixel-update blocks finished this iteration (the last one resets it)
  unsigned ssc_done;   // SSC-check blocks finished this iteration (the last one resets it)
  int pad;
  double r, s, eps_pri, eps_dual, nmse;
};
enum : int { HALT_CONV = 1, HALT_PRUNE = 2, HALT_MAXIT = 4, HALT_NAN = 8, HALT_NMSE = 16, HALT_BAL = 32 };
