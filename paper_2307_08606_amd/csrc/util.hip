// Data movement kernels: operator ingest, SSC selector compaction, gathers.
#include "util.h"

namespace {

template <int ST> __device__ inline void store_entry(void* col, int i, int KMp, double re, double im) {
  if constexpr (ST == ST_FP64) {
    reinterpret_cast<double2*>(col)[i] = make_double2(re, im);
  } else if constexpr (ST == ST_FP32) {
    reinterpret_cast<float2*>(col)[i] = make_float2((float)re, (float)im);
  } else if constexpr (ST == ST_FP16P) {
    uint16_t* c = reinterpret_cast<uint16_t*>(col);
    c[i] = __half_as_ushort(__float2half((float)re));
    c[KMp + i] = __half_as_ushort(__float2half((float)im));
  } else {
    uint16_t* c = reinterpret_cast<uint16_t*>(col);
    c[i] = __bfloat16_as_ushort(__float2bfloat16((float)re));
    c[KMp + i] = __bfloat16_as_ushort(__float2bfloat16((float)im));
  }
}

template <int ST> __device__ inline void* col_wptr(void* base, int64_t ld, int64_t n) {
  return const_cast<void*>(col_ptr<ST>(base, ld, n));
}

template <int ST>
__global__ void convert_kernel(const void* src, int src_c128, int64_t src_ld, int KM, int N,
                               void* dst, int64_t ldA, int KMp) {
  const int n = blockIdx.x;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (n >= N || i >= KMp) return;
  double re = 0.0, im = 0.0;
  if (i < KM) {
    if (src_c128) {
      const double2 v = reinterpret_cast<const double2*>(src)[(int64_t)n * src_ld + i];
      re = v.x; im = v.y;
    } else {
      const float2 v = reinterpret_cast<const float2*>(src)[(int64_t)n * src_ld + i];
      re = v.x; im = v.y;
    }
  }
  store_entry<ST>(col_wptr<ST>(dst, ldA, n), i, KMp, re, im);
}

template <int ST>
__global__ void geometry_kernel(const double* tx, const double* rx, const double* pix, int M, int K,
                                int N, double f0, double bw, void* dst, int64_t ldA, int KMp) {
  const int n = blockIdx.x;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (n >= N || i >= KMp) return;
  double re = 0.0, im = 0.0;
  if (i < K * M) {
    const int m = i / K, k = i - m * K;
    const double px = pix[2 * n], py = pix[2 * n + 1];
    const double dt = hypot(px - tx[0], py - tx[1]);
    const double dr = hypot(px - rx[2 * m], py - rx[2 * m + 1]);
    const double tau = (dt + dr) / 299792458.0;
    const double f = f0 + bw * (double)k / (double)K;
    double cyc = f * tau;
    cyc = cyc - floor(cyc);
    double sn, cs;
    sincospi(2.0 * cyc, &sn, &cs);
    re = cs;
    im = -sn;
  }
  store_entry<ST>(col_wptr<ST>(dst, ldA, n), i, KMp, re, im);
}

// Matrix-free records (see Store<ST_MF>): one thread per pixel.
__global__ void mf_records_kernel(const double* tx, const double* rx, const double* pix, int M, int K,
                                  int N, double f0, double bw, double* rec, int64_t ld) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const double px = pix[2 * n], py = pix[2 * n + 1];
  const double dt = hypot(px - tx[0], py - tx[1]);
  double* r = rec + (int64_t)n * ld;
  r[0] = (double)K;
  r[1] = (double)M;
  for (int m = 0; m < M; ++m) {
    const double tau = (dt + hypot(px - rx[2 * m], py - rx[2 * m + 1])) / 299792458.0;
    const double a = f0 * tau, b = bw * tau / (double)K;
    double* p = r + MF_REC_BASE + MF_REC_PER_RX * m;
    p[0] = a - floor(a);
    p[1] = b - floor(b);
    double sn, cs;
    sincospi(2.0 * p[1], &sn, &cs);   // rotation from row k to k + 1
    p[2] = cs;
    p[3] = sn;
  }
}

// One work-group of 1024 threads walks the flags in tiles of 1024 with a
// running offset; wave ballots give the in-wave ranks.
__global__ __launch_bounds__(1024) void partition_kernel(const uint8_t* flag, const int* in, int n,
                                                         int* kept, int* dropped, int* counts) {
  __shared__ int wsum[16];
  __shared__ int base_keep;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) base_keep = 0;
  __syncthreads();
  for (int b0 = 0; b0 < n; b0 += 1024) {
    const int i = b0 + t;
    const bool valid = i < n;
    const bool f = valid && flag[i] != 0;
    const unsigned long long bal = __ballot(f);
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int rank = __popcll(bal & lt);
    if (lane == 0) wsum[w] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int v = 0; v < w; ++v) before += wsum[v];
    const int bk = base_keep;
    if (valid) {
      const int val = in ? in[i] : i;
      const int kpos = bk + before + rank;
      if (f) {
        if (kept) kept[kpos] = val;
      } else if (dropped) {
        dropped[i - kpos] = val;
      }
    }
    __syncthreads();
    if (t == 0) {
      int tot = 0;
      for (int v = 0; v < 16; ++v) tot += wsum[v];
      base_keep += tot;
    }
    __syncthreads();
  }
  if (t == 0) {
    counts[0] = base_keep;
    counts[1] = n - base_keep;
  }
}

__global__ void gather_cols_kernel(const uint4* src, uint4* dst, int64_t col_vecs, const int* idx,
                                   int count) {
  const int p = blockIdx.x;
  if (p >= count) return;
  const int64_t sc = (int64_t)idx[p] * col_vecs, dc = (int64_t)p * col_vecs;
  for (int64_t v = blockIdx.y * 256 + threadIdx.x; v < col_vecs; v += (int64_t)gridDim.y * 256)
    dst[dc + v] = src[sc + v];
}

template <int ST>
__global__ void gather_fp64_kernel(const void* src, int64_t ldA, int KMp, const int* idx, int count,
                                   cd* dst) {
  const int p = blockIdx.x;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (p >= count || i >= KMp) return;
  dst[(int64_t)p * KMp + i] = Store<ST>::get(col_ptr<ST>(src, ldA, idx[p]), i, KMp);
}

__global__ void set_bytes_kernel(uint8_t* base, const int* idx, int count, uint8_t v) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < count) base[idx[j]] = v;
}
__global__ void zero_complex_kernel(void* base, int dbl, const int* idx, int count) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= count) return;
  if (dbl) reinterpret_cast<double2*>(base)[idx[j]] = make_double2(0.0, 0.0);
  else reinterpret_cast<float2*>(base)[idx[j]] = make_float2(0.f, 0.f);
}
__global__ void ring_inf_kernel(void* D, int dbl, int Kp, int Q, int N, int q, const int* idx,
                                int count) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= count) return;
  for (int s = 0; s < Kp; ++s) {
    const int64_t o = ((int64_t)s * Q + q) * N + idx[j];
    if (dbl) reinterpret_cast<double*>(D)[o] = __builtin_huge_val();
    else reinterpret_cast<float*>(D)[o] = __builtin_huge_valf();
  }
}
__global__ void iota_kernel(int* dst, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = i;
}
__global__ void scale_f32_kernel(float* x, int64_t n, float sc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] *= sc;
}

__global__ void scale_c128_kernel(const double* src, double* dst, int n2, double sc) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n2) dst[i] = src[i] * sc;
}
__global__ void c128_to_compute_kernel(const double* src, void* dst, int dbl, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (dbl) reinterpret_cast<double2*>(dst)[i] = make_double2(src[2 * i], src[2 * i + 1]);
  else reinterpret_cast<float2*>(dst)[i] = make_float2((float)src[2 * i], (float)src[2 * i + 1]);
}
__global__ void compute_to_c128_kernel(const void* src, int dbl, double* dst, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (dbl) {
    const double2 v = reinterpret_cast<const double2*>(src)[i];
    dst[2 * i] = v.x; dst[2 * i + 1] = v.y;
  } else {
    const float2 v = reinterpret_cast<const float2*>(src)[i];
    dst[2 * i] = v.x; dst[2 * i + 1] = v.y;
  }
}
__global__ void compute_to_c64_kernel(const void* src, int dbl, float* dst, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (dbl) {
    const double2 v = reinterpret_cast<const double2*>(src)[i];
    dst[2 * i] = (float)v.x; dst[2 * i + 1] = (float)v.y;
  } else {
    const float2 v = reinterpret_cast<const float2*>(src)[i];
    dst[2 * i] = v.x; dst[2 * i + 1] = v.y;
  }
}
__global__ void c64_to_compute_kernel(const float* src, void* dst, int dbl, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (dbl) reinterpret_cast<double2*>(dst)[i] = make_double2(src[2 * i], src[2 * i + 1]);
  else reinterpret_cast<float2*>(dst)[i] = make_float2(src[2 * i], src[2 * i + 1]);
}
__global__ void load_meas_kernel(const void* src, int c128, int KM, int KMp, double* dst) {
  const int q = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= KMp) return;
  double re = 0.0, im = 0.0;
  if (i < KM) {
    if (c128) {
      const double2 v = reinterpret_cast<const double2*>(src)[(int64_t)q * KM + i];
      re = v.x; im = v.y;
    } else {
      const float2 v = reinterpret_cast<const float2*>(src)[(int64_t)q * KM + i];
      re = v.x; im = v.y;
    }
  }
  dst[2 * ((int64_t)q * KMp + i)] = re;
  dst[2 * ((int64_t)q * KMp + i) + 1] = im;
}

// out[0] = sum_i |a_i - b_i|^2 over n complex128 entries; one work-group of
// 1024 threads, fixed reduction order.
// |a - b|^2 over n interleaved complex entries (T = double or float),
// accumulated in FP64 by one work-group.
template <class T>
__global__ __launch_bounds__(1024) void diff_norm2_kernel(const T* a, const T* b, int64_t n,
                                                          double* out) {
  __shared__ double sm[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double dr = (double)a[2 * i] - (double)b[2 * i], di = (double)a[2 * i + 1] - (double)b[2 * i + 1];
    acc += dr * dr + di * di;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sm[w];
    out[0] = t;
  }
}

// max_i |x_i| over n interleaved complex entries (T = double or float), one
// work-group.
template <class T>
__global__ __launch_bounds__(1024) void maxabs_kernel(const T* x, int64_t n, double* out) {
  __shared__ double sm[16];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, hypot((double)x[2 * i], (double)x[2 * i + 1]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < 16; ++w) r = fmax(r, sm[w]);
    out[0] = r;
  }
}

// out[n] = |sum_q c[q N + n]| (c complex128, Q x N).
__global__ __launch_bounds__(256) void bp_sum_kernel(const double* __restrict__ c, int Q, int64_t N,
                                                     double* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  double re = 0.0, im = 0.0;
  for (int q = 0; q < Q; ++q) {
    re += c[2 * (q * N + n)];
    im += c[2 * (q * N + n) + 1];
  }
  out[n] = hypot(re, im);
}

// Rendering level of pixel n: the number of thresholds thr[L] * mx (L < 255,
// ascending) at or below |x_n|; x real (cplx = 0) or complex128.
__global__ __launch_bounds__(256) void level_kernel(const double* __restrict__ x, int cplx, int64_t n,
                                                   const double* __restrict__ thr, const double* __restrict__ mx,
                                                   uint8_t* __restrict__ out) {
  __shared__ double t[255];
  const double m = mx[0];
  for (int i = threadIdx.x; i < 255; i += 256) t[i] = thr[i] * m;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double v = cplx ? hypot(x[2 * i], x[2 * i + 1]) : fabs(x[i]);
  int lo = 0, hi = 255;                  // count of t[k] <= v: first k with t[k] > v
  if (m > 0.0) {
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (t[mid] <= v) lo = mid + 1;
      else hi = mid;
    }
  }
  out[i] = (uint8_t)lo;
}

// max |x_i| over n real doubles, one work-group.
__global__ __launch_bounds__(1024) void maxabs_real_kernel(const double* x, int64_t n, double* out) {
  __shared__ double sm[16];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, fabs(x[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < 16; ++w) r = fmax(r, sm[w]);
    out[0] = r;
  }
}

// out[0] += sum_p |sum_i conj(F[i, p]) (a - b)[J[i]]|^2 over p < nq: the
// squared norm of F (a - b) restricted to the active pixels J (F Hermitian,
// column-major with leading dimension fld; a, b complex128 by pixel).  One
// wave per column.
__global__ __launch_bounds__(256) void herm_apply_norm2_kernel(const double* __restrict__ F, int fld, int nq,
                                                              const int* __restrict__ J,
                                                              const double* __restrict__ a,
                                                              const double* __restrict__ b,
                                                              double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= nq) return;
  const double* col = F + 2 * (int64_t)p * fld;
  double re = 0.0, im = 0.0;
  for (int i = lane; i < nq; i += 64) {
    const int n = J[i];
    const double dr = a[2 * n] - b[2 * n], di = a[2 * n + 1] - b[2 * n + 1];
    const double fr = col[2 * i], fi = col[2 * i + 1];
    re += fr * dr + fi * di;     // conj(f) * d
    im += fr * di - fi * dr;
  }
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o);
    im += __shfl_xor(im, o);
  }
  if (lane == 0) atomicAdd(out, re * re + im * im);
}

// dst[n (2 rows) + i] = (Re S[i, n], 0), dst[n (2 rows) + rows + i] = (Im S[i, n], 0)
template <class T>
__global__ __launch_bounds__(256) void stack_real_kernel(const T* __restrict__ src, int64_t rows, int64_t cols,
                                                         int64_t ld, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t n = e / rows, i = e - n * rows;
  const T* s = src + 2 * (n * ld + i);
  double* d = dst + 2 * (n * 2 * rows + i);
  d[0] = (double)s[0];
  d[1] = 0.0;
  d[2 * rows] = (double)s[1];
  d[2 * rows + 1] = 0.0;
}

// flag[p] = |g_p| > thr (g complex128)
__global__ __launch_bounds__(256) void grad_flag_kernel(const double* __restrict__ g, int n, double thr,
                                                        uint8_t* __restrict__ flag) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < n) flag[p] = hypot(g[2 * p], g[2 * p + 1]) > thr ? 1 : 0;
}

inline int blocks(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

void diff_norm2_c128(const double* a, const double* b, int64_t n, double* out, hipStream_t s) {
  diff_norm2_kernel<double><<<1, 1024, 0, s>>>(a, b, n, out);
}

void herm_apply_norm2(const double* F, int fld, int nq, const int* J, const double* a, const double* b,
                      double* out, hipStream_t s) {
  hipMemsetAsync(out, 0, sizeof(double), s);
  if (nq > 0) herm_apply_norm2_kernel<<<(nq + 3) / 4, 256, 0, s>>>(F, fld, nq, J, a, b, out);
}

void stack_real(const void* src, bool c128, int64_t rows, int64_t cols, int64_t ld, double* dst, hipStream_t s) {
  const int64_t n = rows * cols;
  const unsigned g = (unsigned)((n + 255) / 256);
  if (c128) stack_real_kernel<double><<<g, 256, 0, s>>>(static_cast<const double*>(src), rows, cols, ld, dst);
  else stack_real_kernel<float><<<g, 256, 0, s>>>(static_cast<const float*>(src), rows, cols, ld, dst);
}

void grad_flag(const double* g, int n, double thr, uint8_t* flag, hipStream_t s) {
  if (n > 0) grad_flag_kernel<<<blocks(n), 256, 0, s>>>(g, n, thr, flag);
}

void bp_sum(const double* c, int Q, int64_t N, double* out, hipStream_t s) {
  bp_sum_kernel<<<blocks(N), 256, 0, s>>>(c, Q, N, out);
}

void render_levels(const double* x, bool cplx, int64_t n, const double* thr, double* mx, uint8_t* out,
                   hipStream_t s) {
  if (cplx) maxabs_kernel<double><<<1, 1024, 0, s>>>(x, n, mx);
  else maxabs_real_kernel<<<1, 1024, 0, s>>>(x, n, mx);
  level_kernel<<<blocks(n), 256, 0, s>>>(x, cplx ? 1 : 0, n, thr, mx, out);
}

void maxabs_c(const void* x, bool dbl, int64_t n, double* out, hipStream_t s) {
  if (dbl) maxabs_kernel<double><<<1, 1024, 0, s>>>(static_cast<const double*>(x), n, out);
  else maxabs_kernel<float><<<1, 1024, 0, s>>>(static_cast<const float*>(x), n, out);
}

void diff_norm2_c64(const float* a, const float* b, int64_t n, double* out, hipStream_t s) {
  diff_norm2_kernel<float><<<1, 1024, 0, s>>>(a, b, n, out);
}

void convert_operator(const void* src, bool src_c128, int64_t src_ld, int KM, int N, int st,
                      void* dst, int64_t ldA, int KMp, hipStream_t s) {
  dim3 g(N, blocks(KMp));
  switch (st) {
    case ST_FP64: convert_kernel<ST_FP64><<<g, 256, 0, s>>>(src, src_c128, src_ld, KM, N, dst, ldA, KMp); break;
    case ST_FP32: convert_kernel<ST_FP32><<<g, 256, 0, s>>>(src, src_c128, src_ld, KM, N, dst, ldA, KMp); break;
    case ST_FP16P: convert_kernel<ST_FP16P><<<g, 256, 0, s>>>(src, src_c128, src_ld, KM, N, dst, ldA, KMp); break;
    case ST_BF16P: convert_kernel<ST_BF16P><<<g, 256, 0, s>>>(src, src_c128, src_ld, KM, N, dst, ldA, KMp); break;
  }
}

void geometry_operator(const double* tx, const double* rx, const double* pix, int M, int K, int N,
                       double f0, double bw, int st, void* dst, int64_t ldA, int KMp,
                       hipStream_t s) {
  dim3 g(N, blocks(KMp));
  switch (st) {
    case ST_FP64: geometry_kernel<ST_FP64><<<g, 256, 0, s>>>(tx, rx, pix, M, K, N, f0, bw, dst, ldA, KMp); break;
    case ST_FP32: geometry_kernel<ST_FP32><<<g, 256, 0, s>>>(tx, rx, pix, M, K, N, f0, bw, dst, ldA, KMp); break;
    case ST_FP16P: geometry_kernel<ST_FP16P><<<g, 256, 0, s>>>(tx, rx, pix, M, K, N, f0, bw, dst, ldA, KMp); break;
    case ST_BF16P: geometry_kernel<ST_BF16P><<<g, 256, 0, s>>>(tx, rx, pix, M, K, N, f0, bw, dst, ldA, KMp); break;
  }
}

void mf_records(const double* tx, const double* rx, const double* pix, int M, int K, int N, double f0,
                double bw, double* rec, int64_t ld, hipStream_t s) {
  mf_records_kernel<<<(N + 255) / 256, 256, 0, s>>>(tx, rx, pix, M, K, N, f0, bw, rec, ld);
}

void partition_flags(const uint8_t* flag, const int* in, int n, int* kept, int* dropped,
                     int* counts, hipStream_t s) {
  partition_kernel<<<1, 1024, 0, s>>>(flag, in, n, kept, dropped, counts);
}

void gather_columns(const void* src, void* dst, int64_t ld, int64_t slot_bytes, const int* idx,
                    int count, hipStream_t s) {
  if (count <= 0) return;
  const int64_t col_vecs = ld * slot_bytes / 16;
  const int gy = (int)std::min<int64_t>((col_vecs + 255) / 256, 16);
  gather_cols_kernel<<<dim3(count, gy), 256, 0, s>>>(reinterpret_cast<const uint4*>(src),
                                                     reinterpret_cast<uint4*>(dst), col_vecs, idx, count);
}

void gather_columns_fp64(const void* src, int64_t ldA, int st, int KMp, const int* idx, int count,
                         cd* dst, hipStream_t s) {
  if (count <= 0) return;
  dim3 g(count, blocks(KMp));
  switch (st) {
    case ST_FP64: gather_fp64_kernel<ST_FP64><<<g, 256, 0, s>>>(src, ldA, KMp, idx, count, dst); break;
    case ST_FP32: gather_fp64_kernel<ST_FP32><<<g, 256, 0, s>>>(src, ldA, KMp, idx, count, dst); break;
    case ST_FP16P: gather_fp64_kernel<ST_FP16P><<<g, 256, 0, s>>>(src, ldA, KMp, idx, count, dst); break;
    case ST_BF16P: gather_fp64_kernel<ST_BF16P><<<g, 256, 0, s>>>(src, ldA, KMp, idx, count, dst); break;
    case ST_MF: gather_fp64_kernel<ST_MF><<<g, 256, 0, s>>>(src, ldA, KMp, idx, count, dst); break;
  }
}

void set_bytes_at(uint8_t* base, const int* idx, int count, uint8_t v, hipStream_t s) {
  if (count > 0) set_bytes_kernel<<<blocks(count), 256, 0, s>>>(base, idx, count, v);
}
void zero_complex_at(void* base, bool dbl, const int* idx, int count, hipStream_t s) {
  if (count > 0) zero_complex_kernel<<<blocks(count), 256, 0, s>>>(base, dbl ? 1 : 0, idx, count);
}
void set_ring_inf(void* D, bool dbl, int Kp, int Q, int N, int q, const int* idx, int count,
                  hipStream_t s) {
  if (count > 0) ring_inf_kernel<<<blocks(count), 256, 0, s>>>(D, dbl ? 1 : 0, Kp, Q, N, q, idx, count);
}
void iota_int(int* dst, int n, hipStream_t s) {
  if (n > 0) iota_kernel<<<blocks(n), 256, 0, s>>>(dst, n);
}
void scale_cplx(void* x, bool dbl, int64_t n, double scale, hipStream_t s) {
  if (n <= 0) return;
  if (dbl) scale_c128_kernel<<<blocks(2 * n), 256, 0, s>>>(static_cast<double*>(x), static_cast<double*>(x), (int)(2 * n), scale);
  else scale_f32_kernel<<<blocks(2 * n), 256, 0, s>>>(static_cast<float*>(x), 2 * n, (float)scale);
}

void scale_c128(const double* src, double* dst, int n, double scale, hipStream_t s) {
  if (n > 0) scale_c128_kernel<<<blocks(2 * (int64_t)n), 256, 0, s>>>(src, dst, 2 * n, scale);
}
void c128_to_compute(const double* src, void* dst, bool dbl, int n, hipStream_t s) {
  if (n > 0) c128_to_compute_kernel<<<blocks(n), 256, 0, s>>>(src, dst, dbl ? 1 : 0, n);
}
void compute_to_c128(const void* src, bool dbl, double* dst, int n, hipStream_t s) {
  if (n > 0) compute_to_c128_kernel<<<blocks(n), 256, 0, s>>>(src, dbl ? 1 : 0, dst, n);
}
void compute_to_c64(const void* src, bool dbl, float* dst, int n, hipStream_t s) {
  if (n > 0) compute_to_c64_kernel<<<blocks(n), 256, 0, s>>>(src, dbl ? 1 : 0, dst, n);
}
void c64_to_compute(const float* src, void* dst, bool dbl, int n, hipStream_t s) {
  if (n > 0) c64_to_compute_kernel<<<blocks(n), 256, 0, s>>>(src, dst, dbl ? 1 : 0, n);
}
void load_measurements(const void* src, bool src_c128, int Q, int KM, int KMp, double* dst,
                       hipStream_t s) {
  load_meas_kernel<<<dim3(blocks(KMp), Q), 256, 0, s>>>(src, src_c128 ? 1 : 0, KM, KMp, dst);
}
