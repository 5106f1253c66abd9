// Data movement kernels: operator ingest (conversion, LFM generation), stream
// compaction of the SSC selectors, column gathers, small fills.
#pragma once
#include "common.h"

// Convert a caller operator (complex128 if src_c128 else complex64, column
// stride src_ld complex entries, KM x N) into storage `st` with column stride
// ldA slots and KMp rows (rows KM..KMp-1 zero).
void convert_operator(const void* src, bool src_c128, int64_t src_ld, int KM, int N, int st,
                      void* dst, int64_t ldA, int KMp, hipStream_t s);

// Generate A[m*K+k, n] = exp(-j 2 pi f_k tau_{m,n}) on the device (eq. (1)).
// tx: 2 doubles, rx: 2*M doubles, pix: 2*N doubles (device).
void geometry_operator(const double* tx, const double* rx, const double* pix, int M, int K, int N,
                       double f0, double bw, int st, void* dst, int64_t ldA, int KMp,
                       hipStream_t s);

// Matrix-free operator records (per pixel: K, M, then per receiver frac(f0 tau_m),
// frac(bw tau_m / K) and the cosine and sine of 2 pi times the latter), column
// stride ld doubles (>= 2 + 4M).
void mf_records(const double* tx, const double* rx, const double* pix, int M, int K, int N, double f0,
                double bw, double* rec, int64_t ld, hipStream_t s);

// Stable partition of n flags: kept[] receives in[i] (or i when in is null)
// for flag[i] != 0 in order, dropped[] the others in order (either output may
// be null); counts[0] = #kept, counts[1] = #dropped.  One work-group.
void partition_flags(const uint8_t* flag, const int* in, int n, int* kept, int* dropped,
                     int* counts, hipStream_t s);

// dst[:, p] = src[:, idx[p]] for p < count (whole columns of `slots` slots).
void gather_columns(const void* src, void* dst, int64_t ld, int64_t slot_bytes, const int* idx,
                    int count, hipStream_t s);

// dst (complex128, ld KMp) [:, p] = src[:, idx[p]] converted from storage st.
void gather_columns_fp64(const void* src, int64_t ldA, int st, int KMp, const int* idx, int count,
                         cd* dst, hipStream_t s);

// Small element-wise helpers on (q, index list) sets.
void set_bytes_at(uint8_t* base, const int* idx, int count, uint8_t v, hipStream_t s);
void zero_complex_at(void* base, bool dbl, const int* idx, int count, hipStream_t s);
void set_ring_inf(void* D, bool dbl, int Kp, int Q, int N, int q, const int* idx, int count,
                  hipStream_t s);
void iota_int(int* dst, int n, hipStream_t s);
// out[0] (device) = sum |a_i - b_i|^2 over n complex128 entries
void diff_norm2_c128(const double* a, const double* b, int64_t n, double* out, hipStream_t s);
void diff_norm2_c64(const float* a, const float* b, int64_t n, double* out, hipStream_t s);
void maxabs_c(const void* x, bool dbl, int64_t n, double* out, hipStream_t s);
void bp_sum(const double* c, int Q, int64_t N, double* out, hipStream_t s);
// flag[p] = |g_p| > thr (complex128 g)
void grad_flag(const double* g, int n, double thr, uint8_t* flag, hipStream_t s);
void stack_real(const void* src, bool c128, int64_t rows, int64_t cols, int64_t ld, double* dst, hipStream_t s);
// out[0] = |F (a - b)[J]|^2 (F Hermitian nq x nq, leading dimension fld)
void herm_apply_norm2(const double* F, int fld, int nq, const int* J, const double* a, const double* b,
                      double* out, hipStream_t s);
// max |x| into mx[0], then out[i] = number of thr[L] * mx (L < 255) <= |x_i|
void render_levels(const double* x, bool cplx, int64_t n, const double* thr, double* mx, uint8_t* out,
                   hipStream_t s);
// dst = src * scale (complex128 vectors of n entries)
void scale_c128(const double* src, double* dst, int n, double scale, hipStream_t s);
// x *= scale over n complex entries in place (complex128 when dbl, else complex64)
void scale_cplx(void* x, bool dbl, int64_t n, double scale, hipStream_t s);
// complex copy with precision change: dst (T) = src (complex128) for n entries
void c128_to_compute(const double* src, void* dst, bool dbl, int n, hipStream_t s);
void compute_to_c128(const void* src, bool dbl, double* dst, int n, hipStream_t s);
void compute_to_c64(const void* src, bool dbl, float* dst, int n, hipStream_t s);
void c64_to_compute(const float* src, void* dst, bool dbl, int n, hipStream_t s);
// y (c128 or c64, Q x KM) -> dst complex128 Q x KMp zero padded
void load_measurements(const void* src, bool src_c128, int Q, int KM, int KMp, double* dst,
                       hipStream_t s);
