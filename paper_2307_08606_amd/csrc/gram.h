// Gram Ahat Ahat^H of an operator held in FP32, FP16, BF16 or matrix-free
// form, computed exactly in integers on the int8 matrix instructions.
//
// Every entry is rounded to a 30-bit fixed-point integer relative to its row
// (q = round(x * 2^(30 - e_i)), 2^e_i >= the row's largest |Re| or |Im|) and
// written as four signed base-256 digits d_0..d_3 (q = sum_s d_s 256^(3-s)).
// The Gram is the double sum over digit pairs (s, t) of int8 x int8 products
// accumulated in int32, scaled by 2^(e_i + e_j - 12 - 8 (s + t)).  Pairs with
// s + t >= 5 weigh at most 2^-40 of the leading term and are skipped (keeping
// s + t = 4 matters: its products reach 2^-28 of the leading one, which the
// inverse of the factor amplifies by its condition number).  The only
// roundings are the 30-bit fixed point (far below the 24-bit significand of
// the stored FP32 values) and the final FP64 sum of five class terms.
#pragma once
#include "common.h"

// Columns per launch: keeps every int32 accumulator below 2^30.
constexpr int GI8_CHUNK = 8192;

struct GramI8Desc {
  const void* A;     // operator (storage st), column stride ldA slots
  int64_t ldA;
  int kmp;           // rows of the stored operator (plane offset of planar storage)
  int m;             // rows of Ahat (= order of the Gram), <= kmp
  int k;             // columns (active pixels)
  int KMr;           // m rounded up to 64: rows of the digit planes
  int ldS;           // columns of the digit planes: k rounded up to 128
  int8_t* S;         // 8 planes [digit s][re, im] of KMr x ldS bytes, stored in
                     // 32 KB blocks per (64-row block, 64-column stage)
  unsigned long long* rmax;   // KMr: bits of the row's largest |Re| or |Im| (FP64)
  int* rs;           // [chunk][digit t][KMr]: sum over the chunk of imaginary digits
  cd* C;             // output, m x m, column-major, ld = ldc
  int64_t ldc;
  double diag;       // added to the diagonal
};

// Device bytes of the workspace (S, rmax, rs) of one operator.
size_t gram_i8_workspace(int m, int k);
// Carve the workspace at `base` into d.S, d.rmax, d.rs (sets KMr, ldS).
void gram_i8_layout(GramI8Desc& d, void* base);

// C = Ahat Ahat^H + diag I for a batch of operators, in two phases.
// gram_i8_prepare: row scales and digit planes (reads the operator once).
// gram_i8_chunk:   the int8 products of columns [c * GI8_CHUNK, +GI8_CHUNK);
//                  chunk 0 writes C, later chunks add to it (launch them in
//                  order, c < gram_i8_chunks(max_k)).
// d_desc: device copy of the descriptors; max_m / max_k: largest m and k in
// the batch; tiles: device copy of tri_tile_order(ceil(max_m / 64)) (linalg.h).
// rmax_given: d.rmax already holds bounds of the rows' largest |Re| or |Im|
// (any bound >= the maximum keeps the digits in range; the bound of the full
// operator serves its compacted copies), so the row maxima are not recomputed.
void gram_i8_prepare(const GramI8Desc* d_desc, int batch, int max_m, int max_k, int st,
                     bool rmax_given, hipStream_t s);
// Only the row maxima into d.rmax (KMr entries; d.S and d.rs are not used).
void gram_i8_rowmax(const GramI8Desc* d_desc, int batch, int max_m, int max_k, int st, hipStream_t s);
int gram_i8_chunks(int max_k);
// wide: the 32x32x32 instruction (else the 16x16x64 one; identical results).
void gram_i8_chunk(const GramI8Desc* d_desc, int batch, int chunk, const int2* tiles, int ntiles,
                   bool wide, hipStream_t s);
