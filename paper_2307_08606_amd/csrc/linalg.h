// FP64 complex linear algebra used to build and update the per-sensor factor
// W_q = ((c/mu) I + Ahat_q Ahat_q^H)^{-1} (x-update of eq. (3) in Woodbury form).
#pragma once
#include "common.h"

enum : int { OP_N = 0, OP_C = 1 };   // op(X) = X or X^H

// One problem of a batched C = alpha * op(A) * op(B) + beta * C (+ diag on the
// diagonal).  A and B are column-major in the storage given by the launcher's
// template arguments; C is complex128 column-major.  kmpA/kmpB: plane offset
// of planar 16-bit storage (rows per plane), ignored otherwise.
struct GemmDesc {
  const void* A;
  const void* B;
  cd* C;
  int m, n, k;
  int kmpA, kmpB;
  int64_t lda, ldb, ldc;
  double alpha_re, alpha_im, beta, diag;
};

// Batched GEMM launcher.  herm = true computes only tiles on or below the
// diagonal and mirrors them (C must then be Hermitian: m == n).
void zgemm_batched(const GemmDesc* d_desc, int batch, int max_m, int max_n, int sta, int stb,
                   int opa, int opb, bool herm, hipStream_t s);

// One matrix of a batched Hermitian-positive-definite inverse.
struct HpdDesc {
  cd* G;        // n_pad x n_pad column-major, ld = n_pad; rows/cols >= n hold identity.
                // In: the matrix.  Out: its inverse (both triangles).
  int n_pad;    // multiple of HPD_NB
  cd* D;        // scratch NB x n_pad: inverses of the diagonal Cholesky blocks
  cd* X;        // scratch n_pad x n_pad: X = L^{-1}
};
constexpr int HPD_NB = 32;
// G <- G^{-1} through the Cholesky factor G = L L^H: X = L^{-1}, G^{-1} = X^H X.
// *d_fail is set non-zero if a pivot is not positive (loss of definiteness).
void hpd_inverse_batched(const HpdDesc* d_desc, int batch, int max_npad, int* d_fail,
                         hipStream_t s);

// dst (T-complex, ld_dst) = (src + src^H) / 2 for n x n, src complex128 ld_src.
void cast_hermitian(const cd* src, int64_t ld_src, void* dst, int64_t ld_dst, int n,
                    bool to_float, hipStream_t s);

// G <- (G + G^H) / 2 in place (n x n, column-major, ld).
void hermitian_inplace(cd* G, int64_t ld, int n, hipStream_t s);

// G[i,i] += v for i < n; G[i,j] = (i==j) for n <= i or j < n_pad (identity padding).
void set_identity_pad(cd* G, int n, int n_pad, double diag_add, hipStream_t s);
