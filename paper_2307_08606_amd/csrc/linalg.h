// FP64 complex linear algebra used to build and update the per-sensor factor
// W_q = ((c/mu) I + Ahat_q Ahat_q^H)^{-1} (x-update of eq. (3) in Woodbury form).
#pragma once
#include <vector>

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

// One product of a batched FP64 complex GEMM on the matrix instructions,
// C = alpha op(A) op(B) + beta C, all column-major complex128.
struct MmDesc {
  const cd* A;
  const cd* B;
  cd* C;
  int m, n, k;
  int lda, ldb, ldc;
  double alpha_re, alpha_im, beta;
};

// Batched GEMM launcher.  herm = true computes only tiles on or below the
// diagonal and mirrors them (C must then be Hermitian: m == n).
void zgemm_batched(const GemmDesc* d_desc, int batch, int max_m, int max_n, int sta, int stb,
                   int opa, int opb, bool herm, hipStream_t s);

// C = alpha A B + beta C (FP64 matrix instructions, no transposes) for a batch
// of MmDesc products; max_m / max_n bound every product's m and n.
void zgemm_mfma_nn(const MmDesc* d_desc, int count, int max_m, int max_n, hipStream_t s);
// C = alpha A^H B + beta C, and its Hermitian form (lower triangle and mirror,
// C = alpha A^H A with B = A, m = n <= max_n).
void zgemm_mfma_cn(const MmDesc* d_desc, int count, int max_m, int max_n, hipStream_t s);
void zgemm_mfma_gram_cn(const MmDesc* d_desc, int count, int max_n, hipStream_t s);

// Order of the lower-triangle tiles (ti >= tj) of an nt x nt tile grid for the
// Hermitian products: blocks of 4 tile rows x 8 tile columns, so that the
// tiles one XCD runs together (work-groups are dealt to the 8 XCDs in turn,
// and XCD x takes a contiguous slice of this list) share row and column panels
// in its L2.
std::vector<int2> tri_tile_order(int nt);
// Work-group -> tile: XCD x = b % 8 takes list entries [x P, (x + 1) P),
// P = ceil(ntiles / 8); the grid has 8 P work-groups.
__device__ inline bool xcd_tile(const int2* tiles, int ntiles, int* ti, int* tj) {
  const int per = (ntiles + 7) >> 3;
  const int p = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (p >= ntiles) return false;
  const int2 t = tiles[p];
  *ti = t.x;
  *tj = t.y;
  return true;
}

// C = A A^H + diag I (Hermitian, FP64 matrix instructions) for operators in
// storage st; tiles: device copy of tri_tile_order(ceil(max_m / 64)).
void herk_batched(const GemmDesc* d_desc, int batch, int max_m, int st, const int2* tiles,
                  int ntiles, hipStream_t s);


// One matrix of a batched Hermitian-positive-definite inverse.
struct HpdDesc {
  cd* G;        // n_pad x n_pad column-major, ld = n_pad; rows/cols >= n hold identity.
                // In: the matrix.  Out: its inverse (both triangles).
  int n_pad;    // multiple of HPD_NB
  cd* D;        // scratch NB x n_pad: inverses of the diagonal Cholesky blocks
  cd* X;        // scratch n_pad x n_pad: X = L^{-1}
  cd* T;        // scratch n_pad * n_pad / 4: products of the triangular inverse
};
constexpr int HPD_NB = 32;
// Descriptors one matrix of order n_pad needs in the scratch d_mm below.
size_t hpd_mm_count(int n_pad);
// G <- G^{-1} through the Cholesky factor G = L L^H: X = L^{-1}, G^{-1} = X^H X.
// Blocked right-looking Cholesky (NB x NB diagonal blocks factored in LDS by
// the kernel that also forms the panel, trailing update as matrix-instruction
// GEMMs), X by recursive
// doubling (X21 = -X22 L21 X11 over blocks of 32, 64, ...), X^H X over the
// nonzero k-range of each tile.  All matrices of the batch have order n_pad.
// h_desc: host copies of the descriptors (d_desc on the device); d_mm: device
// scratch for batch * hpd_mm_count(n_pad) descriptors.  *d_fail is set
// non-zero if a pivot is not positive (loss of definiteness).
// form_w = false stops before W = X^H X: X = L^{-1} stays in the X scratch
// and G receives U = X^H instead (W t is then X^H (X t); see hpd_form_w).
void hpd_inverse_batched(const HpdDesc* h_desc, const HpdDesc* d_desc, int batch, int n_pad,
                         int* d_fail, MmDesc* d_mm, hipStream_t s, bool form_w = true);
// W = X^H X for `count` products C = X^H X (MmDesc: A = B = X, C = W, m = n = k
// = n_pad, ld n_pad, alpha 1, beta 0): the last step of the inverse, run later.
void hpd_form_w(const MmDesc* d_desc, int count, int n_pad, hipStream_t s);

// dst (T-complex, ld_dst) = (src + src^H) / 2 for n x n, src complex128 ld_src.
void cast_hermitian(const cd* src, int64_t ld_src, void* dst, int64_t ld_dst, int n,
                    bool to_float, hipStream_t s);

// G <- (G + G^H) / 2 in place (n x n, column-major, ld).
void hermitian_inplace(cd* G, int64_t ld, int n, hipStream_t s);

// G[i,i] += v for i < n; G[i,j] = (i==j) for n <= i or j < n_pad (identity padding).
void set_identity_pad(cd* G, int n, int n_pad, double diag_add, hipStream_t s);
