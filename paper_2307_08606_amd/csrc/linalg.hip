// FP64 complex linear algebra on the device: batched GEMM, the Hermitian Gram
// of the operator on the FP64 matrix instructions, and the Cholesky-based
// inverse of Hermitian positive definite matrices.
//
// These build W_q = ((c/mu) I + Ahat_q Ahat_q^H)^{-1}, the factor through which
// the ridge x-update of eq. (3) is applied in Woodbury form, and apply the
// low-rank corrections of W_q when SSC (Alg. 1) removes columns of Ahat_q or
// the optimality re-check puts them back.  MI355X has the same FP64 peak on
// the vector units as on the matrix units, but a register-blocked vector FMA
// tile needs one 16-byte LDS read per two FMAs and is capped by LDS bandwidth;
// the 16x16x4 FP64 instruction needs 8x fewer operand reads, so the Gram (the
// dominant cost of a factor build) runs on it.  The smaller products keep the
// vector kernel.
#include <algorithm>

#include "linalg.h"

namespace {

constexpr int TM = 64, TN = 64, TK = 16;

template <int ST, int OP>
__device__ inline cd load_op(const void* base, int64_t ld, int kmp, int row, int col) {
  // element (row, col) of op(X)
  if constexpr (OP == OP_N) {
    return Store<ST>::get(col_ptr<ST>(base, ld, col), row, kmp);
  } else {
    cd v = Store<ST>::get(col_ptr<ST>(base, ld, row), col, kmp);
    v.im = -v.im;
    return v;
  }
}

template <int STA, int STB, int OPA, int OPB, bool HERM>
__global__ __launch_bounds__(256) void zgemm_kernel(const GemmDesc* __restrict__ descs) {
  const GemmDesc d = descs[blockIdx.z];
  const int ti = blockIdx.x, tj = blockIdx.y;
  if (HERM && tj > ti) return;
  const int i0 = ti * TM, j0 = tj * TN;
  if (i0 >= d.m || j0 >= d.n) return;
  __shared__ cd sA[TK][TM + 1];
  __shared__ cd sB[TK][TN + 1];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  cd acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = {0.0, 0.0};

  for (int p0 = 0; p0 < d.k; p0 += TK) {
    // ---- stage op(A)[i0:i0+64, p0:p0+16] and op(B)[p0:p0+16, j0:j0+64]
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int ii, pp;
      if constexpr (OPA == OP_N) { ii = t & 63; pp = (t >> 6) + 4 * e; }
      else { pp = t & 15; ii = (t >> 4) + 16 * e; }
      const int gi = i0 + ii, gp = p0 + pp;
      cd v = {0.0, 0.0};
      if (gi < d.m && gp < d.k) v = load_op<STA, OPA>(d.A, d.lda, d.kmpA, gi, gp);
      sA[pp][ii] = v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int jj, pp;
      if constexpr (OPB == OP_N) { pp = t & 15; jj = (t >> 4) + 16 * e; }
      else { jj = t & 63; pp = (t >> 6) + 4 * e; }
      const int gj = j0 + jj, gp = p0 + pp;
      cd v = {0.0, 0.0};
      if (gj < d.n && gp < d.k) v = load_op<STB, OPB>(d.B, d.ldb, d.kmpB, gp, gj);
      sB[pp][jj] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TK; ++kk) {
      cd av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sA[kk][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sB[kk][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) cfma(acc[a][b], av[a], bv[b]);
    }
    __syncthreads();
  }
  // ---- epilogue: C = alpha*acc + beta*C (+diag)
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + tx + 16 * a;
    if (i >= d.m) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + ty + 16 * b;
      if (j >= d.n) continue;
      if (HERM && j > i) continue;
      cd v = {d.alpha_re * acc[a][b].re - d.alpha_im * acc[a][b].im,
              d.alpha_re * acc[a][b].im + d.alpha_im * acc[a][b].re};
      cd* cij = d.C + (int64_t)j * d.ldc + i;
      if (d.beta != 0.0) { v.re += d.beta * cij->re; v.im += d.beta * cij->im; }
      if (i == j) v.re += d.diag;
      if (HERM && i == j) v.im = 0.0;
      *cij = v;
      if (HERM && i != j) {
        cd* cji = d.C + (int64_t)i * d.ldc + j;
        *cji = {v.re, -v.im};
      }
    }
  }
}

// ------------------------------------------------------------------ HPD inverse
// W = G^{-1} for Hermitian positive definite G through its Cholesky factor:
//   1. blocked right-looking Cholesky G = L L^H (NB x NB diagonal blocks
//      factored in LDS, panel solve, rank-NB trailing update of the lower part)
//   2. X = L^{-1} by blocked forward substitution, block row by block row
//   3. W = X^H X
// All steps in FP64.  (Gauss-Jordan elimination without pivoting is
// unstable on the strongly correlated Gram matrices of radar operators.)

// Factor the diagonal block G[k0:k0+NB, k0:k0+NB] = Lkk Lkk^H in LDS; write
// Lkk into G (upper part zeroed) and Lkk^{-1} into Dinv[:, k0:k0+NB].
__global__ __launch_bounds__(256) void chol_diag_kernel(const HpdDesc* __restrict__ descs, int k0,
                                                        int* fail) {
  const HpdDesc h = descs[blockIdx.x];
  if (k0 >= h.n_pad) return;
  constexpr int NB = HPD_NB;
  __shared__ cd P[NB][NB + 1];    // P[c][r] = element (r, c)
  __shared__ cd Li[NB][NB + 1];   // Li[c][r] = element (r, c) of Lkk^{-1}
  __shared__ double sdiag;
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e % NB, c = e / NB;
    P[c][r] = h.G[(int64_t)(k0 + c) * h.n_pad + k0 + r];
  }
  __syncthreads();
  for (int c = 0; c < NB; ++c) {
    if (t == 0) {
      const double d = P[c][c].re;
      if (!(d > 0.0)) atomicOr(fail, 1);
      sdiag = sqrt(fmax(d, 1e-300));
    }
    __syncthreads();
    const double sd = sdiag;
    if (t > c && t < NB) P[c][t] = cscale(P[c][t], 1.0 / sd);   // column c below the diagonal
    if (t == c) P[c][c] = {sd, 0.0};
    __syncthreads();
    for (int e = t; e < NB * NB; e += 256) {
      const int r = e % NB, s2 = e / NB;
      if (s2 > c && r >= s2) {
        // (r, s2) -= L(r, c) conj(L(s2, c))
        const cd a = P[c][r], b = P[c][s2];
        cd v = P[s2][r];
        v.re -= a.re * b.re + a.im * b.im;
        v.im -= a.im * b.re - a.re * b.im;
        P[s2][r] = v;
      }
    }
    __syncthreads();
  }
  // column j of Lkk^{-1} by forward substitution (one thread per column)
  if (t < NB) {
    const int j = t;
    for (int r = 0; r < j; ++r) Li[j][r] = {0.0, 0.0};
    const double djj = P[j][j].re;
    Li[j][j] = {1.0 / djj, 0.0};
    for (int r = j + 1; r < NB; ++r) {
      cd acc = {0.0, 0.0};
      for (int k = j; k < r; ++k) cfma(acc, P[k][r], Li[j][k]);
      Li[j][r] = cscale(acc, -1.0 / P[r][r].re);
    }
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e % NB, c = e / NB;
    h.G[(int64_t)(k0 + c) * h.n_pad + k0 + r] = (r >= c) ? P[c][r] : cd{0.0, 0.0};
    h.D[(int64_t)(k0 + c) * NB + r] = Li[c][r];
  }
}

// Panel: L[i, kb] = G[i, kb] Lkk^{-H} for rows i >= k0 + NB (in place).
__global__ __launch_bounds__(256) void chol_panel_kernel(const HpdDesc* __restrict__ descs, int k0) {
  const HpdDesc h = descs[blockIdx.y];
  constexpr int NB = HPD_NB;
  if (k0 >= h.n_pad) return;
  __shared__ cd Ls[NB][NB + 1];   // Ls[c][r] = element (r, c) of Lkk^{-1}
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 256) Ls[e / NB][e % NB] = h.D[(int64_t)k0 * NB + e];
  __syncthreads();
  const int i = k0 + NB + blockIdx.x * 256 + t;
  if (i >= h.n_pad) return;
  cd g[NB];
  for (int s2 = 0; s2 < NB; ++s2) g[s2] = h.G[(int64_t)(k0 + s2) * h.n_pad + i];
  for (int c = 0; c < NB; ++c) {
    cd acc = {0.0, 0.0};
    for (int s2 = 0; s2 <= c; ++s2) cfmac(acc, Ls[s2][c], g[s2]);   // g[s2] * conj(Linv(c, s2))
    h.G[(int64_t)(k0 + c) * h.n_pad + i] = acc;
  }
}

// Trailing update of the lower part: G[i, j] -= L[i, kb] L[j, kb]^H,
// i >= j >= k0 + NB.  K = NB in two halves (33 KB of LDS).
__global__ __launch_bounds__(256) void chol_update_kernel(const HpdDesc* __restrict__ descs, int k0) {
  const HpdDesc h = descs[blockIdx.z];
  constexpr int NB = HPD_NB;
  constexpr int HB = NB / 2;
  const int ti = blockIdx.x, tj = blockIdx.y;
  if (tj > ti) return;
  const int base = k0 + NB;
  const int i0 = base + ti * TM, j0 = base + tj * TN;
  if (i0 >= h.n_pad || j0 >= h.n_pad) return;
  __shared__ cd sC[HB][TM + 1];
  __shared__ cd sR[HB][TN + 1];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  cd acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = {0.0, 0.0};
  for (int h0 = 0; h0 < NB; h0 += HB) {
    for (int e = t; e < HB * TM; e += 256) {
      const int ii = e % TM, c = e / TM;
      const int gi = i0 + ii;
      sC[c][ii] = gi < h.n_pad ? h.G[(int64_t)(k0 + h0 + c) * h.n_pad + gi] : cd{0.0, 0.0};
    }
    for (int e = t; e < HB * TN; e += 256) {
      const int jj = e % TN, c = e / TN;
      const int gj = j0 + jj;
      cd v = gj < h.n_pad ? h.G[(int64_t)(k0 + h0 + c) * h.n_pad + gj] : cd{0.0, 0.0};
      v.im = -v.im;
      sR[c][jj] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < HB; ++c) {
      cd av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sC[c][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sR[c][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) cfma(acc[a][b], av[a], bv[b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + tx + 16 * a;
    if (i >= h.n_pad) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + ty + 16 * b;
      if (j >= h.n_pad || j > i) continue;
      cd* g = h.G + (int64_t)j * h.n_pad + i;
      *g = csub(*g, acc[a][b]);
    }
  }
}

// Block row ib of X = L^{-1} (X zero-initialised, lower triangular):
//   X[ib, jb] = -Lib,ib^{-1} sum_{k = jb..ib-1} L[ib, k] X[k, jb]   (jb < ib)
//   X[ib, ib] = Lib,ib^{-1}
// One work-group per NB x NB output tile.
__global__ __launch_bounds__(256) void trtri_row_kernel(const HpdDesc* __restrict__ descs, int i0) {
  const HpdDesc h = descs[blockIdx.y];
  constexpr int NB = HPD_NB;
  if (i0 >= h.n_pad) return;
  const int j0 = blockIdx.x * NB;
  if (j0 > i0) return;
  __shared__ cd sL[NB][NB + 1];   // sL[k][r] = L(i0 + r, k0 + k)
  __shared__ cd sX[NB][NB + 1];   // sX[c][k] = X(k0 + k, j0 + c)
  __shared__ cd sT[NB][NB + 1];   // sT[c][r] = T(r, c)
  const int t = threadIdx.x;
  cd* X = h.X;
  if (j0 == i0) {
    for (int e = t; e < NB * NB; e += 256) {
      const int r = e % NB, c = e / NB;
      X[(int64_t)(i0 + c) * h.n_pad + i0 + r] = h.D[(int64_t)(i0 + c) * NB + r];
    }
    return;
  }
  // each thread owns 4 outputs: rows r = t % NB, columns c = t / NB + 8 * q4
  const int r = t % NB, cb = t / NB;
  cd acc[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  for (int k0 = j0; k0 < i0; k0 += NB) {
    for (int e = t; e < NB * NB; e += 256) {
      const int rr = e % NB, cc = e / NB;
      sL[cc][rr] = h.G[(int64_t)(k0 + cc) * h.n_pad + i0 + rr];
      sX[cc][rr] = X[(int64_t)(j0 + cc) * h.n_pad + k0 + rr];
    }
    __syncthreads();
    for (int k = 0; k < NB; ++k) {
      const cd lv = sL[k][r];
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) cfma(acc[q4], lv, sX[cb + 8 * q4][k]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) sT[cb + 8 * q4][r] = acc[q4];
  for (int e = t; e < NB * NB; e += 256) {
    const int rr = e % NB, cc = e / NB;
    sL[cc][rr] = h.D[(int64_t)(i0 + cc) * NB + rr];     // Lii^{-1}
  }
  __syncthreads();
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    const int c = cb + 8 * q4;
    cd v = {0.0, 0.0};
    for (int s2 = 0; s2 <= r; ++s2) cfma(v, sL[s2][r], sT[c][s2]);
    X[(int64_t)(j0 + c) * h.n_pad + i0 + r] = {-v.re, -v.im};
  }
}

__global__ void zero_x_kernel(const HpdDesc* __restrict__ descs) {
  const HpdDesc h = descs[blockIdx.y];
  const int64_t n2 = (int64_t)h.n_pad * h.n_pad;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (int64_t)gridDim.x * 256)
    h.X[e] = {0.0, 0.0};
}

// W = X^H X into G (lower tiles computed, mirrored to the upper part).
__global__ __launch_bounds__(256) void xhx_kernel(const HpdDesc* __restrict__ descs) {
  const HpdDesc h = descs[blockIdx.z];
  const int ti = blockIdx.x, tj = blockIdx.y;
  if (tj > ti) return;
  const int i0 = ti * TM, j0 = tj * TN;
  if (i0 >= h.n_pad || j0 >= h.n_pad) return;
  __shared__ cd sA[TK][TM + 1];
  __shared__ cd sB[TK][TN + 1];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  cd acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = {0.0, 0.0};
  // W[i, j] = sum_k conj(X[k, i]) X[k, j]; X lower triangular: k >= max(i, j) >= j0
  for (int p0 = (j0 / TK) * TK; p0 < h.n_pad; p0 += TK) {
    for (int e = t; e < TK * TM; e += 256) {
      const int pp = e % TK, ii = e / TK;
      const int gi = i0 + ii, gp = p0 + pp;
      cd v = (gi < h.n_pad && gp < h.n_pad) ? h.X[(int64_t)gi * h.n_pad + gp] : cd{0.0, 0.0};
      v.im = -v.im;
      sA[pp][ii] = v;
    }
    for (int e = t; e < TK * TN; e += 256) {
      const int pp = e % TK, jj = e / TK;
      const int gj = j0 + jj, gp = p0 + pp;
      sB[pp][jj] = (gj < h.n_pad && gp < h.n_pad) ? h.X[(int64_t)gj * h.n_pad + gp] : cd{0.0, 0.0};
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TK; ++kk) {
      cd av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sA[kk][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sB[kk][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) cfma(acc[a][b], av[a], bv[b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + tx + 16 * a;
    if (i >= h.n_pad) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + ty + 16 * b;
      if (j >= h.n_pad || j > i) continue;
      cd v = acc[a][b];
      if (i == j) v.im = 0.0;
      h.G[(int64_t)j * h.n_pad + i] = v;
      if (i != j) h.G[(int64_t)i * h.n_pad + j] = {v.re, -v.im};
    }
  }
}

__global__ void cast_herm_kernel(const cd* __restrict__ src, int64_t lds, void* dst, int64_t ldd,
                                 int n, int to_float) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const cd a = src[(int64_t)j * lds + i];
  const cd b = src[(int64_t)i * lds + j];
  cd v = {0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
  if (i == j) v.im = 0.0;
  if (to_float) reinterpret_cast<float2*>(dst)[(int64_t)j * ldd + i] = make_float2((float)v.re, (float)v.im);
  else reinterpret_cast<double2*>(dst)[(int64_t)j * ldd + i] = make_double2(v.re, v.im);
}

__global__ void herm_inplace_kernel(cd* G, int64_t ld, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n || i < j) return;
  cd* a = G + (int64_t)j * ld + i;
  if (i == j) { a->im = 0.0; return; }
  cd* b = G + (int64_t)i * ld + j;
  const cd v = {0.5 * (a->re + b->re), 0.5 * (a->im - b->im)};
  *a = v;
  *b = {v.re, -v.im};
}

__global__ void identity_pad_kernel(cd* G, int n, int n_pad, double diag_add) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n_pad) return;
  cd* g = G + (int64_t)j * n_pad + i;
  if (i < n && j < n) {
    if (i == j) g->re += diag_add;
  } else {
    *g = {i == j ? 1.0 : 0.0, 0.0};
  }
}

// ------------------------------------------------------------------ Gram on MFMA
// C = alpha * A B^H + beta * C (+ diag) for C Hermitian (B = A for the Gram of
// the operator), on the FP64 16x16x4 matrix instruction.  Complex products are
// split into real ones: with L = rows i of A and R = rows j of B,
//   Re C = Lr Rr^T + Li Ri^T,   Im C = Li Rr^T - Lr Ri^T.
// Work-group: 64 x 64 complex tile of the lower triangle (tile order of
// tri_tile_order, dealt to XCDs by xcd_tile), four waves of 32 x 32 (2 x 2 blocks of 16 x 16).  Panels of
// HK pixel columns are staged in LDS as FP64 real/imaginary planes; the next
// panel is fetched into registers while the current one is multiplied.
// Operand lane layout of the instruction: lane l carries A[l % 16][l / 16] and
// B[l / 16][l % 16]; the result block's element (4 r + l / 16, l % 16) is
// component r of lane l.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int HM = 64, HK = 32, HLD = 80;   // HLD: padded LDS row of doubles
constexpr int HPF = HK / 4;                  // panel elements per thread

// Panel staging: each thread fetches HPF elements of a 64-row x HK-column panel
// (rows contiguous across lanes) into registers, then stores them to LDS as
// FP64 real/imaginary planes.
template <int ST>
__device__ inline void fetch_panel(const void* base, int64_t ld, int kmp, int r0, int rows, int p0,
                                   int k, cd (&v)[HPF]) {
  const int t = threadIdx.x;
  const int gr = r0 + (t & 63);
#pragma unroll
  for (int e = 0; e < HPF; ++e) {
    const int gp = p0 + (t >> 6) + 4 * e;
    v[e] = cd{0.0, 0.0};
    if (gr < rows && gp < k) v[e] = Store<ST>::get(col_ptr<ST>(base, ld, gp), gr, kmp);
  }
}
__device__ inline void store_panel(const cd (&v)[HPF], double (*dst)[HK][HLD]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < HPF; ++e) {
    const int pp = (t >> 6) + 4 * e;
    dst[0][pp][t & 63] = v[e].re;
    dst[1][pp][t & 63] = v[e].im;
  }
}

template <int ST>
__global__ __launch_bounds__(256) void herk_mfma_kernel(const GemmDesc* __restrict__ descs,
                                                         const int2* __restrict__ tiles, int ntiles) {
  const GemmDesc d = descs[blockIdx.y];
  int ti, tj;
  if (!xcd_tile(tiles, ntiles, &ti, &tj)) return;
  const int i0 = ti * HM, j0 = tj * HM;
  if (i0 >= d.m) return;
  __shared__ double sL[2][HK][HLD];
  __shared__ double sR[2][HK][HLD];
  // a diagonal tile of a Gram reads one panel
  const bool same = ti == tj && d.A == d.B && d.lda == d.ldb;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  const int c16 = lane & 15, kq = lane >> 4;
  v4d cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      ci[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  double (*R)[HK][HLD] = same ? sL : sR;
  cd vl[HPF], vr[HPF];
  fetch_panel<ST>(d.A, d.lda, d.kmpA, i0, d.m, 0, d.k, vl);
  if (!same) fetch_panel<ST>(d.B, d.ldb, d.kmpB, j0, d.n, 0, d.k, vr);
  for (int p0 = 0; p0 < d.k; p0 += HK) {
    __syncthreads();                       // previous panel consumed
    store_panel(vl, sL);
    if (!same) store_panel(vr, sR);
    __syncthreads();
    if (p0 + HK < d.k) {                   // next panel in flight during the products
      fetch_panel<ST>(d.A, d.lda, d.kmpA, i0, d.m, p0 + HK, d.k, vl);
      if (!same) fetch_panel<ST>(d.B, d.ldb, d.kmpB, j0, d.n, p0 + HK, d.k, vr);
    }
#pragma unroll
    for (int kk = 0; kk < HK; kk += 4) {
      double lr[2], li[2], nlr[2], rr[2], ri[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        lr[a] = sL[0][kk + kq][wr + 16 * a + c16];
        li[a] = sL[1][kk + kq][wr + 16 * a + c16];
        nlr[a] = -lr[a];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        rr[b] = R[0][kk + kq][wc + 16 * b + c16];
        ri[b] = R[1][kk + kq][wc + 16 * b + c16];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lr[a], rr[b], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(li[a], rr[b], ci[a][b], 0, 0, 0);
        }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(li[a], ri[b], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(nlr[a], ri[b], ci[a][b], 0, 0, 0);
        }
    }
  }
  // ---- epilogue: lower triangle and its mirror
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + 16 * a + 4 * r + kq;
        const int j = j0 + wc + 16 * b + c16;
        if (i >= d.m || j >= d.n || j > i) continue;
        const double ar = cr[a][b][r], ai = ci[a][b][r];
        cd v = {d.alpha_re * ar - d.alpha_im * ai, d.alpha_re * ai + d.alpha_im * ar};
        cd* cij = d.C + (int64_t)j * d.ldc + i;
        if (d.beta != 0.0) { v.re += d.beta * cij->re; v.im += d.beta * cij->im; }
        if (i == j) { v.re += d.diag; v.im = 0.0; }
        *cij = v;
        if (i != j) d.C[(int64_t)i * d.ldc + j] = cd{v.re, -v.im};
      }
}

template <int ST>
void launch_herk_mfma(const GemmDesc* d, int batch, const int2* tiles, int ntiles, hipStream_t s) {
  herk_mfma_kernel<ST><<<dim3(8 * ((ntiles + 7) / 8), batch), 256, 0, s>>>(d, tiles, ntiles);
}

template <int STA, int STB, int OPA, int OPB, bool HERM>
void launch_gemm(const GemmDesc* d, int batch, int mm, int mn, hipStream_t s) {
  dim3 grid((mm + TM - 1) / TM, (mn + TN - 1) / TN, batch);
  zgemm_kernel<STA, STB, OPA, OPB, HERM><<<grid, 256, 0, s>>>(d);
}

}  // namespace

void zgemm_batched(const GemmDesc* d_desc, int batch, int max_m, int max_n, int sta, int stb,
                   int opa, int opb, bool herm, hipStream_t s) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  // Instantiated combinations: FP64 x FP64 products for the low-rank factor
  // corrections (the Gram of the operator has its own launcher, herk_batched).
  if (sta == ST_FP64 && stb == ST_FP64 && !herm) {
    if (opa == OP_N && opb == OP_N) { launch_gemm<ST_FP64, ST_FP64, OP_N, OP_N, false>(d_desc, batch, max_m, max_n, s); return; }
    if (opa == OP_C && opb == OP_N) { launch_gemm<ST_FP64, ST_FP64, OP_C, OP_N, false>(d_desc, batch, max_m, max_n, s); return; }
    if (opa == OP_N && opb == OP_C) { launch_gemm<ST_FP64, ST_FP64, OP_N, OP_C, false>(d_desc, batch, max_m, max_n, s); return; }
  }
  if (sta == ST_FP64 && stb == ST_FP64 && herm && opa == OP_C && opb == OP_N) {
    launch_gemm<ST_FP64, ST_FP64, OP_C, OP_N, true>(d_desc, batch, max_m, max_n, s); return;
  }
}

std::vector<int2> tri_tile_order(int nt) {
  constexpr int SR = 4, SC = 8;
  std::vector<int2> out;
  out.reserve((size_t)nt * (nt + 1) / 2);
  for (int I = 0; I * SR < nt; ++I) {
    const int r1 = std::min(nt, I * SR + SR);
    for (int J = 0; J * SC < r1; ++J)
      for (int ti = I * SR; ti < r1; ++ti)
        for (int tj = J * SC; tj < std::min(J * SC + SC, ti + 1); ++tj) out.push_back(make_int2(ti, tj));
  }
  return out;
}

void herk_batched(const GemmDesc* d_desc, int batch, int max_m, int st, const int2* tiles,
                  int ntiles, hipStream_t s) {
  if (batch <= 0 || max_m <= 0 || ntiles <= 0) return;
  switch (st) {
    case ST_FP64: launch_herk_mfma<ST_FP64>(d_desc, batch, tiles, ntiles, s); return;
    case ST_FP32: launch_herk_mfma<ST_FP32>(d_desc, batch, tiles, ntiles, s); return;
    case ST_FP16P: launch_herk_mfma<ST_FP16P>(d_desc, batch, tiles, ntiles, s); return;
    case ST_BF16P: launch_herk_mfma<ST_BF16P>(d_desc, batch, tiles, ntiles, s); return;
    case ST_MF: launch_herk_mfma<ST_MF>(d_desc, batch, tiles, ntiles, s); return;
  }
}

void hpd_inverse_batched(const HpdDesc* d_desc, int batch, int max_npad, int* d_fail,
                         hipStream_t s) {
  if (batch <= 0 || max_npad <= 0) return;
  zero_x_kernel<<<dim3(std::min<int64_t>(((int64_t)max_npad * max_npad + 255) / 256, 4096), batch), 256, 0, s>>>(d_desc);
  for (int k0 = 0; k0 < max_npad; k0 += HPD_NB) {
    chol_diag_kernel<<<batch, 256, 0, s>>>(d_desc, k0, d_fail);
    const int rest = max_npad - k0 - HPD_NB;
    if (rest > 0) {
      chol_panel_kernel<<<dim3((rest + 255) / 256, batch), 256, 0, s>>>(d_desc, k0);
      const int tiles = (rest + TM - 1) / TM;
      chol_update_kernel<<<dim3(tiles, tiles, batch), 256, 0, s>>>(d_desc, k0);
    }
  }
  for (int i0 = 0; i0 < max_npad; i0 += HPD_NB)
    trtri_row_kernel<<<dim3(i0 / HPD_NB + 1, batch), 256, 0, s>>>(d_desc, i0);
  const int tiles = (max_npad + TM - 1) / TM;
  xhx_kernel<<<dim3(tiles, tiles, batch), 256, 0, s>>>(d_desc);
}

void cast_hermitian(const cd* src, int64_t ld_src, void* dst, int64_t ld_dst, int n, bool to_float,
                    hipStream_t s) {
  if (n <= 0) return;
  cast_herm_kernel<<<dim3((n + 255) / 256, n), 256, 0, s>>>(src, ld_src, dst, ld_dst, n, to_float ? 1 : 0);
}

void hermitian_inplace(cd* G, int64_t ld, int n, hipStream_t s) {
  if (n <= 0) return;
  herm_inplace_kernel<<<dim3((n + 255) / 256, n), 256, 0, s>>>(G, ld, n);
}

void set_identity_pad(cd* G, int n, int n_pad, double diag_add, hipStream_t s) {
  if (n_pad <= 0) return;
  identity_pad_kernel<<<dim3((n_pad + 255) / 256, n_pad), 256, 0, s>>>(G, n, n_pad, diag_add);
}

