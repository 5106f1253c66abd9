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
//   1. blocked right-looking Cholesky G = L L^H: NB x NB diagonal blocks
//      factored in LDS (with their inverses) by the kernel that also forms
//      the panel L21 = G21 Lkk^{-H}; the trailing update G22 -= L21 L21^H as
//      matrix-instruction GEMMs
//   2. X = L^{-1} by recursive doubling: with X11, X22 the inverses of two
//      adjacent diagonal blocks, the block below X11 is -X22 (L21 X11)
//   3. W = X^H X
// All steps in FP64.  (Gauss-Jordan elimination without pivoting is
// unstable on the strongly correlated Gram matrices of radar operators.)

// Factor the diagonal block G[k0:k0+NB, k0:k0+NB] = Lkk Lkk^H in LDS and
// form X = Lkk^{-1} alongside, CW = 4 columns c .. c + 3 per step.  Every
// thread derives the CW x CW pivot block l (Cholesky of P[c:c+4, c:c+4]) and
// the reciprocal diagonal rs.  Phase 1: thread NB + j turns rows c .. c + 3
// of Y (Y = I at the start) into rows of X by forward substitution with l:
// X[c + m, j] = (Y[c + m, j] - sum_{k<m} l[m, k] X[c + k, j]) rs[m].
// Phase 2: thread (r, s0) owns the entries (r, s0 + 8 j), j < 4, of both
// matrices, each either a factor entry (s > c + 3: P[r, s] -= sum_m L[r,
// c + m] L[s, c + m]^*) or an inverse entry (s <= c + 3: Y[r, s] -= sum_m
// L[r, c + m] X[c + m, s]), for r > c + 3; the rows of L in the current
// columns are formed on read by the same substitution (L[r, c + m] =
// (P[r, c + m] - sum_{k<m} L[r, c + k] l[m, k]^*) rs[m]) and not stored.  No
// entry is written that another thread reads in the same phase, so each
// thread's loads go out together.  Only Li (Li[c][r] = element (r, c) of Y,
// then of X) is the result; P[c][r] starts as element (r, c) of the block.
constexpr int DIAG_THREADS = 256;
constexpr int PANEL_ROWS = 64;   // panel rows per work-group
constexpr int CW = 4;            // columns per step of the diagonal factor
// 1 / sqrt(d): hardware reciprocal square root, two Newton steps
// r <- r (3 - d r^2) / 2 (each squares the relative error)
__device__ inline double rsqrt_nr(double d) {
  const double dd = fmax(d, 1e-300);
  double rs = __builtin_amdgcn_rsq(dd);
  rs = rs * (1.5 - 0.5 * dd * rs * rs);
  return rs * (1.5 - 0.5 * dd * rs * rs);
}
__device__ inline cd cmulc(cd a, cd b) { return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im}; }   // a conj(b)
// Row of L in the step's columns from the updated entries v[m] = P[row, c + m].
__device__ inline void step_row(const cd (&v)[CW], const cd (&l)[CW][CW], const double (&rs)[CW],
                                cd (&a)[CW]) {
#pragma unroll
  for (int m = 0; m < CW; ++m) {
    cd x = v[m];
#pragma unroll
    for (int k = 0; k < m; ++k) x = csub(x, cmulc(a[k], l[m][k]));
    a[m] = cscale(x, rs[m]);
  }
}
__device__ inline void diag_factor(const HpdDesc& h, int k0, cd (*P)[HPD_NB + 1], cd (*Li)[HPD_NB + 1],
                                   int* fail) {
  constexpr int NB = HPD_NB;
  static_assert(DIAG_THREADS == 8 * NB && NB % CW == 0, "thread (r, s0): r < NB, s0 < 8");
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += DIAG_THREADS) {
    const int r = e % NB, c = e / NB;
    P[c][r] = h.G[(int64_t)(k0 + c) * h.n_pad + k0 + r];
    Li[c][r] = {r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  const int r = t & (NB - 1), s0 = t / NB;
  for (int c = 0; c < NB; c += CW) {
    // pivot block: l[i][m] = L[c + i, c + m] (i > m), rs[m] = 1 / L[c + m, c + m]
    cd l[CW][CW];
    double rs[CW];
    bool ok = true;
#pragma unroll
    for (int m = 0; m < CW; ++m) {
      double d = P[c + m][c + m].re;
#pragma unroll
      for (int k = 0; k < m; ++k) d -= cabs2(l[m][k]);
      ok = ok && d > 0.0;
      rs[m] = rsqrt_nr(d);
#pragma unroll
      for (int i = m + 1; i < CW; ++i) {
        cd x = P[c + m][c + i];
#pragma unroll
        for (int k = 0; k < m; ++k) x = csub(x, cmulc(l[i][k], l[m][k]));
        l[i][m] = cscale(x, rs[m]);
      }
    }
    if (t == 0 && !ok) atomicOr(fail, 1);
    if (t >= NB && t - NB < c + CW) {   // rows c .. c + 3 of X, column j
      const int j = t - NB;
      cd x[CW];
#pragma unroll
      for (int m = 0; m < CW; ++m) {
        cd y = Li[j][c + m];
#pragma unroll
        for (int k = 0; k < m; ++k) y = csub(y, cmul(l[m][k], x[k]));
        x[m] = cscale(y, rs[m]);
      }
#pragma unroll
      for (int m = 0; m < CW; ++m) Li[j][c + m] = x[m];
    }
    __syncthreads();
    if (r >= c + CW) {
      cd v[CW], a[CW];
#pragma unroll
      for (int m = 0; m < CW; ++m) v[m] = P[c + m][r];
      cd u[4][CW], w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int sc = s0 + 8 * j;
        const bool f = sc >= c + CW;
#pragma unroll
        for (int m = 0; m < CW; ++m) u[j][m] = f ? P[c + m][sc] : Li[sc][c + m];   // P[s, c + m] or X[c + m, s]
        w[j] = f ? P[sc][r] : Li[sc][r];
      }
      step_row(v, l, rs, a);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int sc = s0 + 8 * j;
        cd acc = w[j];
        if (sc >= c + CW) {
          if (sc <= r) {   // P(r, s) -= sum_m L(r, c + m) conj(L(s, c + m))
            cd b[CW];
            step_row(u[j], l, rs, b);
#pragma unroll
            for (int m = 0; m < CW; ++m) acc = csub(acc, cmulc(a[m], b[m]));
            P[sc][r] = acc;
          }
        } else {           // Y(r, s) -= sum_m L(r, c + m) X(c + m, s)
#pragma unroll
          for (int m = 0; m < CW; ++m) acc = csub(acc, cmul(a[m], u[j][m]));
          Li[sc][r] = acc;
        }
      }
    }
    __syncthreads();
  }
}

// One column step of the Cholesky: every work-group b factors the diagonal
// block (the same arithmetic, so the same result) and forms panel rows
// [k0 + NB + 64 b, +64) of L21 = G21 Lkk^{-H} in place; work-group 0 also
// writes Lkk^{-1} to D[:, k0:k0+NB].  The diagonal
// block of G itself is only read (its factor lives in D; later steps use
// only the blocks below the diagonal), so no work-group writes what another
// may still be reading.
__global__ __launch_bounds__(DIAG_THREADS) void chol_panel_kernel(const HpdDesc* __restrict__ descs,
                                                                  int k0, int* fail) {
  const HpdDesc h = descs[blockIdx.y];
  constexpr int NB = HPD_NB;
  if (k0 >= h.n_pad) return;
  const int r0 = k0 + NB + PANEL_ROWS * (int)blockIdx.x;
  if (blockIdx.x > 0 && r0 >= h.n_pad) return;
  __shared__ cd P[NB][NB + 1];
  __shared__ cd Li[NB][NB + 1];
  __shared__ cd S[NB][PANEL_ROWS + 1];   // S[k][r] = G21(r0 + r, k)
  const int t = threadIdx.x, r = t & 63, cg = t >> 6;
  // panel rows: thread (r, cg) moves columns cg + 4 e (issued before the
  // factorisation, stored after it)
  cd g[NB / 4];
  const bool row_ok = r0 + r < h.n_pad;
#pragma unroll
  for (int e = 0; e < NB / 4; ++e)
    g[e] = row_ok ? h.G[(int64_t)(k0 + cg + 4 * e) * h.n_pad + r0 + r] : cd{0.0, 0.0};
  diag_factor(h, k0, P, Li, fail);
  if (blockIdx.x == 0) {
    for (int e = t; e < NB * NB; e += DIAG_THREADS) {
      const int rr = e % NB, c = e / NB;
      h.D[(int64_t)(k0 + c) * NB + rr] = Li[c][rr];
    }
    if (r0 >= h.n_pad) return;   // last diagonal block: no panel
  }
#pragma unroll
  for (int e = 0; e < NB / 4; ++e) S[cg + 4 * e][r] = g[e];
  __syncthreads();
  // L21(r, c) = sum_k G21(r, k) conj(X(c, k)), X = Lkk^{-1} lower triangular
  // (Li[k][c] = X(c, k), zero for k > c); thread (r, cg) forms columns cg + 4 j
  cd acc[NB / 4];
#pragma unroll
  for (int j = 0; j < NB / 4; ++j) acc[j] = {0.0, 0.0};
#pragma unroll 4
  for (int k = 0; k < NB; ++k) {
    const cd a = S[k][r];
#pragma unroll
    for (int j = 0; j < NB / 4; ++j) {
      const cd x = Li[k][cg + 4 * j];
      acc[j].re += a.re * x.re + a.im * x.im;
      acc[j].im += a.im * x.re - a.re * x.im;
    }
  }
  if (row_ok) {
#pragma unroll
    for (int j = 0; j < NB / 4; ++j) h.G[(int64_t)(k0 + cg + 4 * j) * h.n_pad + r0 + r] = acc[j];
  }
}

__global__ void zero_x_kernel(const HpdDesc* __restrict__ descs) {
  const HpdDesc h = descs[blockIdx.y];
  const int64_t n2 = (int64_t)h.n_pad * h.n_pad;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (int64_t)gridDim.x * 256)
    h.X[e] = {0.0, 0.0};
}

// Diagonal blocks of X = L^{-1} are the inverses of the diagonal Cholesky
// blocks (from chol_panel_kernel).  One work-group per block.
__global__ void x_diag_kernel(const HpdDesc* __restrict__ descs) {
  const HpdDesc h = descs[blockIdx.y];
  constexpr int NB = HPD_NB;
  const int i0 = blockIdx.x * NB;
  if (i0 >= h.n_pad) return;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int r = e % NB, c = e / NB;
    h.X[(int64_t)(i0 + c) * h.n_pad + i0 + r] = h.D[(int64_t)(i0 + c) * NB + r];
  }
}

// W = X^H X into G (lower tiles computed, mirrored to the upper part).
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

// ------------------------------------------------------------------ FP64 GEMM on MFMA
// C = alpha op(A) op(B) + beta C on the FP64 16x16x4 instruction, same tile
// structure as the Gram kernel (64 x 64 complex tile, four waves of 32 x 32).
// op(A) panels are staged as [re/im][k][i], op(B) panels as [re/im][k][j];
// the conjugate of an OP_C operand is taken while staging, so the products are
//   Re C += Ar Br - Ai Bi,   Im C += Ar Bi + Ai Br.
// KR restricts the k-range of a tile to where both operands can be nonzero:
//   KR_B_LOWER: op(B)[k][j] = 0 for k < j   (kb = j0)
//   KR_A_LOWER: op(A)[i][k] = 0 for k > i   (ke = i0 + 64)
//   KR_GE_MAX:  op(A)[i][k] = 0 for k < i and op(B)[k][j] = 0 for k < j
// OUT: MM_FULL writes every tile; MM_LOWER only entries i >= j (tiles of the
// lower triangle); MM_HERM also writes the conjugate mirror (C Hermitian).
enum : int { KR_ALL = 0, KR_B_LOWER = 1, KR_A_LOWER = 2, KR_GE_MAX = 4 };
enum : int { MM_FULL = 0, MM_LOWER = 1, MM_HERM = 2 };

__device__ inline void tri_of(int x, int* ti, int* tj) {
  // x -> (ti, tj), ti >= tj, x = ti (ti + 1) / 2 + tj
  int i = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= x) ++i;
  while (i * (i + 1) / 2 > x) --i;
  *ti = i;
  *tj = x - i * (i + 1) / 2;
}

// Element (r, c) of op(X) for the staged panel: `rows` indexes the 64-wide
// side (i of A, j of B), k the inner dimension.  ROWSMAJ: the 64-wide index is
// contiguous in memory (OP_N for A, OP_C for B); otherwise k is.
template <bool ROWSMAJ>
__device__ inline void mm_fetch(const cd* X, int ld, bool conj, int r0, int rows, int p0, int ke,
                                cd (&v)[HPF]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < HPF; ++e) {
    int r, k;
    if constexpr (ROWSMAJ) { r = r0 + (t & 63); k = p0 + (t >> 6) + 4 * e; }
    else { k = p0 + (t & 31); r = r0 + (t >> 5) + 8 * e; }
    cd x = {0.0, 0.0};
    if (r < rows && k < ke) {
      x = ROWSMAJ ? X[(int64_t)k * ld + r] : X[(int64_t)r * ld + k];
      if (conj) x.im = -x.im;
    }
    v[e] = x;
  }
}
constexpr int HLDZ = 65;   // odd row length: k-contiguous staging stores hit distinct banks
template <bool ROWSMAJ>
__device__ inline void mm_store(const cd (&v)[HPF], double (*dst)[HK][HLDZ]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < HPF; ++e) {
    int r, k;
    if constexpr (ROWSMAJ) { r = t & 63; k = (t >> 6) + 4 * e; }
    else { k = t & 31; r = (t >> 5) + 8 * e; }
    dst[0][k][r] = v[e].re;
    dst[1][k][r] = v[e].im;
  }
}

// Triangular k-ranges (KR_A_LOWER: the k-range grows with the row tile,
// KR_B_LOWER: it shrinks with the column tile) pair tile t with tile
// T - 1 - t in one work-group, so every work-group does about the same work.
template <int KR> constexpr bool paired_tiles() {
  return (KR & (KR_A_LOWER | KR_B_LOWER)) != 0 && (KR & KR_GE_MAX) == 0;
}

template <int OPA, int OPB, int KR, int OUT>
__device__ inline void zmm_tile(const MmDesc& d, int ti, int tj);

template <int OPA, int OPB, int KR, int OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void zmm_kernel(const MmDesc* __restrict__ descs, int rect) {
  // Work-groups are dealt to the 8 XCDs by linear id modulo 8; taking the
  // product index as the linear id modulo the number of products keeps each
  // product (one sensor's matrix in a batch of 8) on one XCD, so its panels
  // stay in that XCD's L2 instead of being fetched by all eight.
  const unsigned lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned rest = lin / gridDim.z;
  const int bz = (int)(lin % gridDim.z), bx = (int)(rest % gridDim.x), by = (int)(rest / gridDim.x);
  const MmDesc d = descs[bz];
  if constexpr (OUT == MM_FULL && paired_tiles<KR>()) {
    if constexpr ((KR & KR_A_LOWER) != 0) {
      const int mt = (d.m + HM - 1) / HM, t0 = bx, t1 = mt - 1 - bx;
      if (t0 < mt) zmm_tile<OPA, OPB, KR, OUT>(d, t0, by);
      if (t1 > t0) zmm_tile<OPA, OPB, KR, OUT>(d, t1, by);
    } else {
      const int nt = (d.n + HM - 1) / HM, t0 = by, t1 = nt - 1 - by;
      if (t0 < nt) zmm_tile<OPA, OPB, KR, OUT>(d, bx, t0);
      if (t1 > t0) zmm_tile<OPA, OPB, KR, OUT>(d, bx, t1);
    }
  } else {
    int ti, tj;
    if (OUT == MM_FULL || rect) {   // (lower output on a rectangular grid: tiles above skipped)
      ti = bx;
      tj = by;
      if (OUT != MM_FULL && tj > ti) return;
    } else {
      tri_of(bx, &ti, &tj);
    }
    zmm_tile<OPA, OPB, KR, OUT>(d, ti, tj);
  }
}

template <int OPA, int OPB, int KR, int OUT>
__device__ inline void zmm_tile(const MmDesc& d, int ti, int tj) {
  const int i0 = ti * HM, j0 = tj * HM;
  if (i0 >= d.m || j0 >= d.n) return;
  int kb = 0, ke = d.k;
  if constexpr ((KR & KR_B_LOWER) != 0) kb = max(kb, j0);
  if constexpr ((KR & KR_A_LOWER) != 0) ke = min(ke, i0 + HM);
  if constexpr ((KR & KR_GE_MAX) != 0) kb = max(kb, max(i0, j0));
  // A: op N -> element (i, k) at A[k lda + i] (i contiguous); op C -> conj(A[i lda + k]).
  // B: op N -> element (k, j) at B[j ldb + k] (k contiguous); op C -> conj(B[k ldb + j]).
  constexpr bool AROWS = OPA == OP_N, BROWS = OPB == OP_C;
  __shared__ double sA[2][HK][HLDZ];
  __shared__ double sB[2][HK][HLDZ];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  const int c16 = lane & 15, kq = lane >> 4;
  // three real products per complex multiply-add: t1 = sum ar br,
  // t2 = sum ai bi, t3 = sum (ar + ai)(br + bi); Re = t1 - t2, Im = t3 - t1 - t2
  v4d t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      t2[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      t3[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  cd va[HPF], vb[HPF];
  if (kb < ke) {
    mm_fetch<AROWS>(d.A, d.lda, OPA == OP_C, i0, d.m, kb, ke, va);
    mm_fetch<BROWS>(d.B, d.ldb, OPB == OP_C, j0, d.n, kb, ke, vb);
  }
  for (int p0 = kb; p0 < ke; p0 += HK) {
    __syncthreads();
    mm_store<AROWS>(va, sA);
    mm_store<BROWS>(vb, sB);
    __syncthreads();
    if (p0 + HK < ke) {
      mm_fetch<AROWS>(d.A, d.lda, OPA == OP_C, i0, d.m, p0 + HK, ke, va);
      mm_fetch<BROWS>(d.B, d.ldb, OPB == OP_C, j0, d.n, p0 + HK, ke, vb);
    }
#pragma unroll
    for (int kk = 0; kk < HK; kk += 4) {
      double ar[2], ai[2], sa[2], br[2], bi[2], sb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = sA[0][kk + kq][wr + 16 * a + c16];
        ai[a] = sA[1][kk + kq][wr + 16 * a + c16];
        sa[a] = ar[a] + ai[a];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        br[b] = sB[0][kk + kq][wc + 16 * b + c16];
        bi[b] = sB[1][kk + kq][wc + 16 * b + c16];
        sb[b] = br[b] + bi[b];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], t1[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], t2[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[a], sb[b], t3[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + 16 * a + 4 * r + kq;
        const int j = j0 + wc + 16 * b + c16;
        if (i >= d.m || j >= d.n) continue;
        if (OUT != MM_FULL && j > i) continue;
        const double p1 = t1[a][b][r], p2 = t2[a][b][r];
        const double xr = p1 - p2, xi = t3[a][b][r] - p1 - p2;
        cd v = {d.alpha_re * xr - d.alpha_im * xi, d.alpha_re * xi + d.alpha_im * xr};
        cd* cij = d.C + (int64_t)j * d.ldc + i;
        if (d.beta != 0.0) { v.re += d.beta * cij->re; v.im += d.beta * cij->im; }
        if (OUT == MM_HERM && i == j) v.im = 0.0;
        *cij = v;
        if (OUT == MM_HERM && i != j) d.C[(int64_t)i * d.ldc + j] = cd{v.re, -v.im};
      }
}

template <int OPA, int OPB, int KR, int OUT>
void launch_zmm(const MmDesc* d, int count, int max_m, int max_n, hipStream_t s) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return;
  int mt = (max_m + HM - 1) / HM, nt = (max_n + HM - 1) / HM;
  if constexpr (OUT == MM_FULL && paired_tiles<KR>()) {
    if constexpr ((KR & KR_A_LOWER) != 0) mt = (mt + 1) / 2;
    else nt = (nt + 1) / 2;
  }
  // lower output: the triangle of tiles, or for a tall product (few column
  // tiles) the rectangle of row x column tiles
  const bool tall = OUT == MM_LOWER && 2 * nt < mt;
  const dim3 grid = (OUT == MM_FULL || tall) ? dim3(mt, nt, count) : dim3(mt * (mt + 1) / 2, 1, count);
  zmm_kernel<OPA, OPB, KR, OUT><<<grid, 256, 0, s>>>(d, tall ? 1 : 0);
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

void zgemm_mfma_nn(const MmDesc* d_desc, int count, int max_m, int max_n, hipStream_t s) {
  launch_zmm<OP_N, OP_N, KR_ALL, MM_FULL>(d_desc, count, max_m, max_n, s);
}
void zgemm_mfma_cn(const MmDesc* d_desc, int count, int max_m, int max_n, hipStream_t s) {
  launch_zmm<OP_C, OP_N, KR_ALL, MM_FULL>(d_desc, count, max_m, max_n, s);
}
void zgemm_mfma_gram_cn(const MmDesc* d_desc, int count, int max_n, hipStream_t s) {
  launch_zmm<OP_C, OP_N, KR_ALL, MM_HERM>(d_desc, count, max_n, max_n, s);
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

// Cholesky steps of NB columns grouped in outer blocks of HPD_OB columns: the
// trailing update of a step covers only the rest of its outer block; the
// columns beyond it are updated once per outer block with k = HPD_OB (one pass
// over the trailing matrix per HPD_OB columns instead of per NB).
constexpr int HPD_OB = 128;

size_t hpd_mm_count(int n) {
  size_t c = 0;
  for (int K0 = 0; K0 < n; K0 += HPD_OB) {
    const int K1 = std::min(K0 + HPD_OB, n);
    for (int k0 = K0; k0 < K1; k0 += HPD_NB) {
      if (n - k0 - HPD_NB <= 0) continue;
      if (K1 - k0 - HPD_NB > 0) c += 1;                    // update inside the outer block
    }
    if (n - K1 > 0) c += 1;                                // update beyond it
  }
  for (int b = HPD_NB; b < n; b *= 2) c += 2 * (size_t)((n - b + 2 * b - 1) / (2 * b));
  return c + 1;                                            // X^H X
}

// U = X^H into G (complex conjugate transpose of the whole matrix, zeros
// included), 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void conj_transpose_x_kernel(const HpdDesc* __restrict__ descs) {
  const HpdDesc h = descs[blockIdx.z];
  const int n = h.n_pad;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;   // tile of X rows i, columns j
  if (i0 >= n || j0 >= n) return;
  __shared__ cd tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int c = ty; c < 64; c += 4) {
    const int i = i0 + tx, j = j0 + c;
    if (i < n && j < n) tile[c][tx] = h.X[(int64_t)j * n + i];   // X(i, j)
  }
  __syncthreads();
  for (int c = ty; c < 64; c += 4) {
    const int i = j0 + tx, j = i0 + c;   // U(i, j) = conj(X(j, i))
    if (i < n && j < n) {
      const cd v = tile[tx][c];
      h.G[(int64_t)j * n + i] = cd{v.re, -v.im};
    }
  }
}

void hpd_inverse_batched(const HpdDesc* hd, const HpdDesc* d_desc, int batch, int n, int* d_fail,
                         MmDesc* d_mm, hipStream_t s, bool form_w) {
  if (batch <= 0 || n <= 0) return;
  constexpr int NB = HPD_NB;
  // Plan every GEMM of the factorisation (descriptors grouped per launch,
  // all matrices of the batch together), upload once, then launch in order.
  enum Kind { TRAIL, TRI1, TRI2, XHX, DIAG };
  struct Launch { Kind kind; int off, count, m, n, k0; };
  std::vector<MmDesc> mm;
  std::vector<Launch> plan;
  mm.reserve((size_t)batch * hpd_mm_count(n));
  for (int K0 = 0; K0 < n; K0 += HPD_OB) {
    const int K1 = std::min(K0 + HPD_OB, n);
    for (int k0 = K0; k0 < K1; k0 += NB) {
      const int rest = n - k0 - NB;   // rows below the diagonal block (panel)
      plan.push_back({DIAG, 0, batch, std::max(rest, 0), 0, k0});
      if (rest <= 0) continue;
      const int nc = K1 - k0 - NB;   // columns of the outer block still to factor
      if (nc <= 0) continue;
      Launch lt{TRAIL, (int)mm.size(), batch, rest, nc, k0};
      for (int i = 0; i < batch; ++i) {
        const cd* L21 = hd[i].G + (int64_t)k0 * n + k0 + NB;
        mm.push_back(MmDesc{L21, L21, hd[i].G + (int64_t)(k0 + NB) * n + k0 + NB, rest, nc, NB,
                            n, n, n, -1.0, 0.0, 1.0});
      }
      plan.push_back(lt);
    }
    const int rest2 = n - K1;   // G22 -= L21 L21^H with the outer block's columns of L
    if (rest2 <= 0) continue;
    Launch lo{TRAIL, (int)mm.size(), batch, rest2, rest2, K0};
    for (int i = 0; i < batch; ++i) {
      const cd* L21 = hd[i].G + (int64_t)K0 * n + K1;
      mm.push_back(MmDesc{L21, L21, hd[i].G + (int64_t)K1 * n + K1, rest2, rest2, K1 - K0,
                          n, n, n, -1.0, 0.0, 1.0});
    }
    plan.push_back(lo);
  }
  for (int b = NB; b < n; b *= 2) {
    Launch l1{TRI1, (int)mm.size(), 0, b, b, 0};
    for (int i = 0; i < batch; ++i) {
      int64_t toff = 0;
      for (int o = 0; o + b < n; o += 2 * b) {
        const int rows = std::min(b, n - o - b);
        // T = L21 X11
        mm.push_back(MmDesc{hd[i].G + (int64_t)o * n + o + b, hd[i].X + (int64_t)o * n + o,
                            hd[i].T + toff, rows, b, b, n, n, rows, 1.0, 0.0, 0.0});
        toff += (int64_t)rows * b;
      }
    }
    l1.count = (int)mm.size() - l1.off;
    plan.push_back(l1);
    Launch l2{TRI2, (int)mm.size(), 0, b, b, 0};
    for (int i = 0; i < batch; ++i) {
      int64_t toff = 0;
      for (int o = 0; o + b < n; o += 2 * b) {
        const int rows = std::min(b, n - o - b);
        // X21 = -X22 T
        mm.push_back(MmDesc{hd[i].X + (int64_t)(o + b) * n + o + b, hd[i].T + toff,
                            hd[i].X + (int64_t)o * n + o + b, rows, b, rows, n, rows, n,
                            -1.0, 0.0, 0.0});
        toff += (int64_t)rows * b;
      }
    }
    l2.count = (int)mm.size() - l2.off;
    plan.push_back(l2);
  }
  Launch lx{XHX, (int)mm.size(), batch, n, n, 0};
  for (int i = 0; i < batch; ++i)
    mm.push_back(MmDesc{hd[i].X, hd[i].X, hd[i].G, n, n, n, n, n, n, 1.0, 0.0, 0.0});
  plan.push_back(lx);
  if (hipMemcpyAsync(d_mm, mm.data(), sizeof(MmDesc) * mm.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return;

  zero_x_kernel<<<dim3(std::min<int64_t>(((int64_t)n * n + 255) / 256, 4096), batch), 256, 0, s>>>(d_desc);
  bool diag_done = false;
  for (const Launch& l : plan) {
    const MmDesc* p = d_mm + l.off;
    switch (l.kind) {
      case DIAG:
        chol_panel_kernel<<<dim3(std::max(1, (l.m + PANEL_ROWS - 1) / PANEL_ROWS), batch), DIAG_THREADS, 0, s>>>(
            d_desc, l.k0, d_fail);
        break;
      case TRAIL: launch_zmm<OP_N, OP_C, KR_ALL, MM_LOWER>(p, l.count, l.m, l.n, s); break;
      case TRI1:
        if (!diag_done) {   // X's diagonal blocks, once the Cholesky is complete
          x_diag_kernel<<<dim3(n / NB, batch), 256, 0, s>>>(d_desc);
          diag_done = true;
        }
        launch_zmm<OP_N, OP_N, KR_B_LOWER, MM_FULL>(p, l.count, l.m, l.n, s);
        break;
      case TRI2: launch_zmm<OP_N, OP_N, KR_A_LOWER, MM_FULL>(p, l.count, l.m, l.n, s); break;
      case XHX:
        if (!diag_done) {
          x_diag_kernel<<<dim3(n / NB, batch), 256, 0, s>>>(d_desc);
          diag_done = true;
        }
        if (form_w) {
          launch_zmm<OP_C, OP_N, KR_GE_MAX, MM_HERM>(p, l.count, l.m, l.n, s);
        } else {
          const dim3 g((n + 63) / 64, (n + 63) / 64, batch);
          conj_transpose_x_kernel<<<g, 256, 0, s>>>(d_desc);
        }
        break;
    }
  }
}

void hpd_form_w(const MmDesc* d_desc, int count, int n, hipStream_t s) {
  launch_zmm<OP_C, OP_N, KR_GE_MAX, MM_HERM>(d_desc, count, n, n, s);
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

