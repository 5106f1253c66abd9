// FP64 complex GEMM (batched, tiled through LDS) and blocked Gauss-Jordan
// inverse of Hermitian positive definite matrices.
//
// These build W_q = ((c/mu) I + Ahat_q Ahat_q^H)^{-1}, the factor through which
// the ridge x-update of eq. (3) is applied in Woodbury form, and apply the
// low-rank corrections of W_q when SSC (Alg. 1) removes columns of Ahat_q or
// the optimality re-check puts them back.  MI355X runs FP64 FMA on the vector
// units at the same peak as FP64 matrix instructions, so these are plain
// register-blocked FMA kernels.
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

// ------------------------------------------------------------------ Gauss-Jordan
// Pivot block inverse: P = G[k0:k0+NB, k0:k0+NB] -> D = P^{-1}, in LDS.
__global__ __launch_bounds__(256) void gj_diag_kernel(const HpdDesc* __restrict__ descs, int k0,
                                                      int* fail) {
  const HpdDesc h = descs[blockIdx.x];
  if (k0 >= h.n_pad) return;
  constexpr int NB = HPD_NB;
  __shared__ cd P[NB][NB + 1];   // P[col][row]
  __shared__ cd prow[NB], pcol[NB];
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e % NB, c = e / NB;
    P[c][r] = h.G[(int64_t)(k0 + c) * h.n_pad + k0 + r];
  }
  __syncthreads();
  for (int piv = 0; piv < NB; ++piv) {
    const double p = P[piv][piv].re;
    if (t == 0 && !(p > 0.0)) atomicOr(fail, 1);
    const double ip = 1.0 / p;
    if (t < NB) { prow[t] = P[t][piv]; pcol[t] = P[piv][t]; }
    __syncthreads();
    for (int e = t; e < NB * NB; e += 256) {
      const int r = e % NB, c = e / NB;
      cd v = P[c][r];
      if (r == piv && c == piv) {
        v = {ip, 0.0};
      } else if (r == piv) {
        v = cscale(v, ip);                       // pivot row: P^{-1} G_kj
      } else if (c == piv) {
        v = cscale(v, -ip);                      // pivot column: -G_ik P^{-1}
      } else {
        cd prod = cmul(pcol[r], prow[c]);        // G_ik * G_kj / p
        v = csub(v, cscale(prod, ip));
      }
      P[c][r] = v;
    }
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e % NB, c = e / NB;
    h.D[c * NB + r] = P[c][r];
  }
}

// R = D * G[k0:k0+NB, :] with R[:, k0:k0+NB] = D; Cp = G[:, k0:k0+NB].
__global__ __launch_bounds__(256) void gj_panel_kernel(const HpdDesc* __restrict__ descs, int k0) {
  const HpdDesc h = descs[blockIdx.y];
  constexpr int NB = HPD_NB;
  if (k0 >= h.n_pad) return;
  __shared__ cd Ds[NB][NB + 1];
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 256) Ds[e / NB][e % NB] = h.D[e];
  __syncthreads();
  const int j = blockIdx.x * 256 + t;
  if (j >= h.n_pad) return;
  if (j >= k0 && j < k0 + NB) {
    for (int r = 0; r < NB; ++r) h.R[(int64_t)j * NB + r] = Ds[j - k0][r];
  } else {
    cd g[NB];
    for (int c = 0; c < NB; ++c) g[c] = h.G[(int64_t)j * h.n_pad + k0 + c];
    for (int r = 0; r < NB; ++r) {
      cd acc = {0.0, 0.0};
      for (int c = 0; c < NB; ++c) cfma(acc, Ds[c][r], g[c]);
      h.R[(int64_t)j * NB + r] = acc;
    }
  }
  // column panel copy (row j of G[:, k0:k0+NB])
  for (int c = 0; c < NB; ++c) h.Cp[(int64_t)c * h.n_pad + j] = h.G[(int64_t)(k0 + c) * h.n_pad + j];
}

// G[i,j] <- rows in block: R[i-k0, j];  others: (j in block ? 0 : G[i,j]) - Cp[i,:] R[:,j]
__global__ __launch_bounds__(256) void gj_update_kernel(const HpdDesc* __restrict__ descs, int k0) {
  const HpdDesc h = descs[blockIdx.z];
  constexpr int NB = HPD_NB;
  const int i0 = blockIdx.x * TM, j0 = blockIdx.y * TN;
  if (k0 >= h.n_pad || i0 >= h.n_pad || j0 >= h.n_pad) return;
  __shared__ cd sC[NB][TM + 1];
  __shared__ cd sR[NB][TN + 1];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  for (int e = t; e < NB * TM; e += 256) {
    const int ii = e % TM, c = e / TM;
    const int gi = i0 + ii;
    sC[c][ii] = gi < h.n_pad ? h.Cp[(int64_t)c * h.n_pad + gi] : cd{0.0, 0.0};
  }
  for (int e = t; e < NB * TN; e += 256) {
    const int r = e % NB, jj = e / NB;
    const int gj = j0 + jj;
    sR[r][jj] = gj < h.n_pad ? h.R[(int64_t)gj * NB + r] : cd{0.0, 0.0};
  }
  __syncthreads();
  cd acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = {0.0, 0.0};
#pragma unroll 4
  for (int c = 0; c < NB; ++c) {
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
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + tx + 16 * a;
    if (i >= h.n_pad) continue;
    const bool irow = (i >= k0 && i < k0 + NB);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + ty + 16 * b;
      if (j >= h.n_pad) continue;
      cd* g = h.G + (int64_t)j * h.n_pad + i;
      if (irow) {
        *g = sR[i - k0][j - j0];
      } else {
        const bool jcol = (j >= k0 && j < k0 + NB);
        cd base = jcol ? cd{0.0, 0.0} : *g;
        *g = csub(base, acc[a][b]);
      }
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

template <int STA, int STB, int OPA, int OPB, bool HERM>
void launch_gemm(const GemmDesc* d, int batch, int mm, int mn, hipStream_t s) {
  dim3 grid((mm + TM - 1) / TM, (mn + TN - 1) / TN, batch);
  zgemm_kernel<STA, STB, OPA, OPB, HERM><<<grid, 256, 0, s>>>(d);
}

}  // namespace

void zgemm_batched(const GemmDesc* d_desc, int batch, int max_m, int max_n, int sta, int stb,
                   int opa, int opb, bool herm, hipStream_t s) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  // Instantiated combinations: Gram of the operator in its storage (N, C, herm),
  // and FP64 x FP64 products for the low-rank factor corrections.
  if (stb == sta && opa == OP_N && opb == OP_C && herm) {
    switch (sta) {
      case ST_FP64: launch_gemm<ST_FP64, ST_FP64, OP_N, OP_C, true>(d_desc, batch, max_m, max_n, s); return;
      case ST_FP32: launch_gemm<ST_FP32, ST_FP32, OP_N, OP_C, true>(d_desc, batch, max_m, max_n, s); return;
      case ST_FP16P: launch_gemm<ST_FP16P, ST_FP16P, OP_N, OP_C, true>(d_desc, batch, max_m, max_n, s); return;
      case ST_BF16P: launch_gemm<ST_BF16P, ST_BF16P, OP_N, OP_C, true>(d_desc, batch, max_m, max_n, s); return;
    }
  }
  if (sta == ST_FP64 && stb == ST_FP64 && !herm) {
    if (opa == OP_N && opb == OP_N) { launch_gemm<ST_FP64, ST_FP64, OP_N, OP_N, false>(d_desc, batch, max_m, max_n, s); return; }
    if (opa == OP_C && opb == OP_N) { launch_gemm<ST_FP64, ST_FP64, OP_C, OP_N, false>(d_desc, batch, max_m, max_n, s); return; }
    if (opa == OP_N && opb == OP_C) { launch_gemm<ST_FP64, ST_FP64, OP_N, OP_C, false>(d_desc, batch, max_m, max_n, s); return; }
  }
  if (sta == ST_FP64 && stb == ST_FP64 && herm && opa == OP_C && opb == OP_N) {
    launch_gemm<ST_FP64, ST_FP64, OP_C, OP_N, true>(d_desc, batch, max_m, max_n, s); return;
  }
}

void hpd_inverse_batched(const HpdDesc* d_desc, int batch, int max_npad, int* d_fail,
                         hipStream_t s) {
  if (batch <= 0 || max_npad <= 0) return;
  const int tiles = (max_npad + TM - 1) / TM;
  for (int k0 = 0; k0 < max_npad; k0 += HPD_NB) {
    gj_diag_kernel<<<batch, 256, 0, s>>>(d_desc, k0, d_fail);
    gj_panel_kernel<<<dim3((max_npad + 255) / 256, batch), 256, 0, s>>>(d_desc, k0);
    gj_update_kernel<<<dim3(tiles, tiles, batch), 256, 0, s>>>(d_desc, k0);
  }
}

void cast_hermitian(const cd* src, int64_t ld_src, void* dst, int64_t ld_dst, int n, bool to_float,
                    hipStream_t s) {
  if (n <= 0) return;
  cast_herm_kernel<<<dim3((n + 255) / 256, n), 256, 0, s>>>(src, ld_src, dst, ld_dst, n, to_float ? 1 : 0);
}

void set_identity_pad(cd* G, int n, int n_pad, double diag_add, hipStream_t s) {
  if (n_pad <= 0) return;
  identity_pad_kernel<<<dim3((n_pad + 255) / 256, n_pad), 256, 0, s>>>(G, n, n_pad, diag_add);
}
