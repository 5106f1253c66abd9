// Pixel-pruning CNN: forward, backward and Adam on the GPU (FP32).
//
// Network (Q input channels = matched-filter images |A_q^H y_q| scaled by
// their maximum, C hidden channels):
//   a1 = conv(x, W1)+b1, h1 = relu(a1); a2 = conv(h1, W2)+b2, h2 = relu(a2);
//   a3 = conv(h2, W3)+b3, h3 = relu(a3); a4 = conv(h3, W4)+b4, p = sigmoid(a4)
// conv = 3x3 cross-correlation, zero 'same' padding, NCHW (channel planes of
// H x W, pixel n = i*W + j -- the solver's pixel order).  Loss: weighted BCE
// averaged over pixels.  A pixel with p >= threshold is eliminated from every
// sensor's sub-problem before the factor build (eq. (3), initial P_q); the
// optimality re-check after convergence reinstates false eliminations.
//
// Training runs the FP32 direct convolutions: 16x16 output tiles per
// work-group, the input tile plus halo of one channel at a time in LDS, all
// output channels of a pixel accumulated in registers, weights in LDS.
// Inference (forward, and the solver's selector) runs by default on the FP16
// matrix instructions with FP32 accumulation: each layer is a product
// (pixels x 9 cin) . (9 cin x cout) whose left operand is gathered from an
// LDS tile of the input (channel-last, so the four k-slots of a lane are four
// consecutive channels of one tap).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sadmm.h"
#include "common.h"

namespace {

constexpr int TILE = 16;
constexpr int CMAX = 32;    // max channels per layer

struct CnnLayer {
  int cin, cout;
  int64_t w_off, b_off;     // offsets into the flat parameter vector
};

// out[co][p] = b[co] + sum_ci sum_k W[co][ci][k] in[ci][p + off_k]; relu optional
__global__ __launch_bounds__(256) void conv_fwd_kernel(const float* __restrict__ in, int cin,
                                                       const float* __restrict__ Wt,
                                                       const float* __restrict__ b, int cout,
                                                       int H, int W, int relu,
                                                       float* __restrict__ out) {
  __shared__ float sx[TILE + 2][TILE + 2];
  __shared__ float sw[CMAX * CMAX * 9];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int j = blockIdx.x * TILE + tx, i = blockIdx.y * TILE + ty;
  for (int e = threadIdx.x; e < cout * cin * 9; e += 256) sw[e] = Wt[e];
  float acc[CMAX];
#pragma unroll
  for (int o = 0; o < CMAX; ++o) acc[o] = 0.f;
  for (int c = 0; c < cin; ++c) {
    __syncthreads();
    for (int e = threadIdx.x; e < (TILE + 2) * (TILE + 2); e += 256) {
      const int ly = e / (TILE + 2), lx = e % (TILE + 2);
      const int gi = blockIdx.y * TILE + ly - 1, gj = blockIdx.x * TILE + lx - 1;
      sx[ly][lx] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? in[(int64_t)c * H * W + (int64_t)gi * W + gj] : 0.f;
    }
    __syncthreads();
    float v[9];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) v[dy * 3 + dx] = sx[ty + dy][tx + dx];
#pragma unroll
    for (int o = 0; o < CMAX; ++o) {
      if (o < cout) {
        const float* w = sw + ((int64_t)o * cin + c) * 9;
        float s = acc[o];
#pragma unroll
        for (int k = 0; k < 9; ++k) s = fmaf(w[k], v[k], s);
        acc[o] = s;
      }
    }
  }
  if (i >= H || j >= W) return;
#pragma unroll
  for (int o = 0; o < CMAX; ++o) {
    if (o < cout) {
      float a = acc[o] + b[o];
      if (relu) a = fmaxf(a, 0.f);
      out[(int64_t)o * H * W + (int64_t)i * W + j] = a;
    }
  }
}

// The same layer on the 16x16x16 FP16 matrix instruction (FP32 accumulation).
// Work-group: 16 x 16 output pixels; wave w owns rows 4w..4w+3, one 16-pixel
// row per 16-row block of the product; output channels in blocks of 16.
// k = tap * cinP + ci (cinP = cin rounded up to 4, tap = 3 dy + dx), padded
// with zero weights to a multiple of 16.  Lane l supplies A[m = l % 16][k0 +
// 4 (l / 16) + i] and B[k0 + 4 (l / 16) + i][n = l % 16], i < 4, and receives
// C[4 (l / 16) + r][l % 16], r < 4.
typedef _Float16 half4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
constexpr int KMAX = 9 * CMAX;   // 288, a multiple of 16

__global__ __launch_bounds__(256) void conv_fwd_mfma_kernel(const float* __restrict__ in, int cin,
                                                            const float* __restrict__ Wt,
                                                            const float* __restrict__ b, int cout,
                                                            int H, int W, int relu,
                                                            float* __restrict__ out) {
  __shared__ __align__(16) _Float16 sx[(TILE + 2) * (TILE + 2) * CMAX];   // [y][x][ci]
  __shared__ __align__(16) _Float16 sw[CMAX * KMAX];                      // [co][k]
  const int cinP = (cin + 3) & ~3;
  const int Ktot = 9 * cinP, Kpad = (Ktot + 15) & ~15;
  const int nblk = (cout + 15) >> 4;
  for (int e = threadIdx.x; e < 16 * nblk * Kpad; e += 256) {
    const int co = e / Kpad, k = e - co * Kpad;
    float v = 0.f;
    if (co < cout && k < Ktot) {
      const int tap = k / cinP, ci = k - tap * cinP;
      if (ci < cin) v = Wt[((int64_t)co * cin + ci) * 9 + tap];
    }
    sw[co * Kpad + k] = (_Float16)v;
  }
  const int y0 = blockIdx.y * TILE - 1, x0 = blockIdx.x * TILE - 1;
  constexpr int NP = (TILE + 2) * (TILE + 2);
  for (int e = threadIdx.x; e < NP * cinP; e += 256) {
    const int ci = e / NP, pix = e - ci * NP;   // consecutive threads: consecutive pixels
    const int gi = y0 + pix / (TILE + 2), gj = x0 + pix % (TILE + 2);
    float v = 0.f;
    if (ci < cin && gi >= 0 && gi < H && gj >= 0 && gj < W) v = in[(int64_t)ci * H * W + (int64_t)gi * W + gj];
    sx[pix * cinP + ci] = (_Float16)v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  float4v acc[4][2];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = float4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < Kpad; k0 += 16) {
    const int k = k0 + 4 * g;
    half4v bv[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
      bv[nb] = nb < nblk ? *reinterpret_cast<const half4v*>(&sw[(nb * 16 + c16) * Kpad + k])
                         : half4v{0, 0, 0, 0};
    const bool kin = k < Ktot;
    const int tap = kin ? k / cinP : 0, ci = kin ? k - tap * cinP : 0;
    const int dy = tap / 3, dx = tap - 3 * dy;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const int pix = (4 * w + mb + dy) * (TILE + 2) + c16 + dx;
      const half4v av = kin ? *reinterpret_cast<const half4v*>(&sx[pix * cinP + ci]) : half4v{0, 0, 0, 0};
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        if (nb < nblk) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv[nb], acc[mb][nb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int i = blockIdx.y * TILE + 4 * w + mb;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int co = nb * 16 + c16;
      if (nb >= nblk || co >= cout || i >= H) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = blockIdx.x * TILE + 4 * g + r;
        if (j >= W) continue;
        float a = acc[mb][nb][r] + b[co];
        if (relu) a = fmaxf(a, 0.f);
        out[(int64_t)co * H * W + (int64_t)i * W + j] = a;
      }
    }
  }
}

// dx[ci][p] = mask[ci][p] * sum_co sum_k W[co][ci][k] g[co][p - off_k]
// (mask = previous layer's relu derivative: h > 0; null = no mask)
__global__ __launch_bounds__(256) void conv_bwd_data_kernel(const float* __restrict__ g, int cout,
                                                            const float* __restrict__ Wt, int cin,
                                                            int H, int W,
                                                            const float* __restrict__ mask,
                                                            float* __restrict__ dx) {
  __shared__ float sg[TILE + 2][TILE + 2];
  __shared__ float sw[CMAX * CMAX * 9];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int j = blockIdx.x * TILE + tx, i = blockIdx.y * TILE + ty;
  for (int e = threadIdx.x; e < cout * cin * 9; e += 256) sw[e] = Wt[e];
  float acc[CMAX];
#pragma unroll
  for (int c = 0; c < CMAX; ++c) acc[c] = 0.f;
  for (int o = 0; o < cout; ++o) {
    __syncthreads();
    for (int e = threadIdx.x; e < (TILE + 2) * (TILE + 2); e += 256) {
      const int ly = e / (TILE + 2), lx = e % (TILE + 2);
      const int gi = blockIdx.y * TILE + ly - 1, gj = blockIdx.x * TILE + lx - 1;
      sg[ly][lx] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? g[(int64_t)o * H * W + (int64_t)gi * W + gj] : 0.f;
    }
    __syncthreads();
    // g[o][i - dy][j - dx] for tap (dy, dx) -> LDS (ty + 1 - dy, tx + 1 - dx)
    float v[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) v[(dy + 1) * 3 + dx + 1] = sg[ty + 1 - dy][tx + 1 - dx];
#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
      if (c < cin) {
        const float* w = sw + ((int64_t)o * cin + c) * 9;
        float s = acc[c];
#pragma unroll
        for (int k = 0; k < 9; ++k) s = fmaf(w[k], v[k], s);
        acc[c] = s;
      }
    }
  }
  if (i >= H || j >= W) return;
#pragma unroll
  for (int c = 0; c < CMAX; ++c) {
    if (c < cin) {
      const int64_t o = (int64_t)c * H * W + (int64_t)i * W + j;
      float d = acc[c];
      if (mask) d = mask[o] > 0.f ? d : 0.f;
      dx[o] = d;
    }
  }
}

// Per-tile partial weight/bias gradients for one input channel ci:
// part[tile][co][ci][k] = sum_{p in tile} g[co][p] x[ci][p + off_k], k = 0..8;
// k = 9 slot (ci = 0 only) holds sum_p g[co][p].
__global__ __launch_bounds__(256) void conv_bwd_w_kernel(const float* __restrict__ g, int cout,
                                                         const float* __restrict__ x, int cin,
                                                         int H, int W, float* __restrict__ part) {
  __shared__ float sx[TILE + 2][TILE + 2];
  __shared__ float sg[CMAX][TILE * TILE];
  const int ci = blockIdx.z;
  const int tile = blockIdx.y * gridDim.x + blockIdx.x;
  const int t = threadIdx.x;
  for (int e = t; e < (TILE + 2) * (TILE + 2); e += 256) {
    const int ly = e / (TILE + 2), lx = e % (TILE + 2);
    const int gi = blockIdx.y * TILE + ly - 1, gj = blockIdx.x * TILE + lx - 1;
    sx[ly][lx] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? x[(int64_t)ci * H * W + (int64_t)gi * W + gj] : 0.f;
  }
  for (int e = t; e < cout * TILE * TILE; e += 256) {
    const int o = e / (TILE * TILE), pp = e % (TILE * TILE);
    const int gi = blockIdx.y * TILE + pp / TILE, gj = blockIdx.x * TILE + pp % TILE;
    sg[o][pp] = (gi < H && gj < W) ? g[(int64_t)o * H * W + (int64_t)gi * W + gj] : 0.f;
  }
  __syncthreads();
  const int nk = (ci == 0) ? 10 : 9;
  float* out = part + (int64_t)tile * cout * cin * 10;
  for (int e = t; e < cout * nk; e += 256) {
    const int o = e / nk, k = e % nk;
    float s = 0.f;
    if (k < 9) {
      const int dy = k / 3, dx = k % 3;
      for (int pp = 0; pp < TILE * TILE; ++pp) s = fmaf(sg[o][pp], sx[pp / TILE + dy][pp % TILE + dx], s);
    } else {
      for (int pp = 0; pp < TILE * TILE; ++pp) s += sg[o][pp];
    }
    out[((int64_t)o * cin + ci) * 10 + k] = s;
  }
}

// Sum the tile partials (fixed order) into the flat gradient vector.
__global__ void conv_bwd_w_reduce(const float* __restrict__ part, int ntiles, int cout, int cin,
                                  float* __restrict__ gW, float* __restrict__ gb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int per = cout * cin * 10;
  if (e >= per) return;
  const int k = e % 10, ci = (e / 10) % cin, o = e / (10 * cin);
  if (k == 9 && ci != 0) return;
  double s = 0.0;
  for (int tl = 0; tl < ntiles; ++tl) s += part[(int64_t)tl * per + e];
  if (k < 9) gW[((int64_t)o * cin + ci) * 9 + k] = (float)s;
  else gb[o] = (float)s;
}

// p = sigmoid(a4); g = w (p - t) / P; block partials of the loss
__global__ __launch_bounds__(256) void bce_kernel(const float* __restrict__ a4, const float* __restrict__ tgt,
                                                  int P, float pos_weight, float* __restrict__ prob,
                                                  float* __restrict__ g, double* __restrict__ lpart) {
  __shared__ double sm[4 * 1];
  const int n = blockIdx.x * 256 + threadIdx.x;
  double l[1] = {0.0};
  if (n < P) {
    const float a = a4[n];
    const float p = 1.f / (1.f + expf(-a));
    if (prob) prob[n] = p;
    if (tgt) {
      const float t = tgt[n];
      const float w = t > 0.5f ? pos_weight : 1.f;
      g[n] = w * (p - t) / (float)P;
      // log-sigmoid forms stable for large |a|
      const double lp = -log1p(exp(-(double)a));       // log p
      const double lq = -(double)a + lp;                 // log (1 - p)
      l[0] = -(double)w * ((double)t * lp + (1.0 - (double)t) * lq);
    }
  }
  block_sum256<double, 1>(l, sm);
  if (threadIdx.x == 0 && lpart) lpart[blockIdx.x] = l[0];
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void scale_input_kernel(const double* __restrict__ mf, int64_t n, const double* __restrict__ mx,
                                   float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double m = *mx;
  out[i] = (float)(m > 0 ? mf[i] / m : mf[i]);
}

__global__ __launch_bounds__(1024) void max_kernel(const double* __restrict__ x, int64_t n, double* out) {
  __shared__ double sm[16];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, x[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < 16; ++w) r = fmax(r, sm[w]);
    *out = r;
  }
}

}  // namespace

struct sadmm_cnn_s {
  int Q = 0, C = 0, H = 0, W = 0;
  hipStream_t s = nullptr;
  std::string err;
  CnnLayer L[4];
  int64_t nparam = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  float *x = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *a4 = nullptr, *prob = nullptr;
  float *tgt = nullptr, *g4 = nullptr, *gA = nullptr, *gB = nullptr, *part = nullptr;
  double *lpart = nullptr, *mx = nullptr;
  int step = 0;
  int half = 1;               // inference on the FP16 matrix instructions
  std::vector<void*> allocs;
};

namespace {

int cfail(sadmm_cnn_t c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

int calloc_dev(sadmm_cnn_t c, void** p, size_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) return SADMM_E_NOMEM;
  c->allocs.push_back(*p);
  return SADMM_OK;
}

dim3 tiles(int H, int W) { return dim3((W + TILE - 1) / TILE, (H + TILE - 1) / TILE); }

// The four layers of an H x W input x; layer l writes out[l] (out[3] = a4).
void cnn_layers(sadmm_cnn_t c, const float* x, int H, int W, float* const out[4], bool half) {
  const dim3 gr = tiles(H, W);
  for (int l = 0; l < 4; ++l) {
    const float* in = l == 0 ? x : out[l - 1];
    if (half)
      conv_fwd_mfma_kernel<<<gr, 256, 0, c->s>>>(in, c->L[l].cin, c->p + c->L[l].w_off,
                                                 c->p + c->L[l].b_off, c->L[l].cout, H, W,
                                                 l < 3 ? 1 : 0, out[l]);
    else
      conv_fwd_kernel<<<gr, 256, 0, c->s>>>(in, c->L[l].cin, c->p + c->L[l].w_off, c->p + c->L[l].b_off,
                                            c->L[l].cout, H, W, l < 3 ? 1 : 0, out[l]);
  }
}

void cnn_forward_dev(sadmm_cnn_t c, bool half) {
  float* const out[4] = {c->h1, c->h2, c->h3, c->a4};
  cnn_layers(c, c->x, c->H, c->W, out, half);
}

// Scratch of the allocation-free forward (sadmm_cnn_forward_noalloc): two
// ping-pong activation buffers of CMAX channel planes and the pre-sigmoid
// map, for images of at most NOALLOC_MAX_PIXELS pixels (512 x 512: 65 MiB).
// Every entry a call reads was written by the same call, so nothing needs
// clearing between calls.  Host code never passes this symbol to a kernel:
// it passes the device address hipGetSymbolAddress returns for the current
// device (noalloc_scratch).
constexpr int64_t NOALLOC_MAX_PIXELS = 512 * 512;
constexpr int64_t NOALLOC_FLOATS = (2 * CMAX + 1) * NOALLOC_MAX_PIXELS;
__device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of the scratch array on the current device, looked up once
// per device.
int noalloc_scratch(sadmm_cnn_t c, float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return cfail(c, SADMM_E_HIP, "forward_noalloc: no current device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return cfail(c, SADMM_E_HIP, "forward_noalloc: scratch symbol lookup failed");
    g_scratch_dev[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_dev[dev];
  return SADMM_OK;
}

// forward + loss + backward into c->g; returns the loss through *loss (host)
int cnn_backward_dev(sadmm_cnn_t c, float pos_weight, double* loss) {
  const int P = c->H * c->W;
  const int nb = (P + 255) / 256;
  cnn_forward_dev(c, false);   // gradients of the FP32 forward
  bce_kernel<<<nb, 256, 0, c->s>>>(c->a4, c->tgt, P, pos_weight, c->prob, c->g4, c->lpart);
  const dim3 gr = tiles(c->H, c->W);
  const int ntiles = gr.x * gr.y;
  const float* hin[4] = {c->x, c->h1, c->h2, c->h3};
  const float* grad = c->g4;
  float* bufs[2] = {c->gA, c->gB};
  for (int l = 3; l >= 0; --l) {
    const CnnLayer& ly = c->L[l];
    conv_bwd_w_kernel<<<dim3(gr.x, gr.y, ly.cin), 256, 0, c->s>>>(grad, ly.cout, hin[l], ly.cin, c->H, c->W, c->part);
    const int per = ly.cout * ly.cin * 10;
    conv_bwd_w_reduce<<<(per + 255) / 256, 256, 0, c->s>>>(c->part, ntiles, ly.cout, ly.cin, c->g + ly.w_off,
                                                          c->g + ly.b_off);
    if (l > 0) {
      float* dx = bufs[l & 1];
      conv_bwd_data_kernel<<<gr, 256, 0, c->s>>>(grad, ly.cout, c->p + ly.w_off, ly.cin, c->H, c->W, hin[l], dx);
      grad = dx;
    }
  }
  if (hipGetLastError() != hipSuccess) return cfail(c, SADMM_E_HIP, "cnn backward launch failed");
  std::vector<double> lp(nb);
  if (hipMemcpyAsync(lp.data(), c->lpart, sizeof(double) * nb, hipMemcpyDeviceToHost, c->s) != hipSuccess ||
      hipStreamSynchronize(c->s) != hipSuccess)
    return cfail(c, SADMM_E_HIP, "cnn loss copy failed");
  double s = 0.0;
  for (double v : lp) s += v;
  if (loss) *loss = s / P;
  return SADMM_OK;
}

int put_input(sadmm_cnn_t c, float* dst, const float* src, int64_t n, int on_device) {
  hipError_t e = hipMemcpyAsync(dst, src, sizeof(float) * n,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->s);
  return e == hipSuccess ? SADMM_OK : cfail(c, SADMM_E_HIP, "cnn input copy failed");
}

}  // namespace

// Used by the solver: matched-filter images (Q x N doubles, device) -> scaled
// FP32 input -> probability map (N floats, device, owned by the CNN handle).
int sadmm_cnn_prob_from_mf(sadmm_cnn_t c, const double* mf_dev, const float** prob_dev) {
  const int64_t n = (int64_t)c->Q * c->H * c->W;
  max_kernel<<<1, 1024, 0, c->s>>>(mf_dev, n, c->mx);
  scale_input_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->s>>>(mf_dev, n, c->mx, c->x);
  cnn_forward_dev(c, c->half != 0);
  const int P = c->H * c->W;
  bce_kernel<<<(P + 255) / 256, 256, 0, c->s>>>(c->a4, nullptr, P, 1.f, c->prob, nullptr, nullptr);
  if (hipGetLastError() != hipSuccess) return cfail(c, SADMM_E_HIP, "cnn inference launch failed");
  *prob_dev = c->prob;
  return SADMM_OK;
}

hipStream_t sadmm_cnn_stream(sadmm_cnn_t c) { return c->s; }
int sadmm_cnn_shape(sadmm_cnn_t c, int* Q, int* H, int* W) {
  *Q = c->Q; *H = c->H; *W = c->W;
  return SADMM_OK;
}

extern "C" {

int sadmm_cnn_create(int32_t Q, int32_t C, int32_t H, int32_t W, void* stream, sadmm_cnn_t* out) {
  if (!out || Q < 1 || Q > CMAX || C < 1 || C > CMAX || H < 1 || W < 1) return SADMM_E_ARG;
  sadmm_cnn_t c = new sadmm_cnn_s();
  c->Q = Q; c->C = C; c->H = H; c->W = W;
  c->s = static_cast<hipStream_t>(stream);
  const int cin[4] = {Q, C, C, C}, cout[4] = {C, C, C, 1};
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    c->L[l].cin = cin[l];
    c->L[l].cout = cout[l];
    c->L[l].w_off = off;
    off += (int64_t)cout[l] * cin[l] * 9;
    c->L[l].b_off = off;
    off += cout[l];
  }
  c->nparam = off;
  const int64_t P = (int64_t)H * W;
  const dim3 gr = tiles(H, W);
  const int64_t ntiles = (int64_t)gr.x * gr.y;
  int rc = SADMM_OK;
  auto A = [&](void** p, size_t b) { if (rc == SADMM_OK) rc = calloc_dev(c, p, b); };
  A((void**)&c->p, 4 * off); A((void**)&c->g, 4 * off); A((void**)&c->m, 4 * off); A((void**)&c->v, 4 * off);
  A((void**)&c->x, 4 * P * Q);
  A((void**)&c->h1, 4 * P * C); A((void**)&c->h2, 4 * P * C); A((void**)&c->h3, 4 * P * C);
  A((void**)&c->a4, 4 * P); A((void**)&c->prob, 4 * P); A((void**)&c->tgt, 4 * P); A((void**)&c->g4, 4 * P);
  A((void**)&c->gA, 4 * P * CMAX); A((void**)&c->gB, 4 * P * CMAX);
  A((void**)&c->part, 4 * (size_t)ntiles * CMAX * CMAX * 10);
  A((void**)&c->lpart, 8 * (size_t)((P + 255) / 256));
  A((void**)&c->mx, 8);
  if (rc == SADMM_OK && (hipMemsetAsync(c->p, 0, 4 * off, c->s) != hipSuccess ||
                         hipMemsetAsync(c->m, 0, 4 * off, c->s) != hipSuccess ||
                         hipMemsetAsync(c->v, 0, 4 * off, c->s) != hipSuccess ||
                         hipStreamSynchronize(c->s) != hipSuccess))
    rc = SADMM_E_HIP;
  if (rc != SADMM_OK) {
    sadmm_cnn_destroy(c);
    return rc;
  }
  *out = c;
  return SADMM_OK;
}

int64_t sadmm_cnn_param_count(sadmm_cnn_t c) { return c ? c->nparam : -1; }

int sadmm_cnn_set_params(sadmm_cnn_t c, const float* params, int64_t count) {
  if (!c) return SADMM_E_ARG;
  if (!params || count != c->nparam) return cfail(c, SADMM_E_SHAPE, "set_params: count mismatch");
  if (hipMemcpyAsync(c->p, params, 4 * count, hipMemcpyHostToDevice, c->s) != hipSuccess ||
      hipMemsetAsync(c->m, 0, 4 * count, c->s) != hipSuccess ||
      hipMemsetAsync(c->v, 0, 4 * count, c->s) != hipSuccess || hipStreamSynchronize(c->s) != hipSuccess)
    return cfail(c, SADMM_E_HIP, "set_params: copy failed");
  c->step = 0;
  return SADMM_OK;
}

int sadmm_cnn_get_params(sadmm_cnn_t c, float* params, int64_t count) {
  if (!c) return SADMM_E_ARG;
  if (!params || count != c->nparam) return cfail(c, SADMM_E_SHAPE, "get_params: count mismatch");
  if (hipMemcpyAsync(params, c->p, 4 * count, hipMemcpyDeviceToHost, c->s) != hipSuccess ||
      hipStreamSynchronize(c->s) != hipSuccess)
    return cfail(c, SADMM_E_HIP, "get_params: copy failed");
  return SADMM_OK;
}

int sadmm_cnn_forward(sadmm_cnn_t c, const float* x, int32_t x_on_device, float* prob,
                      int32_t prob_on_device) {
  if (!c) return SADMM_E_ARG;
  if (!x || !prob) return cfail(c, SADMM_E_ARG, "forward: null pointer");
  const int64_t P = (int64_t)c->H * c->W;
  int rc = put_input(c, c->x, x, P * c->Q, x_on_device);
  if (rc) return rc;
  cnn_forward_dev(c, c->half != 0);
  bce_kernel<<<(unsigned)((P + 255) / 256), 256, 0, c->s>>>(c->a4, nullptr, (int)P, 1.f, c->prob, nullptr, nullptr);
  if (hipMemcpyAsync(prob, c->prob, 4 * P, prob_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                     c->s) != hipSuccess ||
      hipStreamSynchronize(c->s) != hipSuccess)
    return cfail(c, SADMM_E_HIP, "forward failed");
  return SADMM_OK;
}

int sadmm_cnn_forward_noalloc(sadmm_cnn_t c, const float* x, int32_t H, int32_t W, float* prob) {
  if (!c) return SADMM_E_ARG;
  if (!x || !prob) return cfail(c, SADMM_E_ARG, "forward_noalloc: null pointer");
  if (H < 1 || W < 1 || (int64_t)H * W > NOALLOC_MAX_PIXELS)
    return cfail(c, SADMM_E_SHAPE, "forward_noalloc: H * W must lie in [1, 262144]");
  float* sc = nullptr;
  const int rc = noalloc_scratch(c, &sc);
  if (rc) return rc;
  const int64_t P = (int64_t)H * W;
  float* const s0 = sc;
  float* const s1 = sc + CMAX * P;
  float* const out[4] = {s0, s1, s0, sc + 2 * CMAX * P};
  cnn_layers(c, x, H, W, out, c->half != 0);
  bce_kernel<<<(unsigned)((P + 255) / 256), 256, 0, c->s>>>(out[3], nullptr, (int)P, 1.f, prob, nullptr, nullptr);
  if (hipGetLastError() != hipSuccess) return cfail(c, SADMM_E_HIP, "forward_noalloc: launch failed");
  return SADMM_OK;
}

int sadmm_cnn_set_half(sadmm_cnn_t c, int32_t on) {
  if (!c) return SADMM_E_ARG;
  if (on != 0 && on != 1) return cfail(c, SADMM_E_ARG, "set_half: 0 or 1");
  c->half = on;
  return SADMM_OK;
}

int sadmm_cnn_gradients(sadmm_cnn_t c, const float* x, const float* target, int32_t on_device,
                        float pos_weight, float* grads, double* loss) {
  if (!c) return SADMM_E_ARG;
  if (!x || !target || !grads) return cfail(c, SADMM_E_ARG, "gradients: null pointer");
  const int64_t P = (int64_t)c->H * c->W;
  int rc = put_input(c, c->x, x, P * c->Q, on_device);
  if (!rc) rc = put_input(c, c->tgt, target, P, on_device);
  if (!rc) rc = cnn_backward_dev(c, pos_weight, loss);
  if (rc) return rc;
  if (hipMemcpyAsync(grads, c->g, 4 * c->nparam, hipMemcpyDeviceToHost, c->s) != hipSuccess ||
      hipStreamSynchronize(c->s) != hipSuccess)
    return cfail(c, SADMM_E_HIP, "gradients: copy failed");
  return SADMM_OK;
}

int sadmm_cnn_train_step(sadmm_cnn_t c, const float* x, const float* target, int32_t on_device,
                         float pos_weight, float lr, double* loss) {
  if (!c) return SADMM_E_ARG;
  if (!x || !target) return cfail(c, SADMM_E_ARG, "train_step: null pointer");
  const int64_t P = (int64_t)c->H * c->W;
  int rc = put_input(c, c->x, x, P * c->Q, on_device);
  if (!rc) rc = put_input(c, c->tgt, target, P, on_device);
  if (!rc) rc = cnn_backward_dev(c, pos_weight, loss);
  if (rc) return rc;
  c->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)c->step), c2 = 1.f - powf(b2, (float)c->step);
  adam_kernel<<<(unsigned)((c->nparam + 255) / 256), 256, 0, c->s>>>(c->p, c->g, c->m, c->v, c->nparam, lr, b1,
                                                                     b2, 1e-8f, c1, c2);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->s) != hipSuccess)
    return cfail(c, SADMM_E_HIP, "train_step: adam failed");
  return SADMM_OK;
}

void sadmm_cnn_destroy(sadmm_cnn_t c) {
  if (!c) return;
  if (c->s) hipStreamSynchronize(c->s);
  for (void* p : c->allocs) hipFree(p);
  delete c;
}

const char* sadmm_cnn_last_error(sadmm_cnn_t c) { return c ? c->err.c_str() : "null handle"; }

}  // extern "C"
