// Multi-right-hand-side iteration for scenes that share one FP32 operator.
//
// Frames taken with the same array geometry share A_q and, without pixel
// elimination, the factor W_q.  The x-update of eq. (3) (Woodbury form,
// x = Ahat^H W y' + (beta/c)(v - Ahat^H W Ahat v)) then needs, per sensor and
// iteration, T = Ahat V and Y = Ahat^H (W T) for the S columns v of the S
// scenes: skinny GEMMs that read the operator once for all scenes.  They run on
// the FP32 16x16x4 matrix instruction (FP32 operands as in the single-scene
// path, FP32 accumulation); W T is an FP64 GEMM (the factor stays FP64).
// Lane layout of the instruction: lane l carries A[l % 16][l / 16] and
// B[l / 16][l % 16]; result element (4 (l / 16) + r, l % 16) is component r.
#include "iter.h"
#include "linalg.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// V[q][n][s] = x_q - xbar + z - u of scene s at pixel n (zero for halted scenes).
__global__ __launch_bounds__(256) void mrhs_v_kernel(BatchView bv, SharedBatch sb, int N) {
  const int q = blockIdx.y;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int S = sb.S;
  if (t >= (int64_t)N * S) return;
  const int s = (int)(t % S), n = (int)(t / S);
  const IterArgs& a = bv.args[s];
  float2 v = make_float2(0.f, 0.f);
  if (!a.ctl->halt) {
    const float2 x = reinterpret_cast<const float2*>(a.X)[(int64_t)q * a.N + n];
    const float2 xb = reinterpret_cast<const float2*>(a.xbar)[n];
    const float2 z = reinterpret_cast<const float2*>(a.z)[n];
    const float2 u = reinterpret_cast<const float2*>(a.u)[n];
    v = make_float2(((x.x - xb.x) + z.x) - u.x, ((x.y - xb.y) + z.y) - u.y);
  }
  reinterpret_cast<float2*>(sb.Vb)[((int64_t)q * N + n) * S + s] = v;
}

// Forward partial sums: work-group = 64 rows x all scenes over one chunk of
// MRHS_CHUNK pixels of sensor blockIdx.z; wave w owns rows 16w..16w+15 and
// SB blocks of 16 scenes.
template <int SB>
__global__ __launch_bounds__(256) void mrhs_fwd_kernel(BatchView bv, SharedBatch sb, int KMp, int N) {
  const int q = blockIdx.z, c = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + 16 * w + (lane & 15);
  const int kq = lane >> 4;
  const SensorDesc sd = bv.args[0].sens[q];
  const float2* A = reinterpret_cast<const float2*>(sd.A);
  const float2* V = reinterpret_cast<const float2*>(sb.Vb) + (int64_t)q * N * sb.S;
  const int S = sb.S;
  v4f cr[SB], ci[SB];
#pragma unroll
  for (int b = 0; b < SB; ++b) { cr[b] = v4f{0.f, 0.f, 0.f, 0.f}; ci[b] = v4f{0.f, 0.f, 0.f, 0.f}; }
  // V is the same for the four waves (they differ by rows): blocks of 64
  // pixels x all scenes are staged in LDS once per work-group.  Within a block,
  // rounds of four k-steps take k = p + 4 g + i for instruction i and lane
  // group g = lane / 16 (any assignment of k shared by both operands gives the
  // same sum).
  constexpr int PB = 64;
  __shared__ float2 sV[PB][16 * SB + 1];
  const int p0 = c * MRHS_CHUNK, p1 = min(N, p0 + MRHS_CHUNK);
  for (int pb = p0; pb < p1; pb += PB) {
    __syncthreads();
    for (int e = threadIdx.x; e < PB * 16 * SB; e += 256) {
      const int ss = e % (16 * SB), pp = e / (16 * SB);
      const int pk = pb + pp;
      sV[pp][ss] = (pk < p1 && ss < S) ? V[(int64_t)pk * S + ss] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int pr = 0; pr < PB; pr += 16) {
      float2 av[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pk = pb + pr + 4 * kq + i;
        av[i] = (pk < p1 && row < KMp) ? A[(int64_t)pk * sd.lda + row] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float2 vv[SB];
#pragma unroll
        for (int b = 0; b < SB; ++b) vv[b] = sV[pr + 4 * kq + i][16 * b + (lane & 15)];
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, vv[b].x, cr[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, vv[b].y, ci[b], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-av[i].y, vv[b].y, cr[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, vv[b].x, ci[b], 0, 0, 0);
        }
      }
    }
  }
  float2* Tp = reinterpret_cast<float2*>(sb.Tp) + ((int64_t)c * gridDim.z + q) * KMp * S;
#pragma unroll
  for (int b = 0; b < SB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = blockIdx.x * 64 + 16 * w + 4 * kq + r;
      const int s = 16 * b + (lane & 15);
      if (rr < KMp && s < S) Tp[(int64_t)rr * S + s] = make_float2(cr[b][r], ci[b][r]);
    }
}

// T64[q][s][row] = sum over chunks (FP64).
__global__ __launch_bounds__(256) void mrhs_reduce_kernel(SharedBatch sb, int Q, int KMp) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int S = sb.S;
  if (t >= (int64_t)Q * KMp * S) return;
  const int s = (int)(t % S);
  const int64_t qr = t / S;
  const int row = (int)(qr % KMp), q = (int)(qr / KMp);
  const float2* Tp = reinterpret_cast<const float2*>(sb.Tp);
  double re = 0.0, im = 0.0;
  for (int c = 0; c < sb.nch; ++c) {
    const float2 v = Tp[(((int64_t)c * Q + q) * KMp + row) * S + s];
    re += v.x;
    im += v.y;
  }
  sb.T64[((int64_t)q * S + s) * KMp + row] = cd{re, im};
}

// W T to FP32 for the adjoint operands.
__global__ __launch_bounds__(256) void mrhs_cvt_kernel(SharedBatch sb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const cd v = sb.Wt64[i];
  reinterpret_cast<float2*>(sb.Wt32)[i] = make_float2((float)v.re, (float)v.im);
}

// Adjoint and x-update: work-group = 64 pixels x all scenes of sensor
// blockIdx.y; wave w owns pixels 16w..16w+15.  Y = Ahat^H (W T); the epilogue
// is the x-update of every (pixel, scene) as in the single-scene path.
template <int SB>
__global__ __launch_bounds__(256) void mrhs_adj_kernel(BatchView bv, SharedBatch sb, int KMp) {
  const int q = blockIdx.y;
  const IterArgs& a0 = bv.args[0];
  const SensorDesc sd = a0.sens[q];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kq = lane >> 4;
  const int pa = blockIdx.x * 64 + 16 * w + (lane & 15);   // pixel of this lane's A operand
  const int nq = sd.nq;
  const float2* A = reinterpret_cast<const float2*>(sd.A);
  const int S = sb.S;
  const float2* Wt = reinterpret_cast<const float2*>(sb.Wt32) + (int64_t)q * S * KMp;
  v4f cr[SB], ci[SB];
#pragma unroll
  for (int b = 0; b < SB; ++b) { cr[b] = v4f{0.f, 0.f, 0.f, 0.f}; ci[b] = v4f{0.f, 0.f, 0.f, 0.f}; }
  // W T is the same for the four waves: blocks of 64 k x all scenes are staged
  // in LDS ([k][scene]).  Rounds of four k-steps take k = k0 + 4 g + i
  // (g = lane / 16): each lane reads 4 consecutive entries of its column.
  constexpr int KB = 64;
  __shared__ float2 sW[KB][16 * SB + 1];
  for (int kb0 = 0; kb0 < KMp; kb0 += KB) {
    __syncthreads();
    for (int e = threadIdx.x; e < KB * 16 * SB; e += 256) {
      const int kk = e % KB, ss = e / KB;
      sW[kk][ss] = (ss < S && kb0 + kk < KMp) ? Wt[(int64_t)ss * KMp + kb0 + kk] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int kr = 0; kr < KB; kr += 16) {
      const int kb = kb0 + kr + 4 * kq;
      float4 a01 = make_float4(0.f, 0.f, 0.f, 0.f), a23 = a01;
      if (pa < nq && kb < KMp) {   // KMp is a multiple of 32: kb + 3 < KMp
        const float4* ap = reinterpret_cast<const float4*>(A + (int64_t)pa * sd.lda + kb);
        a01 = ap[0];
        a23 = ap[1];
      }
      const float ar[4] = {a01.x, a01.z, a23.x, a23.z};
      const float ai[4] = {a01.y, a01.w, a23.y, a23.w};
      // (ar - j ai)(wr + j wi) = (ar wr + ai wi) + j (ar wi - ai wr)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float2 wv[SB];
#pragma unroll
        for (int b = 0; b < SB; ++b) wv[b] = sW[kr + 4 * kq + i][16 * b + (lane & 15)];
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], wv[b].x, cr[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], wv[b].y, ci[b], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], wv[b].y, cr[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[i], wv[b].x, ci[b], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < SB; ++b) {
    const int s = 16 * b + (lane & 15);
    if (s >= S) continue;
    const IterArgs& a = bv.args[s];
    if (a.ctl->halt) continue;
    const SensorDesc ss = a.sens[q];
    const float bc = (float)a.bc;
    const int slot = a.ctl->k % a.Kp;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = blockIdx.x * 64 + 16 * w + 4 * kq + r;
      if (p >= nq) continue;
      const int n = ss.J[p];
      const int64_t o = (int64_t)q * a.N + n;
      const float2 x = reinterpret_cast<const float2*>(a.X)[o];
      const float2 xb = reinterpret_cast<const float2*>(a.xbar)[n];
      const float2 z = reinterpret_cast<const float2*>(a.z)[n];
      const float2 u = reinterpret_cast<const float2*>(a.u)[n];
      const float vr = ((x.x - xb.x) + z.x) - u.x, vi = ((x.y - xb.y) + z.y) - u.y;
      const float2 xy = reinterpret_cast<const float2*>(ss.xy)[p];
      const float xr = xy.x + bc * (vr - cr[b][r]), xi = xy.y + bc * (vi - ci[b][r]);
      const float dr = xr - x.x, di = xi - x.y;
      reinterpret_cast<float2*>(a.X)[o] = make_float2(xr, xi);
      reinterpret_cast<float2*>(a.dX)[o] = make_float2(dr, di);
      reinterpret_cast<float*>(a.D)[((int64_t)slot * a.Q + q) * a.N + n] = hypotf(dr, di);
    }
  }
}

template <int SB>
void launch_products(const BatchView& b, const BatchDims& d, const SharedBatch& sb, int Q, int N,
                     int KMp, hipStream_t s, const std::function<void(int, bool)>* hook) {
  auto mark = [&](int stage, bool begin) { if (hook) (*hook)(stage, begin); };
  mark(0, true);
  mrhs_v_kernel<<<dim3((unsigned)(((int64_t)N * sb.S + 255) / 256), Q), 256, 0, s>>>(b, sb, N);
  mrhs_fwd_kernel<SB><<<dim3((KMp + 63) / 64, sb.nch, Q), 256, 0, s>>>(b, sb, KMp, N);
  mrhs_reduce_kernel<<<(unsigned)(((int64_t)Q * KMp * sb.S + 255) / 256), 256, 0, s>>>(sb, Q, KMp);
  mark(0, false);
  mark(1, true);
  zgemm_mfma_nn(static_cast<const MmDesc*>(sb.wdesc), Q, KMp, sb.S, s);
  mrhs_cvt_kernel<<<(unsigned)(((int64_t)Q * KMp * sb.S + 255) / 256), 256, 0, s>>>(sb, (int64_t)Q * KMp * sb.S);
  mark(1, false);
  mark(2, true);
  mrhs_adj_kernel<SB><<<dim3((N + 63) / 64, Q), 256, 0, s>>>(b, sb, KMp);
  mark(2, false);
  (void)d;
}

}  // namespace

void launch_iteration_shared(const BatchView& b, const BatchDims& d, const SharedBatch& sb,
                             hipStream_t s, const std::function<void(int, bool)>* hook) {
  // every scene has the same Q, N and KMp (checked by the caller)
  const int Q = d.nslot / d.nscene, N = d.N_max, KMp = d.KMp_max;
  switch ((sb.S + 15) / 16) {
    case 1: launch_products<1>(b, d, sb, Q, N, KMp, s, hook); break;
    case 2: launch_products<2>(b, d, sb, Q, N, KMp, s, hook); break;
    case 3: launch_products<3>(b, d, sb, Q, N, KMp, s, hook); break;
    default: launch_products<4>(b, d, sb, Q, N, KMp, s, hook); break;
  }
  if (hook) (*hook)(3, true);
  launch_pixel_stage(b, d, false, s);
  if (hook) (*hook)(3, false);
}
