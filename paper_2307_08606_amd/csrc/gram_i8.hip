// Exact-integer Gram Ahat Ahat^H on the int8 16x16x64 matrix instruction.
//
// The Gram is the dense contraction of a factor build (x-update of eq. (3) in
// Woodbury form).  MI355X runs int8 matrix products 64 times faster than FP64
// ones, and the operator entries are bounded (|A| = 1 for the steering vectors
// of eq. (1)), so the product is split into digit products that are exact in
// int32 (see gram.h for the number format and the error bound).
//
// Complex product with L = rows i and R = rows j of Ahat:
//   Re G = Lr Rr^T + Li Ri^T,   Im G = Li Rr^T - Lr Ri^T.
// The subtraction uses bitwise NOT of the real digits (~d = -d - 1, exact in
// int8 for every d) and adds back the sum of the imaginary digits of row j.
//
// Work-group: 64 x 64 complex tile of the lower triangle (XCD-aware order, see
// tri_tile_order), eight waves of 32 x 16 (2 x 1 blocks of 16 x 16, two waves
// per SIMD), each accumulating all 13 digit pairs with s + t <= 4 into five
// int32 class accumulators (c = s + t).
// Lane layout of the instruction: lane l carries A row l % 16 and B column
// l % 16 with k-slots 16 (l / 16) + byte (any order shared by A and B gives
// the same product); result element (4 (l / 16) + r, l % 16) is component r
// of lane l (unlike the FP64 16x16x4 instruction, whose rows are 4 r + l / 16).
#include <algorithm>

#include "gram.h"
#include "linalg.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int GT = 64;      // tile rows / columns (complex)
constexpr int GKS = 64;     // columns per stage (k of one instruction)
constexpr int GROW = 64;    // LDS bytes per staged row (16-byte quarters swizzled, see swz)
constexpr int GLD = 2 * GKS;  // digit-plane rows padded to an even number of stages

inline int round_up_i(int x, int m) { return (x + m - 1) / m * m; }

// Digit planes are stored stage-blocked: for row block rb (64 rows) and stage
// st (64 columns), the 8 planes' 64 x 64-byte tiles lie in one contiguous
// 32 KB block, so a work-group's stage of a panel is one contiguous read.
constexpr int64_t kStageBlock = 8 * 64 * 64;
__host__ __device__ inline int64_t stage_block(int rb, int st, int ldS) {
  return ((int64_t)rb * (ldS / 64) + st) * kStageBlock;
}

// Zeroes rmax (when clear_rmax) and the per-chunk digit sums rs.
__global__ void clear_kernel(const GramI8Desc* __restrict__ descs, int clear_rmax, int clear_rs) {
  const GramI8Desc d = descs[blockIdx.y];
  const int nch = (d.ldS + GI8_CHUNK - 1) / GI8_CHUNK;
  const int64_t n1 = d.KMr, n2 = clear_rs ? (int64_t)nch * 4 * d.KMr : 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n1) {
      if (clear_rmax) d.rmax[i] = 0ull;
    } else {
      d.rs[i - n1] = 0;
    }
  }
}

// rmax[i] = bits of max_n max(|Re A[i,n]|, |Im A[i,n]|) (non-negative doubles
// order like their bit patterns).
template <int ST>
__global__ __launch_bounds__(256) void rowmax_kernel(const GramI8Desc* __restrict__ descs) {
  const GramI8Desc d = descs[blockIdx.z];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d.m) return;
  const int per = (d.k + gridDim.y - 1) / gridDim.y;
  const int n0 = blockIdx.y * per, n1 = min(d.k, n0 + per);
  double mx = 0.0;
  for (int n = n0; n < n1; ++n) {
    const cd v = Store<ST>::get_stream(col_ptr<ST>(d.A, d.ldA, n), i, d.kmp);
    mx = fmax(mx, fmax(fabs(v.re), fabs(v.im)));
  }
  if (n1 > n0) atomicMax(&d.rmax[i], (unsigned long long)__double_as_longlong(mx));
}

// Digit planes.  Block: 64 rows x SL_SUB sub-tiles of SL_COLS columns, one
// after the other.  Thread (row = t & 63, column group cg = t >> 6) reads
// SL_COLS / 4 consecutive columns of its row per sub-tile (the lanes of a
// wave read 64 consecutive rows of one column: coalesced), forms the digits in
// FP32 / int32 (the stored values have at most 24 significant bits, so the
// power-of-two scaling and the rounding to an integer are exact) and packs
// them into LDS; the block then writes the sub-tile's stage blocks with
// consecutive lanes on consecutive 16-byte pieces.  The per-row digit sums of
// the block's columns go out with one atomic add per (row, digit).  Rows >= m
// and columns >= k get zero digits.
constexpr int SL_COLS = 128;
constexpr int SL_SUB = 1;   // sub-tiles of SL_COLS columns per block (GI8_CHUNK is a multiple of their width)
static_assert(GI8_CHUNK % (SL_COLS * SL_SUB) == 0, "a block's columns stay in one chunk");
constexpr int SL_W = SL_COLS / 4 + 1;   // LDS words per tile row (+1: no bank conflicts)

template <int ST>
__global__ __launch_bounds__(256) void slice_kernel(const GramI8Desc* __restrict__ descs) {
  const GramI8Desc d = descs[blockIdx.z];
  const int row = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int gi = blockIdx.y * 64 + row;
  const int cb0 = blockIdx.x * SL_COLS * SL_SUB;
  if (blockIdx.y * 64 >= d.KMr || cb0 >= d.ldS) return;
  __shared__ uint32_t sd[8][64][SL_W];   // [2 digit + re/im][row][column word]
  __shared__ int red[4][4][64];          // [column group][digit][row]
  const double mx = gi < d.m ? __longlong_as_double((long long)d.rmax[gi]) : 0.0;
  int E = 0;
  if (mx > 0.0) (void)frexp(mx, &E);
  int rsum[4] = {0, 0, 0, 0};
  constexpr int PER = SL_COLS / 4;       // columns per thread
  for (int sub = 0; sub < SL_SUB; ++sub) {
    const int cb = cb0 + sub * SL_COLS;
    if (cb >= d.ldS) break;              // (uniform across the block)
    if (sub > 0) __syncthreads();        // the previous sub-tile is written out
#pragma unroll
    for (int wd = 0; wd < PER / 4; ++wd) {   // one packed word (4 columns) per plane
      uint32_t pk[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gn = cb + PER * cg + 4 * wd + e;
        float vv[2] = {0.f, 0.f};
        if (gi < d.m && gn < d.k) {
          const cd v = Store<ST>::get_stream(col_ptr<ST>(d.A, d.ldA, gn), gi, d.kmp);
          vv[0] = (float)v.re;
          vv[1] = (float)v.im;
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          int x = (int)rintf(ldexpf(vv[p], 30 - E));   // |x| < 2^30
          int dg[4];
#pragma unroll
          for (int t = 3; t >= 1; --t) {
            const int lo = (int)(int8_t)(uint8_t)(x & 0xff);
            dg[t] = lo;
            x = (x - lo) >> 8;
          }
          dg[0] = x;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            pk[2 * t + p] |= ((uint32_t)(uint8_t)dg[t]) << (8 * e);
            if (p == 1) rsum[t] += dg[t];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) sd[q][row][(PER / 4) * cg + wd] = pk[q];
    }
    __syncthreads();
    // write-out: consecutive threads take the 4 pieces of a stage row, then
    // rows, then planes, then stages: contiguous stores in the stage-blocked
    // layout
    constexpr int PCS = SL_COLS / 16;   // pieces per row
    for (int e = threadIdx.x; e < 8 * 64 * PCS; e += 256) {
      const int c4 = e & 3, r = (e >> 2) & 63, q = (e >> 8) & 7, sg = e >> 11;
      const int col = cb + 64 * sg + 16 * c4;
      if (col >= d.ldS) continue;
      const uint32_t* w = &sd[q][r][(64 * sg + 16 * c4) / 4];
      typedef unsigned u4 __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(u4{w[0], w[1], w[2], w[3]},
                                  reinterpret_cast<u4*>(d.S + stage_block(blockIdx.y, col / 64, d.ldS) +
                                                        (int64_t)q * 4096 + r * 64 + 16 * c4));
    }
  }
  // per-row digit sums of the block's columns (all in one chunk)
#pragma unroll
  for (int t = 0; t < 4; ++t) red[cg][t][row] = rsum[t];
  __syncthreads();
  {
    const int t = threadIdx.x >> 6;   // thread (t, row) adds the four column groups
    const int v = red[0][t][row] + red[1][t][row] + red[2][t][row] + red[3][t][row];
    const int chunk = cb0 / GI8_CHUNK;
    if (v != 0 && gi < d.KMr) atomicAdd(&d.rs[((int64_t)chunk * 4 + t) * d.KMr + gi], v);
  }
}

using Panel = int8_t[2][4][2][GT][GROW];   // [L/R][digit][re/im][row][bytes]
// Quarter q of staged row `row` sits at 16 (q ^ swz(row)).  The 16 lanes
// reading one operand block take rows 16 m + [0, 16) at one quarter, and the
// lanes of a store take four consecutive rows: with unpadded 64-byte rows
// both land on distinct banks (32 or 64 banks of 4 bytes).
__device__ inline int swz(int row) {
  const int r = row & 15;
  return ((r >> 1) + (r >> 3)) & 3;
}
constexpr int NCLS = 5;                      // classes c = s + t = 0..4
#define LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))
// Wait until every global load of the wave (register or LDS destination) has
// landed; LDS and export counters untouched.
__device__ inline void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Staging of one stage (16 planes: L/R x digit x re/im, 64 rows x 64 bytes
// each) by a work-group of 512 threads, straight from the stage blocks into
// LDS with no register staging.  Thread t moves row (t >> 2) & 63 of the
// eight planes of side t >> 8 (L, then R).  The instruction writes lane l's
// 16 bytes at 16 l from the wave's LDS base, i.e. at row prow, quarter slot
// l & 3 of the wave's 16 rows, so the lane fetches the row's quarter
// (l & 3) ^ swz(prow): the swizzle is applied on the global side.
struct StageLoader {
  static constexpr int64_t kPlane = 4096;        // between the planes of a stage block
  static constexpr int kPlaneLds = GT * GROW;    // between the (digit, re/im) planes in LDS
  const int8_t* src;
  int8_t* lds[2];
  __device__ StageLoader(const GramI8Desc& d, Panel (&sp)[2], int ti, int tj) {
    const int t = threadIdx.x, prow = (t >> 2) & 63, side = t >> 8, lrow = 16 * ((t >> 6) & 3);
    src = d.S + stage_block(side ? tj : ti, 0, d.ldS) + prow * 64 + 16 * ((t & 3) ^ swz(prow));
    lds[0] = &sp[0][side][0][0][lrow][0];
    lds[1] = &sp[1][side][0][0][lrow][0];
  }
  // stage `stage` (columns 64 stage ..) of both panels into sp[buf]
  __device__ void issue(int stage, int buf) const {
    const int8_t* g = src + (int64_t)stage * kStageBlock;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      __builtin_amdgcn_global_load_lds(g + e * kPlane, LDS_PTR(lds[buf] + e * kPlaneLds), 16, 0, 0);
    __builtin_amdgcn_sched_barrier(0x0008);   // not sunk to the wait; matrix products may pass
  }
};

// Eight waves per work-group (two per SIMD, so one wave's LDS reads overlap
// the other's matrix instructions): wave w owns rows 32 (w & 1) + [0, 32)
// (two 16-row blocks a) and columns 16 (w >> 1) + [0, 16) (one block).
constexpr int GWAVES = 8;
constexpr int GTHREADS = 64 * GWAVES;
constexpr int BB = 1;                        // 16-column blocks per wave

// Digit s of the wave's two L row blocks (real, imaginary, NOT of real).
struct LDigit { v4i r[2], i[2], nr[2]; };
template <int S>
__device__ inline LDigit load_l(const Panel& sp, int wr, int r16, int kq) {
  LDigit L;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    L.r[a] = *reinterpret_cast<const v4i*>(&sp[0][S][0][wr + 16 * a + r16][16 * kq]);
    L.i[a] = *reinterpret_cast<const v4i*>(&sp[0][S][1][wr + 16 * a + r16][16 * kq]);
    L.nr[a] = ~L.r[a];
  }
  return L;
}
// R digits of the wave's column block(s), all four held for the stage.
struct RDigits { v4i r[4][BB], i[4][BB]; };
__device__ inline void load_r(const Panel& sp, int wc, int r16, int kq, RDigits& R) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int b = 0; b < BB; ++b) {
      R.r[t][b] = *reinterpret_cast<const v4i*>(&sp[1][t][0][wc + 16 * b + r16][16 * kq]);
      R.i[t][b] = *reinterpret_cast<const v4i*>(&sp[1][t][1][wc + 16 * b + r16][16 * kq]);
    }
}
// Accumulate the products of an L digit with R digit T into class slot C.
template <int T, int C>
__device__ inline void pair_mma(const LDigit& L, const RDigits& R, v4i (&re)[NCLS][2][BB],
                                v4i (&im)[NCLS][2][BB]) {
  // in rounds over the (a, b) blocks, so that the two products into one
  // accumulator are apart
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b) {
      re[C][a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(L.r[a], R.r[T][b], re[C][a][b], 0, 0, 0);
      im[C][a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(L.i[a], R.r[T][b], im[C][a][b], 0, 0, 0);
    }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b) {
      re[C][a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(L.i[a], R.i[T][b], re[C][a][b], 0, 0, 0);
      im[C][a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(L.nr[a], R.i[T][b], im[C][a][b], 0, 0, 0);
    }
}

// One stage of 64 columns: the R digits read once, the 13 pairs grouped by L
// digit (the compiler may load the next L digit during the current group's
// products).
__device__ inline void kstep(const Panel& sp, int wr, int wc, int r16, int kq,
                             v4i (&re)[NCLS][2][BB], v4i (&im)[NCLS][2][BB]) {
  RDigits R;
  load_r(sp, wc, r16, kq, R);
  { const LDigit L = load_l<0>(sp, wr, r16, kq);
    pair_mma<0, 0>(L, R, re, im);
    pair_mma<1, 1>(L, R, re, im);
    pair_mma<2, 2>(L, R, re, im);
    pair_mma<3, 3>(L, R, re, im); }
  { const LDigit L = load_l<1>(sp, wr, r16, kq);
    pair_mma<0, 1>(L, R, re, im);
    pair_mma<1, 2>(L, R, re, im);
    pair_mma<2, 3>(L, R, re, im);
    pair_mma<3, 4>(L, R, re, im); }
  { const LDigit L = load_l<2>(sp, wr, r16, kq);
    pair_mma<0, 2>(L, R, re, im);
    pair_mma<1, 3>(L, R, re, im);
    pair_mma<2, 4>(L, R, re, im); }
  { const LDigit L = load_l<3>(sp, wr, r16, kq);
    pair_mma<0, 3>(L, R, re, im);
    pair_mma<1, 4>(L, R, re, im); }
}


// One chunk of columns [chunk * GI8_CHUNK, +GI8_CHUNK): chunk 0 writes
// C = G_0 + diag I, later chunks add.
__global__ __launch_bounds__(GTHREADS) void gram_i8_kernel(const GramI8Desc* __restrict__ descs, int chunk,
                                                             const int2* __restrict__ tiles, int ntiles) {
  const GramI8Desc d = descs[blockIdx.y];
  int ti, tj;
  if (!xcd_tile(tiles, ntiles, &ti, &tj)) return;
  const int i0 = ti * GT, j0 = tj * GT;
  if (i0 >= d.m) return;
  const int n0 = chunk * GI8_CHUNK;
  if (chunk > 0 && n0 >= d.ldS) return;   // nothing to add
  const int n1 = min(n0 + GI8_CHUNK, d.ldS);
  __shared__ __align__(16) Panel sp[2];   // double buffer: stage 2 s in sp[0], 2 s + 1 in sp[1]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = 32 * (w & 1), wc = 16 * BB * (w >> 1);
  const int r16 = lane & 15, kq = lane >> 4;
  const int kqs = kq ^ swz(r16);   // swizzled quarter of the lane's operand rows
  v4i re[NCLS][2][BB], im[NCLS][2][BB];
#pragma unroll
  for (int c = 0; c < NCLS; ++c)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < BB; ++b) {
        re[c][a][b] = v4i{0, 0, 0, 0};
        im[c][a][b] = v4i{0, 0, 0, 0};
      }
  const StageLoader ld(d, sp, ti, tj);
  // Stage s lands in sp[s & 1]; its loads are issued as the products of
  // stage s - 1 start and waited for before the barrier that ends them.  One
  // barrier per stage: a buffer is refilled only after the barrier that
  // follows the products reading it.
  if (n0 < n1) {
    ld.issue(n0 / GKS, 0);
    wait_loads();
    __syncthreads();
  }
  for (int nb = n0; nb < n1; nb += 2 * GKS) {
    ld.issue(nb / GKS + 1, 1);                                   // sp[1] is free since the last barrier
    kstep(sp[0], wr, wc, r16, kqs, re, im);                      // stage nb
    wait_loads();
    __syncthreads();
    // the last pair reloads its own second stage (L2-resident, never read):
    // without a branch the loads can issue among the products that trail the barrier
    ld.issue(min(nb / GKS + 2, n1 / GKS - 1), 0);
    kstep(sp[1], wr, wc, r16, kqs, re, im);                      // stage nb + GKS
    wait_loads();
    __syncthreads();
  }
  // ---- epilogue: FP64 sum of the classes, lower triangle and its mirror
  const int* rs = d.rs + (int64_t)chunk * 4 * d.KMr;
  int cre[BB][NCLS];   // imaginary correction: sum of rs_t over the class's pairs
  double sj[BB];
#pragma unroll
  for (int b = 0; b < BB; ++b) {
    const int j = j0 + wc + 16 * b + r16;
    int r4[4] = {0, 0, 0, 0};
    double mx = 0.0;
    if (j < d.m) {
#pragma unroll
      for (int q = 0; q < 4; ++q) r4[q] = rs[(int64_t)q * d.KMr + j];
      mx = __longlong_as_double((long long)d.rmax[j]);
    }
    int E = 0;
    if (mx > 0.0) (void)frexp(mx, &E);
    sj[b] = ldexp(1.0, E - 6);
    // class c holds the pairs (c - t, t), max(0, c - 3) <= t <= min(3, c)
    cre[b][0] = r4[0];
    cre[b][1] = r4[0] + r4[1];
    cre[b][2] = r4[0] + r4[1] + r4[2];
    cre[b][3] = r4[0] + r4[1] + r4[2] + r4[3];
    cre[b][4] = r4[1] + r4[2] + r4[3];
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + wr + 16 * a + 4 * kq + r;
      const double mx = i < d.m ? __longlong_as_double((long long)d.rmax[i]) : 0.0;
      int E = 0;
      if (mx > 0.0) (void)frexp(mx, &E);
      const double si = ldexp(1.0, E - 6);
#pragma unroll
      for (int b = 0; b < BB; ++b) {
        const int j = j0 + wc + 16 * b + r16;
        if (i >= d.m || j >= d.m || j > i) continue;
        // smallest class first: every partial sum keeps full FP64 accuracy
        double vr = 0.0, vi = 0.0;
#pragma unroll
        for (int c = NCLS - 1; c >= 0; --c) {
          const double wgt = ldexp(1.0, -8 * c);
          vr += (double)re[c][a][b][r] * wgt;
          vi += ((double)im[c][a][b][r] + (double)cre[b][c]) * wgt;
        }
        cd v = {vr * (si * sj[b]), vi * (si * sj[b])};
        cd* cij = d.C + (int64_t)j * d.ldc + i;
        if (chunk > 0) { v.re += cij->re; v.im += cij->im; }
        else if (i == j) v.re += d.diag;
        if (i == j) v.im = 0.0;
        *cij = v;
        if (i != j) d.C[(int64_t)i * d.ldc + j] = cd{v.re, -v.im};
      }
    }
}

// ---------------------------------------------------------------------------
// The same products on the int8 32x32x32 instruction, which a register-only
// loop issues about 1.5 times as fast as the 16x16x64 one on this GPU (up to
// 4.5 against 3.0 POP/s).  Work-group: the same 64 x 64 complex tile
// and double-buffered stages, eight waves: each 32 x 32 block of the tile
// has two, one accumulating the classes 0..2 (six digit pairs), the other the
// classes 3..4 (seven pairs), so that a wave holds at most six 16-register
// accumulators and two waves fit each SIMD.  The classes' FP64 sum meets in
// LDS, in the order of the 16x16x64 kernel (identical results).  It runs
// 6.7 ms per c2 chunk against 5.8 for gram_i8_kernel: inside the kernel a
// 32x32x32 product occupies the matrix unit exactly as long as two 16x16x64
// ones (equal busy-cycle counters), so the larger shape gains nothing here;
// it is kept as a cross-check of the integer arithmetic.
// Lane layout (pinned by an in-bounds probe): lane l carries A row l % 32 and
// B column l % 32 with k-bytes 16 (l / 32) + [0, 16) of the 32-byte step;
// result component e of lane l is element (8 (e / 4) + 4 (l / 32) + e % 4,
// l % 32).
typedef int v16i __attribute__((ext_vector_type(16)));
constexpr int G32_WAVES = 8;
constexpr int G32_THREADS = 64 * G32_WAVES;

__device__ inline v16i mma32(v4i a, v4i b, v16i c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}
// Digit pairs (s, t) of the two class groups, class c = s + t.
template <int G> struct Pairs32;
template <> struct Pairs32<0> {           // classes 0, 1, 2: digits 0..2
  static constexpr int NP = 6, NC = 3, C0 = 0, ND = 3;
  static constexpr int s[NP] = {0, 0, 1, 0, 1, 2};
  static constexpr int t[NP] = {0, 1, 0, 2, 1, 0};
};
template <> struct Pairs32<1> {           // classes 3, 4: digits 0..3
  static constexpr int NP = 7, NC = 2, C0 = 3, ND = 4;
  static constexpr int s[NP] = {0, 1, 2, 3, 1, 2, 3};
  static constexpr int t[NP] = {3, 2, 1, 0, 3, 2, 1};
};

// One 32-byte step of the wave's block for class group G: operands of
// digits 0 .. ND-1 read once (L rows lrow, R rows rrow, quarter q), then the
// first halves of all pairs and the second halves (the two products into one
// accumulator 2 NP instructions apart).
template <int G>
__device__ inline void kstep32(const Panel& sp, int lrow, int rrow, int q, v16i (&re)[Pairs32<G>::NC],
                               v16i (&im)[Pairs32<G>::NC]) {
  using P = Pairs32<G>;
  const int loff = 16 * (q ^ swz(lrow)), roff = 16 * (q ^ swz(rrow));
  v4i lr[P::ND], li[P::ND], rr[P::ND], ri[P::ND];
#pragma unroll
  for (int d = 0; d < P::ND; ++d) {
    lr[d] = *reinterpret_cast<const v4i*>(&sp[0][d][0][lrow][loff]);
    li[d] = *reinterpret_cast<const v4i*>(&sp[0][d][1][lrow][loff]);
    rr[d] = *reinterpret_cast<const v4i*>(&sp[1][d][0][rrow][roff]);
    ri[d] = *reinterpret_cast<const v4i*>(&sp[1][d][1][rrow][roff]);
  }
#pragma unroll
  for (int k = 0; k < P::NP; ++k) {
    const int c = P::s[k] + P::t[k] - P::C0;
    re[c] = mma32(lr[P::s[k]], rr[P::t[k]], re[c]);
    im[c] = mma32(li[P::s[k]], rr[P::t[k]], im[c]);
  }
#pragma unroll
  for (int k = 0; k < P::NP; ++k) {
    const int c = P::s[k] + P::t[k] - P::C0;
    re[c] = mma32(li[P::s[k]], ri[P::t[k]], re[c]);
    im[c] = mma32(~lr[P::s[k]], ri[P::t[k]], im[c]);
  }
}

// The stages of the chunk for class group G (every wave of the work-group
// runs the same barriers), then the group's classes of the block's elements
// in FP64 (x = largest class first, see the epilogue).  Group 1 leaves its
// partial sums in `part` (doubles, [re/im][element e][lane]); group 0 adds
// its classes to them and writes C.
template <int G>
__device__ inline void gram32_wave(const GramI8Desc& d, Panel (&sp)[2], int chunk, int ti, int tj, int n0,
                                   int n1, int blk, double* part) {
  using P = Pairs32<G>;
  const int t = threadIdx.x, lane = t & 63;
  const int ba = blk & 1, bb = blk >> 1;   // L rows 32 ba.., R rows 32 bb..
  const int lrow = 32 * ba + (lane & 31), rrow = 32 * bb + (lane & 31), kh = lane >> 5;
  v16i re[P::NC], im[P::NC];
#pragma unroll
  for (int c = 0; c < P::NC; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      re[c][e] = 0;
      im[c][e] = 0;
    }
  // staging and barriers as in gram_i8_kernel
  const StageLoader ld(d, sp, ti, tj);
  if (n0 < n1) {
    ld.issue(n0 / GKS, 0);
    wait_loads();
    __syncthreads();
  }
  for (int nb = n0; nb < n1; nb += 2 * GKS) {
    ld.issue(nb / GKS + 1, 1);
    kstep32<G>(sp[0], lrow, rrow, kh, re, im);                   // stage nb
    kstep32<G>(sp[0], lrow, rrow, 2 + kh, re, im);
    wait_loads();
    __syncthreads();
    ld.issue(min(nb / GKS + 2, n1 / GKS - 1), 0);
    kstep32<G>(sp[1], lrow, rrow, kh, re, im);                   // stage nb + GKS
    kstep32<G>(sp[1], lrow, rrow, 2 + kh, re, im);
    wait_loads();
    __syncthreads();
  }
  // ---- epilogue: the classes summed in FP64 from the largest c down (the
  // order of gram_i8_kernel); group 1 (classes 4, 3) first, through LDS
  const int* rs = d.rs + (int64_t)chunk * 4 * d.KMr;
  const int j = tj * GT + 32 * bb + (lane & 31);
  int r4[4] = {0, 0, 0, 0};
  double mxj = 0.0;
  if (j < d.m) {
#pragma unroll
    for (int q = 0; q < 4; ++q) r4[q] = rs[(int64_t)q * d.KMr + j];
    mxj = __longlong_as_double((long long)d.rmax[j]);
  }
  // class c holds the pairs (c - t, t), max(0, c - 3) <= t <= min(3, c)
  const int cre_all[NCLS] = {r4[0], r4[0] + r4[1], r4[0] + r4[1] + r4[2], r4[0] + r4[1] + r4[2] + r4[3],
                             r4[1] + r4[2] + r4[3]};
  double* pr = part + (int64_t)blk * 2 * 16 * 64;       // [re/im][e][lane] of this block
  __syncthreads();                                      // the panels are free: part aliases them
  if constexpr (G == 1) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      double vr = 0.0, vi = 0.0;
#pragma unroll
      for (int c = NCLS - 1; c >= P::C0; --c) {
        const double wgt = ldexp(1.0, -8 * c);
        vr += (double)re[c - P::C0][e] * wgt;
        vi += ((double)im[c - P::C0][e] + (double)cre_all[c]) * wgt;
      }
      pr[e * 64 + lane] = vr;
      pr[(16 + e) * 64 + lane] = vi;
    }
  }
  __syncthreads();
  if constexpr (G == 0) {
    int E = 0;
    if (mxj > 0.0) (void)frexp(mxj, &E);
    const double sj = ldexp(1.0, E - 6);
    const int i0 = ti * GT;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = i0 + 32 * ba + 8 * (e >> 2) + 4 * kh + (e & 3);
      if (i >= d.m || j >= d.m || j > i) continue;
      const double mx = __longlong_as_double((long long)d.rmax[i]);
      int Ei = 0;
      if (mx > 0.0) (void)frexp(mx, &Ei);
      const double si = ldexp(1.0, Ei - 6);
      double vr = pr[e * 64 + lane], vi = pr[(16 + e) * 64 + lane];
#pragma unroll
      for (int c = P::NC - 1; c >= 0; --c) {
        const double wgt = ldexp(1.0, -8 * c);
        vr += (double)re[c][e] * wgt;
        vi += ((double)im[c][e] + (double)cre_all[c]) * wgt;
      }
      cd v = {vr * (si * sj), vi * (si * sj)};
      cd* cij = d.C + (int64_t)j * d.ldc + i;
      if (chunk > 0) { v.re += cij->re; v.im += cij->im; }
      else if (i == j) v.re += d.diag;
      if (i == j) v.im = 0.0;
      *cij = v;
      if (i != j) d.C[(int64_t)i * d.ldc + j] = cd{v.re, -v.im};
    }
  }
}

__global__ __launch_bounds__(G32_THREADS) void gram_i8_32_kernel(const GramI8Desc* __restrict__ descs, int chunk,
                                                                   const int2* __restrict__ tiles, int ntiles) {
  const GramI8Desc d = descs[blockIdx.y];
  int ti, tj;
  if (!xcd_tile(tiles, ntiles, &ti, &tj)) return;
  if (ti * GT >= d.m) return;
  const int n0 = chunk * GI8_CHUNK;
  if (chunk > 0 && n0 >= d.ldS) return;   // nothing to add
  const int n1 = min(n0 + GI8_CHUNK, d.ldS);
  __shared__ __align__(16) Panel sp[2];   // double buffer: stage 2 s in sp[0], 2 s + 1 in sp[1]
  static_assert(sizeof(Panel) * 2 >= 4 * 2 * 16 * 64 * sizeof(double), "class partials fit the panels");
  double* part = reinterpret_cast<double*>(&sp[0][0][0][0][0][0]);
  const int w = threadIdx.x >> 6;
  if (w < 4) gram32_wave<0>(d, sp, chunk, ti, tj, n0, n1, w, part);
  else gram32_wave<1>(d, sp, chunk, ti, tj, n0, n1, w - 4, part);
}

template <int ST>
void launch_prep(const GramI8Desc* d, int batch, int KMr, int ldS, int max_k, bool rmax_given,
                 bool planes, hipStream_t s) {
  const int nb = std::max(1, std::min(2048, (KMr * ((ldS + GI8_CHUNK - 1) / GI8_CHUNK) * 5 + 255) / 256));
  clear_kernel<<<dim3(nb, batch), 256, 0, s>>>(d, rmax_given ? 0 : 1, planes ? 1 : 0);
  if (!rmax_given) {
    const int cy = std::max(1, std::min(64, max_k / 256));
    rowmax_kernel<ST><<<dim3((KMr + 255) / 256, cy, batch), 256, 0, s>>>(d);
  }
  if (planes)
    slice_kernel<ST><<<dim3((ldS + SL_COLS * SL_SUB - 1) / (SL_COLS * SL_SUB), KMr / 64, batch), 256, 0, s>>>(d);
}

}  // namespace

size_t gram_i8_workspace(int m, int k) {
  const size_t KMr = (size_t)round_up_i(m, 64), ldS = (size_t)round_up_i(std::max(k, 1), GLD);
  const size_t nch = (ldS + GI8_CHUNK - 1) / GI8_CHUNK;
  return 8 * KMr * ldS + 8 * KMr + 4 * 4 * KMr * nch + 256;
}

void gram_i8_layout(GramI8Desc& d, void* base) {
  d.KMr = round_up_i(d.m, 64);
  d.ldS = round_up_i(std::max(d.k, 1), GLD);
  char* p = static_cast<char*>(base);
  d.S = reinterpret_cast<int8_t*>(p);
  p += 8 * (size_t)d.KMr * d.ldS;
  d.rmax = reinterpret_cast<unsigned long long*>(p);
  p += 8 * (size_t)d.KMr;
  d.rs = reinterpret_cast<int*>(p);
}

static void prep_dispatch(const GramI8Desc* d_desc, int batch, int max_m, int max_k, int st,
                          bool rmax_given, bool planes, hipStream_t s) {
  if (batch <= 0 || max_m <= 0) return;
  const int KMr = round_up_i(max_m, 64), ldS = round_up_i(std::max(max_k, 1), GLD);
  switch (st) {
    case ST_FP32: launch_prep<ST_FP32>(d_desc, batch, KMr, ldS, max_k, rmax_given, planes, s); break;
    case ST_FP16P: launch_prep<ST_FP16P>(d_desc, batch, KMr, ldS, max_k, rmax_given, planes, s); break;
    case ST_BF16P: launch_prep<ST_BF16P>(d_desc, batch, KMr, ldS, max_k, rmax_given, planes, s); break;
    case ST_MF: launch_prep<ST_MF>(d_desc, batch, KMr, ldS, max_k, rmax_given, planes, s); break;
    default: return;
  }
}

void gram_i8_prepare(const GramI8Desc* d_desc, int batch, int max_m, int max_k, int st,
                     bool rmax_given, hipStream_t s) {
  prep_dispatch(d_desc, batch, max_m, max_k, st, rmax_given, true, s);
}

void gram_i8_rowmax(const GramI8Desc* d_desc, int batch, int max_m, int max_k, int st, hipStream_t s) {
  prep_dispatch(d_desc, batch, max_m, max_k, st, false, false, s);
}

int gram_i8_chunks(int max_k) {
  return (round_up_i(std::max(max_k, 1), GLD) + GI8_CHUNK - 1) / GI8_CHUNK;
}

void gram_i8_chunk(const GramI8Desc* d_desc, int batch, int chunk, const int2* tiles, int ntiles,
                   bool wide, hipStream_t s) {
  if (batch <= 0 || ntiles <= 0) return;
  if (wide)
    gram_i8_32_kernel<<<dim3(8 * ((ntiles + 7) / 8), batch), G32_THREADS, 0, s>>>(d_desc, chunk, tiles, ntiles);
  else
    gram_i8_kernel<<<dim3(8 * ((ntiles + 7) / 8), batch), GTHREADS, 0, s>>>(d_desc, chunk, tiles, ntiles);
}
