// Host engine and C ABI of the sharing-ADMM radar imager (see include/sadmm.h).
//
// Layout in HBM (per handle; KMp = K*M rounded up to 32, rows beyond K*M zero):
//   Afull[q]  operator A_q, column-major, one column per pixel, storage format
//             per sadmm_storage (ldA slots per column)
//   Ahat[q]   active columns of A_q in ascending pixel order (the compacted
//             A_q P_q^T of eq. (3)); aliases Afull[q] while every pixel is active
//   W64[q]    ((c/mu) I + Ahat Ahat^H)^{-1}, complex128 KMp x KMp, applied every
//             iteration in FP64 (see the W product in iter.hip)
//   X, dX     Q x N compute-precision complex, sensor-major
//   xbar,z,u  N complex;  D  Kp x Q x N ring of |x^(i) - x^(i-1)|
//   y, yp     Q x KMp complex128 measurements and y' (frozen pixels removed)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/sadmm.h"
#include "gram.h"
#include "iter.h"
#include "linalg.h"
#include "util.h"

// provided by cnn.hip
int sadmm_cnn_prob_from_mf(sadmm_cnn_t c, const double* mf_dev, const float** prob_dev);
hipStream_t sadmm_cnn_stream(sadmm_cnn_t c);
int sadmm_cnn_shape(sadmm_cnn_t c, int* Q, int* H, int* W);

namespace {

constexpr int KKT_ROUNDS = 8;
thread_local std::string g_create_err;   // message of the last failed sadmm_create

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct sadmm_s {
  sadmm_params p{};
  int Q = 0, K = 0, M = 0, KM = 0, KMp = 0, N = 0;
  int st = ST_FP32;
  bool dbl = false;
  size_t csz = 8;        // bytes per compute-precision complex
  int64_t ldA = 0;       // slots per operator column
  size_t slot = 8;       // bytes per slot
  hipStream_t s = nullptr;
  std::string err;
  std::vector<void*> allocs;

  std::vector<void*> Afull, Ahat_buf, W, Wc;   // Wc: compute-precision W
  std::vector<cd*> W64;
  std::vector<int*> J, Jnew;
  std::vector<void*> xy;                      // Ahat^H W y' per sensor (compute precision)
  std::vector<int> nq;
  std::vector<bool> op_set, fac_valid;
  std::vector<std::vector<int>> facJ;          // active set the factor was built for
  std::vector<std::vector<uint8_t>> mask0;     // caller's initial selectors

  void *X = nullptr, *dX = nullptr, *xbar = nullptr, *z = nullptr, *u = nullptr, *D = nullptr;
  void *tpart = nullptr, *t = nullptr, *w = nullptr, *gtmp = nullptr, *xref = nullptr;
  double *y = nullptr, *yp = nullptr, *e = nullptr, *red = nullptr, *hist = nullptr, *wy = nullptr;
  double* mf = nullptr;
  uint8_t *mask = nullptr, *keep = nullptr, *flag = nullptr, *ones = nullptr;
  int *gone = nullptr, *fail = nullptr, *counts = nullptr, *lst = nullptr, *lst2 = nullptr;
  Ctl* ctl = nullptr;
  Ctl* ctl_h = nullptr;      // pinned mirror
  int* counts_h = nullptr;   // pinned
  int* halt_h = nullptr;     // pinned
  SensorDesc* sens_d = nullptr;
  std::vector<SensorDesc> sens_h;
  GemmDesc* gemm_d = nullptr;
  HpdDesc* hpd_d = nullptr;
  // direct form (mu Ahat^H Ahat + cI)^{-1} for small active sets
  std::vector<uint8_t> direct;   // per sensor
  std::vector<cd*> Fd, b0d, rdir;
  std::vector<int> fld;
  int dir_cap = 0;               // order the direct buffers hold (0: none yet)
  cd *A64 = nullptr, *dirD = nullptr, *dirX = nullptr, *dirT = nullptr;
  MmDesc* dir_desc = nullptr;    // 2 products
  // correction of 16-bit storage toward the accurate (regenerated) operator
  std::vector<double*> rec;      // per sensor: phase records of the geometry, or null
  SensorDesc* sens_mf_d = nullptr;   // sensor table viewing rec as a matrix-free operator
  double *gfix = nullptr, *re1 = nullptr, *re2 = nullptr, *rw = nullptr;
  double *gprev = nullptr, *dg = nullptr;   // previous correction, per-sensor squared changes
  double* dg_h = nullptr;                   // pinned host copy of dg
  void *g32 = nullptr, *xfix = nullptr, *xprev = nullptr;
  int k_refined = 0;             // iteration of the last correction
  double shift = 0.0;            // x-update move caused by the last correction
  bool settled = false;          // that move was within the settling tolerance
  int k_jump = 0;                // iteration of the last correction that did not settle
  // W not formed after a build (W64 holds U = X^H, hpdX holds X = L^{-1})
  std::vector<uint8_t> wtri;
  double* ws = nullptr;          // Q x KMp complex128: X v of the triangular products
  sadmm_t shared_src = nullptr;  // operator and factor borrowed from this handle
  int n_sharers = 0;             // handles borrowing this one's operator
  GramI8Desc* gi8_d = nullptr;   // integer Gram descriptors (Q)
  std::vector<unsigned long long*> rmaxc;   // per sensor: row maxima of the full operator
  int2* tiles_d = nullptr;       // Gram tile order (tri_tile_order)
  int ntiles = 0;
  int dev = 0;                   // device the handle was created on
  cd *Ar = nullptr, *V = nullptr, *Tm = nullptr, *Cm = nullptr, *Dg = nullptr, *Xg = nullptr,
     *Tg = nullptr;
  MmDesc* mm_d = nullptr;     // GEMM descriptors of the factorisations
  std::vector<cd*> hpdD, hpdX, hpdT;          // per-sensor inverse scratch
  int rmax = 0, rpad_max = 0;
  int chunk = 256, nchunk = 0, nblk = 0;
  int chunk_min = 256;            // narrowest forward tile this handle may take
  int nchunk_cap = 0;             // chunks the forward buffers hold (at chunk_min)
  double xref_norm2 = 0.0, nmse_target = 0.0;
  bool have_ref = false;
  sadmm_cnn_t cnn = nullptr;
  double cnn_thr = 0.5;
  int cnn_pruned = 0;            // pixels the CNN eliminated at the last solve

  // results of the last solve
  sadmm_info info{};
  std::vector<double> hist_h;   // 9 x max_iter
  int hist_count = 0;
  double t_total = 0, t_factor = 0, t_iter = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evf0 = nullptr, evf1 = nullptr;
  bool solved = false;

  // iteration-loop resources: argument table and slot table of this handle
  // as a batch of one, its own stream for graph capture, the cached graph
  IterArgs* args_d = nullptr;
  int2* slots_d = nullptr;
  hipStream_t gs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // per-solve loop state
  std::vector<std::pair<int, double>> frac_pts;   // (iteration, max active fraction from it on)
  std::vector<std::pair<int, double>> beta_pts;   // (iteration, beta in force after it)
  double beta0 = 1.0;              // the beta of the parameters (balancing changes p.beta in a solve)
  double* kg = nullptr;             // optimality re-check: gradients of one sensor's eliminated pixels
  bool args_dirty = false;         // the device copy of the iteration arguments is stale
  int kkt_rounds = 0, status = 1;
  bool done = false;
  bool start_restricted = false;   // the solve started with eliminated pixels
  double last_dg = 0.0;            // x-update change of the last correction retake
  std::vector<std::pair<int, double>> retake_pts;   // (iteration, that change) per retake
  std::vector<std::pair<int, double>> shift_pts;    // (iteration, x-update move) per correction

  // optional per-kernel-class event timing (sadmm_set_profiling)
  bool prof = false;
  int prof_level = 0;
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  std::vector<std::array<int, 3>> marks;       // (class, start event, end event)
  double kt_ms[SADMM_KC_COUNT] = {0};
  int kt_n[SADMM_KC_COUNT] = {0};
  double kt_work[SADMM_KC_COUNT] = {0};       // algorithmic flops or bytes
};

namespace {

int fail_msg(sadmm_t h, int code, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return code;
}

#define HIPCHK(h, call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail_msg(h, SADMM_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
  } while (0)

#define TRY(x)              \
  do {                      \
    int rc_ = (x);          \
    if (rc_ != SADMM_OK) return rc_; \
  } while (0)

int dalloc(sadmm_t h, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    fail_msg(h, SADMM_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    g_create_err = h->err;
    return SADMM_E_NOMEM;
  }
  h->allocs.push_back(*p);
  return SADMM_OK;
}
template <class P> int dalloc_t(sadmm_t h, P** p, size_t bytes) {
  void* v = nullptr;
  int rc = dalloc(h, &v, bytes);
  *p = static_cast<P*>(v);
  return rc;
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ---- per-kernel-class timing: events recorded around launches on the
// handle's stream when profiling is on; resolved after the stream syncs.
int prof_begin(sadmm_t h) {
  if (!h->prof) return -1;
  if (h->evnext + 2 > h->evpool.size()) return -1;
  const int e = (int)h->evnext;
  h->evnext += 2;
  hipEventRecord(h->evpool[e], h->s);
  return e;
}
void prof_end(sadmm_t h, int cls, int e) {
  if (e < 0) return;
  hipEventRecord(h->evpool[e + 1], h->s);
  h->marks.push_back({cls, e, e + 1});
}
void prof_work(sadmm_t h, int cls, double w) {
  if (h->prof) h->kt_work[cls] += w;
}
// bytes per stored complex operator entry
double op_bytes(sadmm_t h) {
  if (h->st == ST_MF) return 8.0 * (MF_REC_BASE + MF_REC_PER_RX * h->M) / h->KM;   // record bytes per entry
  return h->st == ST_FP64 ? 16.0 : (h->st == ST_FP32 ? 8.0 : 4.0);
}

void prof_resolve(sadmm_t h) {
  if (h->marks.empty()) { h->evnext = 0; return; }
  hipEventSynchronize(h->evpool[h->marks.back()[2]]);
  for (auto& m : h->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->evpool[m[1]], h->evpool[m[2]]) == hipSuccess) {
      h->kt_ms[m[0]] += ms;
      h->kt_n[m[0]] += 1;
    }
  }
  h->marks.clear();
  h->evnext = 0;
}

// Forward-product tile width (columns per work-group) chosen by
// sadmm_autotune, per (storage, rows rounded to 32, pixel-count bucket); a
// handle created later for the same key starts from it.
constexpr int FWD_CHUNKS[] = {64, 128, 256, 512, 1024};
static_assert(FWD_CHUNKS[4] <= MAX_CHUNK, "forward tile wider than its LDS coefficient tile");
// Narrowest tile: images below 4096 pixels (every pixel-count bucket below
// 2^12) take tiles from 64 columns, so that their few rows still spread over
// enough work-groups; larger ones from 256 (their partial-sum buffers stay
// within Q * N / 256 * KMp entries).
int fwd_chunk_min(int N) { return N < 4096 ? 64 : 256; }
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tuned;
int n_bucket(int N) {   // power-of-two bucket of the pixel count
  int b = 0;
  while ((1 << (b + 1)) <= N) ++b;
  return b;
}
int tuned_chunk(int st, int KMp, int N) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(std::make_tuple(st, KMp, n_bucket(N)));
  return it == g_tuned.end() ? 0 : it->second;
}
void set_tuned_chunk(int st, int KMp, int N, int chunk) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[std::make_tuple(st, KMp, n_bucket(N))] = chunk;
}

IterArgs make_args(sadmm_t h) {
  IterArgs a{};
  a.Q = h->Q; a.KMp = h->KMp; a.N = h->N; a.Kp = h->p.Kp;
  a.chunk = h->chunk; a.nchunk = h->nchunk;
  a.prune = h->p.prune; a.stop = h->p.stop;
  a.beta = h->p.beta;
  a.c = h->p.beta + h->p.gamma;
  a.bc = a.beta / a.c;
  a.tau = h->p.lambda / h->p.beta;
  a.nonneg = h->p.nonneg;
  a.bal_every = h->p.balance_every;
  a.bal_mu = h->p.balance_mu;
  a.eps_abs = h->p.eps_abs; a.eps_rel = h->p.eps_rel; a.eps_p = h->p.eps_p;
  a.inv_Q = 1.0 / h->Q;
  a.nmse_target = h->nmse_target;
  a.xref_norm2 = h->xref_norm2;
  a.sens = h->sens_d;
  a.X = h->X; a.dX = h->dX; a.xbar = h->xbar; a.z = h->z; a.u = h->u; a.D = h->D;
  a.tpart = h->tpart; a.t = h->t; a.w = h->w;
  a.xref = h->have_ref ? h->xref : nullptr;
  a.yp = h->yp;
  a.wy = h->wy;
  a.red = h->red; a.nblk = h->nblk;
  a.max_iter = h->p.max_iter;
  a.ctl = h->ctl; a.hist = h->hist;
  a.keep = h->keep; a.gone = h->gone;
  a.ws = h->ws;
  a.gfix = h->p.refine_every > 0 ? h->gfix : nullptr;
  a.xfix = h->p.refine_every > 0 ? h->xfix : nullptr;
  // With the correction of a 16-bit operator, SSC judges only iterates of
  // the corrected problem once that problem has settled: the latest
  // correction moved the x-update by at most the settling tolerance, and the
  // K_p-window starts after the last correction that moved it by more
  // (its x jumps).  Pixels frozen while the correction still moves keep
  // values of a fixed point that is not the final one, and the consensus
  // then reaches the tolerance only as slowly as the dual absorbs the
  // difference.
  a.ssc_from = h->p.refine_every <= 0 ? 0
               : (h->settled ? h->k_jump + h->p.Kp + 1 : std::numeric_limits<int>::max());
  // Operator and factor bytes one iteration reads: above half of the 256 MB
  // last-level cache nothing is found again at the next pass, and the
  // products stream them with non-temporal loads (c2 FP32: 841 -> 787 us per
  // iteration); below it (c1: 8 MB) normal loads keep them cached.
  static constexpr double kStreamBytes = 128.0 * (1 << 20);
  double opb = 0.0, wb = 0.0;
  for (int q = 0; q < h->Q; ++q) {
    opb += (double)h->KMp * h->nq[q] * op_bytes(h);
    if (!h->direct[q]) wb += 16.0 * h->KMp * h->KMp;
  }
  a.stream_op = opb > kStreamBytes ? 1 : 0;
  a.stream_w = wb > kStreamBytes ? 1 : 0;
  return a;
}

const void* ahat_ptr(sadmm_t h, int q) {
  return (h->nq[q] == h->N) ? h->Afull[q] : h->Ahat_buf[q];
}

int push_descs(sadmm_t h) {
  for (int q = 0; q < h->Q; ++q) {
    SensorDesc& d = h->sens_h[q];
    d.A = ahat_ptr(h, q);
    d.Afull = h->Afull[q];
    d.J = h->J[q];
    d.xy = h->xy[q];
    d.W = h->W64[q];
    d.W64 = h->W64[q];
    d.lda = h->ldA;
    d.nq = h->nq[q];
    d.direct = h->direct[q];
    d.F = h->Fd[q];
    d.b0 = h->b0d[q];
    d.rdir = h->rdir[q];
    d.fld = h->fld[q];
    d.wtri = h->wtri[q];
    d.X = h->hpdX[q];
  }
  HIPCHK(h, hipMemcpyAsync(h->sens_d, h->sens_h.data(), sizeof(SensorDesc) * h->Q,
                           hipMemcpyHostToDevice, h->s));
  if (h->sens_mf_d) {
    std::vector<SensorDesc> m = h->sens_h;
    for (int q = 0; q < h->Q; ++q) {
      m[q].A = m[q].Afull = h->rec[q];
      m[q].lda = MF_REC_BASE + MF_REC_PER_RX * (int64_t)h->M;
    }
    HIPCHK(h, hipMemcpyAsync(h->sens_mf_d, m.data(), sizeof(SensorDesc) * h->Q,
                             hipMemcpyHostToDevice, h->s));
  }
  HIPCHK(h, hipStreamSynchronize(h->s));
  return SADMM_OK;
}

// Ahat[q] <- Afull[q][:, J[q]] (only when some pixel is inactive)
int compact_operator(sadmm_t h, int q) {
  if (h->nq[q] == h->N) return SADMM_OK;
  if (!h->Ahat_buf[q]) TRY(dalloc(h, &h->Ahat_buf[q], (size_t)h->ldA * h->slot * h->N));
  gather_columns(h->Afull[q], h->Ahat_buf[q], h->ldA, (int64_t)h->slot, h->J[q], h->nq[q], h->s);
  return SADMM_OK;
}

int check_fail(sadmm_t h) {
  int f = 0;
  HIPCHK(h, hipMemcpyAsync(&f, h->fail, sizeof(int), hipMemcpyDeviceToHost, h->s));
  HIPCHK(h, hipStreamSynchronize(h->s));
  if (f) {
    HIPCHK(h, hipMemsetAsync(h->fail, 0, sizeof(int), h->s));
    return fail_msg(h, SADMM_E_NUMERIC, "factor lost positive definiteness");
  }
  return SADMM_OK;
}

// One factor to build: sensor q of handle h.
struct FacItem {
  sadmm_t h;
  int q;
};

double factor_rho(sadmm_t h) { return (h->p.beta + h->p.gamma) / h->p.mu; }
bool integer_gram(sadmm_t h) { return (h->p.gram == 0 || h->p.gram == 2) && h->st != ST_FP64; }

// Device table of `need` descriptors: h0's own when it is large enough, else a
// temporary one (freed by the caller through tmp after the stream syncs).
template <class T>
int desc_table(sadmm_t h0, T* own, size_t own_cap, size_t need, std::vector<void*>& tmp, T** out) {
  if (need <= own_cap) { *out = own; return SADMM_OK; }
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * need) != hipSuccess)
    return fail_msg(h0, SADMM_E_NOMEM, "factor build: descriptor table");
  tmp.push_back(p);
  *out = static_cast<T*>(p);
  return SADMM_OK;
}

// Digit-plane workspace of the integer Gram: one per device, shared by every
// handle on it (a build needs it only while its Gram kernels run).  Builds
// order themselves by an event: a build's stream waits for the previous
// user's last Gram kernel before its own touch the buffer, and records the
// event after them; growing the buffer waits for it to go idle first.
struct GramWorkspace {
  void* p = nullptr;
  size_t bytes = 0;
  hipEvent_t last = nullptr;      // after the latest user's kernels
  bool used = false;
};
std::mutex g_gws_mu;
std::map<int, GramWorkspace> g_gws;

// W64 = Ahat Ahat^H + rho I by the integer digit products (gram.h) for the
// items, in groups whose digit planes fit a bounded workspace.
int gram_integer(sadmm_t h0, const std::vector<FacItem>& items, std::vector<void*>& tmp) {
  constexpr size_t kCap = size_t(4) << 30;
  int max_n = 0;
  for (const FacItem& it : items) max_n = std::max(max_n, it.h->N);
  const size_t per = (gram_i8_workspace(h0->KMp, max_n) + 255) / 256 * 256;
  const size_t group = std::max<size_t>(1, std::min<size_t>(items.size(), kCap / per));
  std::lock_guard<std::mutex> lock(g_gws_mu);     // held while this factor build's kernels are queued
  GramWorkspace& ws = g_gws[h0->dev];
  if (!ws.last && hipEventCreateWithFlags(&ws.last, hipEventDisableTiming) != hipSuccess) {
    ws.last = nullptr;
    return fail_msg(h0, SADMM_E_HIP, "integer Gram workspace: event creation");
  }
  if (ws.bytes < group * per) {
    if (ws.p) {
      if (ws.used) HIPCHK(h0, hipEventSynchronize(ws.last));
      hipFree(ws.p);
    }
    ws.p = nullptr;
    ws.bytes = 0;
    ws.used = false;
    const hipError_t e = hipMalloc(&ws.p, group * per);
    if (e != hipSuccess) {
      ws.p = nullptr;
      return fail_msg(h0, SADMM_E_NOMEM, "integer Gram workspace (%zu bytes): %s", group * per,
                      hipGetErrorString(e));
    }
    ws.bytes = group * per;
  } else if (ws.used) {
    HIPCHK(h0, hipStreamWaitEvent(h0->s, ws.last, 0));
  }
  GramI8Desc* dd = nullptr;
  TRY(desc_table(h0, h0->gi8_d, (size_t)h0->Q, group, tmp, &dd));
  for (size_t g0 = 0; g0 < items.size(); g0 += group) {
    const size_t n = std::min(group, items.size() - g0);
    std::vector<GramI8Desc> gd(n);
    int max_k = 0;
    // the row maxima of the full operators (computed when they were set) bound
    // those of the compacted ones
    bool given = true;
    for (size_t i = 0; i < n; ++i) {
      const sadmm_t h = items[g0 + i].h;
      const int q = items[g0 + i].q;
      given = given && q < (int)h->rmaxc.size() && h->rmaxc[q];
    }
    for (size_t i = 0; i < n; ++i) {
      const sadmm_t h = items[g0 + i].h;
      const int q = items[g0 + i].q;
      GramI8Desc& d = gd[i];
      d.A = ahat_ptr(h, q); d.ldA = h->ldA; d.kmp = h->KMp;
      d.m = h->KMp; d.k = h->nq[q];
      d.C = h->W64[q]; d.ldc = h->KMp; d.diag = factor_rho(h);
      gram_i8_layout(d, static_cast<char*>(ws.p) + i * per);
      if (given) d.rmax = h->rmaxc[q];
      max_k = std::max(max_k, d.k);
      prof_work(h0, SADMM_KC_SLICE, (double)h->nq[q] * h->KMp * (op_bytes(h) + 8.0));
    }
    // (stream order keeps a later group's upload behind the kernels reading this one)
    HIPCHK(h0, hipMemcpyAsync(dd, gd.data(), sizeof(GramI8Desc) * n, hipMemcpyHostToDevice, h0->s));
    int pe = prof_begin(h0);
    gram_i8_prepare(dd, (int)n, h0->KMp, max_k, h0->st, given, h0->s);
    prof_end(h0, SADMM_KC_SLICE, pe);
    for (int c = 0; c < gram_i8_chunks(max_k); ++c) {
      pe = prof_begin(h0);
      gram_i8_chunk(dd, (int)n, c, h0->tiles_d, h0->ntiles, h0->p.gram == 2, h0->s);
      prof_end(h0, SADMM_KC_GRAM, pe);
    }
    HIPCHK(h0, hipGetLastError());
  }
  HIPCHK(h0, hipEventRecord(ws.last, h0->s));
  ws.used = true;
  return SADMM_OK;
}

// Row maxima of sensor q's full operator for the integer Gram (FP32, 16-bit
// and matrix-free storage), once per operator.
int cache_rowmax(sadmm_t h, int q) {
  if (!integer_gram(h) || h->shared_src) return SADMM_OK;
  const int KMr = round_up(h->KMp, 64);
  if ((int)h->rmaxc.size() < h->Q) h->rmaxc.assign(h->Q, nullptr);
  if (!h->rmaxc[q] && hipMalloc((void**)&h->rmaxc[q], sizeof(unsigned long long) * KMr) != hipSuccess) {
    h->rmaxc[q] = nullptr;
    return fail_msg(h, SADMM_E_NOMEM, "row maxima");
  }
  GramI8Desc d{};
  d.A = h->Afull[q]; d.ldA = h->ldA; d.kmp = h->KMp;
  d.m = h->KMp; d.k = h->N;
  d.KMr = KMr; d.ldS = round_up(h->N, 128);
  d.rmax = h->rmaxc[q];
  HIPCHK(h, hipMemcpyAsync(h->gi8_d, &d, sizeof d, hipMemcpyHostToDevice, h->s));
  gram_i8_rowmax(h->gi8_d, 1, h->KMp, h->N, h->st, h->s);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->s));
  return SADMM_OK;
}

// Full factor build W64 = ((c/mu) I + Ahat Ahat^H)^{-1} of the items, which
// share KMp, storage and Gram path; runs on h0's stream.  Used for the sensors
// of one handle, and by sadmm_solve_batch for the sensors of every handle at
// once (one Gram and one inverse chain for the whole batch).
int build_factors_items(sadmm_t h0, const std::vector<FacItem>& items) {
  if (items.empty()) return SADMM_OK;
  const size_t n = items.size();
  std::vector<void*> tmp;
  auto cleanup = [&]() {
    if (!tmp.empty()) hipStreamSynchronize(h0->s);
    for (void* p : tmp) hipFree(p);
  };
  std::vector<GemmDesc> gd(n);
  std::vector<HpdDesc> hd(n);
  for (size_t i = 0; i < n; ++i) {
    const sadmm_t h = items[i].h;
    const int q = items[i].q;
    GemmDesc& g = gd[i];
    g.A = ahat_ptr(h, q); g.B = ahat_ptr(h, q); g.C = h->W64[q];
    g.m = h->KMp; g.n = h->KMp; g.k = h->nq[q];
    g.kmpA = h->KMp; g.kmpB = h->KMp;
    g.lda = h->ldA; g.ldb = h->ldA; g.ldc = h->KMp;
    g.alpha_re = 1.0; g.alpha_im = 0.0; g.beta = 0.0; g.diag = factor_rho(h);
    hd[i] = HpdDesc{h->W64[q], h->KMp, h->hpdD[q], h->hpdX[q], h->hpdT[q]};
    // Hermitian product: KM(KM+1)/2 entries, N_q complex MACs each (8 flops)
    prof_work(h0, SADMM_KC_GRAM, 8.0 * 0.5 * h->KM * (h->KM + 1.0) * h->nq[q]);
  }
  // W = X^H X is left unformed (the iterations apply X^H (X v)) unless an
  // item's operator is shared: multi-right-hand-side products read W itself.
  bool form_w = false;
  for (const FacItem& it : items) form_w = form_w || it.h->shared_src || it.h->n_sharers > 0;
  for (const FacItem& it : items) {
    const double km = it.h->KM;
    // Cholesky n^3/3, triangular inverse n^3/6 (+ X^H X n^3/3) complex MACs
    prof_work(h0, SADMM_KC_INVERSE, 8.0 * (form_w ? 5.0 / 6.0 : 0.5) * km * km * km);
  }
  int rc = SADMM_OK;
  HpdDesc* hpd = nullptr;
  MmDesc* mm = nullptr;
  GemmDesc* gemm = nullptr;
  const size_t mm_need = n * hpd_mm_count(h0->KMp);
  const size_t mm_own = std::max((size_t)h0->Q * hpd_mm_count(h0->KMp), hpd_mm_count(h0->rpad_max));
  if ((rc = desc_table(h0, h0->hpd_d, (size_t)h0->Q, n, tmp, &hpd)) != SADMM_OK ||
      (rc = desc_table(h0, h0->mm_d, mm_own, mm_need, tmp, &mm)) != SADMM_OK ||
      (rc = desc_table(h0, h0->gemm_d, (size_t)std::max(h0->Q, 4), n, tmp, &gemm)) != SADMM_OK) {
    cleanup();
    return rc;
  }
  if (hipMemcpyAsync(hpd, hd.data(), sizeof(HpdDesc) * n, hipMemcpyHostToDevice, h0->s) != hipSuccess) {
    cleanup();
    return fail_msg(h0, SADMM_E_HIP, "factor build: descriptor upload");
  }
  if (integer_gram(h0)) {
    rc = gram_integer(h0, items, tmp);
  } else {
    if (hipMemcpyAsync(gemm, gd.data(), sizeof(GemmDesc) * n, hipMemcpyHostToDevice, h0->s) != hipSuccess)
      rc = fail_msg(h0, SADMM_E_HIP, "factor build: descriptor upload");
    const int pe = prof_begin(h0);
    if (rc == SADMM_OK) herk_batched(gemm, (int)n, h0->KMp, h0->st, h0->tiles_d, h0->ntiles, h0->s);
    prof_end(h0, SADMM_KC_GRAM, pe);
  }
  if (rc == SADMM_OK) {
    const int pe = prof_begin(h0);
    hpd_inverse_batched(hd.data(), hpd, (int)n, h0->KMp, h0->fail, mm, h0->s, form_w);
    prof_end(h0, SADMM_KC_INVERSE, pe);
    if (hipGetLastError() != hipSuccess) rc = fail_msg(h0, SADMM_E_HIP, "factor build: launch failed");
  }
  if (rc == SADMM_OK) rc = check_fail(h0);   // synchronises h0's stream
  cleanup();
  if (rc != SADMM_OK) return rc;
  std::vector<sadmm_t> touched;
  for (const FacItem& it : items) {
    it.h->fac_valid[it.q] = true;
    it.h->wtri[it.q] = form_w ? 0 : 1;
    if (std::find(touched.begin(), touched.end(), it.h) == touched.end()) touched.push_back(it.h);
  }
  for (sadmm_t h : touched) TRY(push_descs(h));
  return SADMM_OK;
}

// W64 = X^H X for a sensor whose factor was left as X (wtri), for the
// consumers that need W itself (low-rank updates, shared operators, the
// correction's W v, get_factor).
int ensure_w(sadmm_t h, int q) {
  if (!h->wtri[q]) return SADMM_OK;
  const int n = h->KMp;
  const MmDesc d{h->hpdX[q], h->hpdX[q], h->W64[q], n, n, n, n, n, n, 1.0, 0.0, 0.0};
  HIPCHK(h, hipMemcpyAsync(h->mm_d, &d, sizeof d, hipMemcpyHostToDevice, h->s));
  hpd_form_w(h->mm_d, 1, n, h->s);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->s));
  h->wtri[q] = 0;
  return push_descs(h);
}

int build_factors(sadmm_t h, const std::vector<int>& qs) {
  std::vector<FacItem> items;
  for (int q : qs) items.push_back({h, q});
  return build_factors_items(h, items);
}

// Low-rank correction of W64[q] for r columns (pixel list lst) leaving
// (sign = -1: removal) or joining (sign = +1: reinstatement) Ahat:
//   G' = G + sign * Ar Ar^H,
//   W' = W - sign * W Ar (I + sign * Ar^H W Ar)^{-1} Ar^H W.
int lowrank_update(sadmm_t h, int q, const int* d_list, int r, int sign) {
  TRY(ensure_w(h, q));
  const int KMp = h->KMp;
  const int rp = round_up(r, HPD_NB);
  gather_columns_fp64(h->Afull[q], h->ldA, h->st, KMp, d_list, r, h->Ar, h->s);
  std::array<GemmDesc, 4> g;
  // V = W Ar
  g[0] = GemmDesc{h->W64[q], h->Ar, h->V, KMp, r, KMp, KMp, KMp, KMp, KMp, KMp, 1.0, 0.0, 0.0, 0.0};
  // Cm = I + sign * Ar^H V   (identity-padded to rp)
  g[1] = GemmDesc{h->Ar, h->V, h->Cm, r, r, KMp, KMp, KMp, KMp, KMp, rp, (double)sign, 0.0, 1.0, 0.0};
  // Tm = V Cm^{-1}
  g[2] = GemmDesc{h->V, h->Cm, h->Tm, KMp, r, r, KMp, KMp, KMp, rp, KMp, 1.0, 0.0, 0.0, 0.0};
  // W += -sign * Tm V^H
  g[3] = GemmDesc{h->Tm, h->V, h->W64[q], KMp, KMp, r, KMp, KMp, KMp, KMp, KMp, -(double)sign, 0.0, 1.0, 0.0};
  HpdDesc hd{h->Cm, rp, h->Dg, h->Xg, h->Tg};
  HIPCHK(h, hipMemcpyAsync(h->gemm_d, g.data(), sizeof(GemmDesc) * 4, hipMemcpyHostToDevice, h->s));
  HIPCHK(h, hipMemcpyAsync(h->hpd_d, &hd, sizeof hd, hipMemcpyHostToDevice, h->s));
  zgemm_batched(h->gemm_d, 1, KMp, r, ST_FP64, ST_FP64, OP_N, OP_N, false, h->s);
  HIPCHK(h, hipMemsetAsync(h->Cm, 0, sizeof(cd) * (size_t)rp * rp, h->s));
  set_identity_pad(h->Cm, 0, rp, 0.0, h->s);
  zgemm_batched(h->gemm_d + 1, 1, r, r, ST_FP64, ST_FP64, OP_C, OP_N, false, h->s);
  hpd_inverse_batched(&hd, h->hpd_d, 1, rp, h->fail, h->mm_d, h->s);
  zgemm_batched(h->gemm_d + 2, 1, KMp, r, ST_FP64, ST_FP64, OP_N, OP_N, false, h->s);
  zgemm_batched(h->gemm_d + 3, 1, KMp, KMp, ST_FP64, ST_FP64, OP_N, OP_C, false, h->s);
  hermitian_inplace(h->W64[q], KMp, KMp, h->s);
  HIPCHK(h, hipGetLastError());
  h->info.updates += 1;
  return check_fail(h);
}

// Is a rank-r correction cheaper than rebuilding the factor for nq_new columns?
bool prefer_lowrank(sadmm_t h, int r, int nq_new) {
  if (r > h->rmax) return false;
  const double K2 = (double)h->KMp * h->KMp;
  const double upd = 2.0 * K2 * r + (double)r * r * r;
  const double full = 0.5 * K2 * nq_new + (double)h->KMp * K2;
  return upd < full;
}

// Direct form: largest active set for which x = F (b0 + beta v) reads fewer
// bytes per iteration than the Woodbury form (16 N^2 for F against
// 2 KM N b_A + 16 KM^2 for the operator passes and W).
int direct_threshold(sadmm_t h) {
  double f;
  switch (h->st) {
    case ST_FP64: f = 1.0 + std::sqrt(2.0); break;            // b_A = 16
    case ST_FP32: f = 0.5 * (1.0 + std::sqrt(5.0)); break;    // b_A = 8
    case ST_MF: f = 1.0; break;                               // entries recomputed
    default: f = 0.25 + std::sqrt(1.0625); break;             // b_A = 4
  }
  return (int)(f * h->KM);
}
// Order the direct buffers hold: the threshold rounded to the factor block.
// Fixed per handle (params, storage, KM), so an iteration graph captured
// before any switch already covers it.
int direct_cap(sadmm_t h) {
  return (h->p.direct == 0 && !h->shared_src) ? round_up(direct_threshold(h), HPD_NB) : 0;
}
bool want_direct(sadmm_t h, int nq) {
  return h->p.direct == 0 && !h->shared_src && h->n_sharers == 0 && nq > 0 &&
         nq <= direct_threshold(h);
}

// Buffers of the direct form, sized once for the largest order it can take.
int ensure_direct_buffers(sadmm_t h, int q) {
  const int cap = direct_cap(h);
  auto grab = [&](void** p, size_t bytes) -> int {
    if (*p) return SADMM_OK;
    if (hipMalloc(p, bytes) != hipSuccess) {
      *p = nullptr;
      return fail_msg(h, SADMM_E_NOMEM, "direct form: %zu bytes", bytes);
    }
    return SADMM_OK;
  };
  const size_t c2 = (size_t)cap * cap;
  TRY(grab((void**)&h->A64, sizeof(cd) * (size_t)h->KMp * cap));
  TRY(grab((void**)&h->dirD, sizeof(cd) * (size_t)HPD_NB * cap));
  TRY(grab((void**)&h->dirX, sizeof(cd) * c2));
  TRY(grab((void**)&h->dirT, sizeof(cd) * (c2 / 4 + 1)));
  TRY(grab((void**)&h->dir_desc, sizeof(MmDesc) * 2));
  TRY(grab((void**)&h->Fd[q], sizeof(cd) * c2));
  TRY(grab((void**)&h->b0d[q], sizeof(cd) * cap));
  TRY(grab((void**)&h->rdir[q], sizeof(cd) * cap));
  h->dir_cap = cap;
  return SADMM_OK;
}

// Sensor q to the direct form for its current active set:
// F = (mu Ahat^H Ahat + cI)^{-1} (FP64 Gram on the matrix instructions, the
// Cholesky inverse) and b0 = mu Ahat^H y'.
int build_direct(sadmm_t h, int q, bool count = true) {
  TRY(ensure_direct_buffers(h, q));
  hipStream_t s = h->s;
  const int nq = h->nq[q], KMp = h->KMp;
  const int n = round_up(std::max(nq, 1), HPD_NB);
  const double c = h->p.beta + h->p.gamma, mu = h->p.mu;
  gather_columns_fp64(h->Afull[q], h->ldA, h->st, KMp, h->J[q], nq, h->A64, s);
  MmDesc g[2];
  g[0] = MmDesc{h->A64, h->A64, h->Fd[q], nq, nq, KMp, KMp, KMp, n, mu, 0.0, 0.0};
  g[1] = MmDesc{h->A64, reinterpret_cast<const cd*>(h->yp) + (size_t)q * KMp, h->b0d[q], nq, 1, KMp,
                KMp, KMp, n, mu, 0.0, 0.0};
  HIPCHK(h, hipMemcpyAsync(h->dir_desc, g, sizeof g, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemsetAsync(h->Fd[q], 0, sizeof(cd) * (size_t)n * n, s));
  zgemm_mfma_gram_cn(h->dir_desc, 1, nq, s);                   // lower + mirror
  set_identity_pad(h->Fd[q], nq, n, c, s);                     // + cI, identity padding
  zgemm_mfma_cn(h->dir_desc + 1, 1, nq, 1, s);                 // b0
  HpdDesc hd{h->Fd[q], n, h->dirD, h->dirX, h->dirT};
  std::vector<void*> tmp;
  MmDesc* mm = nullptr;
  const size_t own = std::max((size_t)h->Q * hpd_mm_count(KMp), hpd_mm_count(h->rpad_max));
  TRY(desc_table(h, h->mm_d, own, hpd_mm_count(n), tmp, &mm));
  HIPCHK(h, hipMemcpyAsync(h->hpd_d, &hd, sizeof hd, hipMemcpyHostToDevice, s));
  hpd_inverse_batched(&hd, h->hpd_d, 1, n, h->fail, mm, s);
  HIPCHK(h, hipGetLastError());
  const int rc = check_fail(h);   // synchronises
  for (void* p : tmp) hipFree(p);
  TRY(rc);
  h->direct[q] = 1;
  h->fld[q] = n;
  h->fac_valid[q] = false;        // the Woodbury factor no longer matches
  if (count) h->info.refactors += 1;
  return push_descs(h);
}

// Sensor q from the direct form back to the Woodbury form (its active set
// grew past the crossover, or emptied): full factor build and data term.
int to_woodbury(sadmm_t h, int q) {
  h->direct[q] = 0;
  h->info.refactors += 1;
  TRY(build_factors(h, std::vector<int>{q}));
  TRY(push_descs(h));
  h->fac_valid[q] = false;
  launch_xy(make_args(h), h->st, h->dbl, q, q + 1, h->s);
  HIPCHK(h, hipGetLastError());
  return SADMM_OK;
}

int read_counts(sadmm_t h) {
  HIPCHK(h, hipMemcpyAsync(h->counts_h, h->counts, 2 * sizeof(int), hipMemcpyDeviceToHost, h->s));
  HIPCHK(h, hipStreamSynchronize(h->s));
  return SADMM_OK;
}

// Apply the eliminations the SSC check decided at the last iteration.
// Rebuilds the factors of the listed sensors from their current active sets
// in one batched Gram and inverse (one chain of launches for all of them,
// not one per sensor), then their data terms.
int rebuild_factors(sadmm_t h, const std::vector<int>& qs) {
  if (qs.empty()) return SADMM_OK;
  h->info.refactors += (int)qs.size();
  TRY(build_factors(h, qs));
  for (int q : qs) {
    h->fac_valid[q] = false;
    launch_xy(make_args(h), h->st, h->dbl, q, q + 1, h->s);
  }
  HIPCHK(h, hipGetLastError());
  return SADMM_OK;
}

int apply_prune(sadmm_t h) {
  std::vector<int> rebuild;
  std::vector<int> gone(h->Q);
  HIPCHK(h, hipMemcpyAsync(gone.data(), h->gone, sizeof(int) * h->Q, hipMemcpyDeviceToHost, h->s));
  HIPCHK(h, hipStreamSynchronize(h->s));
  const IterArgs a0 = make_args(h);
  for (int q = 0; q < h->Q; ++q) {
    if (gone[q] <= 0) continue;
    const int nq_old = h->nq[q];
    partition_flags(h->keep + (size_t)q * h->N, h->J[q], nq_old, h->Jnew[q], h->lst, h->counts, h->s);
    TRY(read_counts(h));
    const int kept = h->counts_h[0], r = h->counts_h[1];
    if (r != gone[q] || kept != nq_old - r)
      return fail_msg(h, SADMM_E_STATE, "selector compaction mismatch (sensor %d)", q);
    if (h->p.prune_mode == 0) {
      launch_gather_fwd(a0, h->st, h->dbl, q, h->lst, r, -1.0, h->yp + 2 * (size_t)q * h->KMp,
                        h->gtmp, h->s);
    } else {
      zero_complex_at(static_cast<char*>(h->X) + h->csz * (size_t)q * h->N, h->dbl, h->lst, r, h->s);
    }
    set_bytes_at(h->mask + (size_t)q * h->N, h->lst, r, 0, h->s);
    zero_complex_at(static_cast<char*>(h->dX) + h->csz * (size_t)q * h->N, h->dbl, h->lst, r, h->s);
    std::swap(h->J[q], h->Jnew[q]);
    h->nq[q] = kept;
    TRY(compact_operator(h, q));
    TRY(push_descs(h));
    if (want_direct(h, kept)) {
      TRY(build_direct(h, q));
      continue;
    }
    if (h->direct[q]) {   // the active set emptied
      TRY(to_woodbury(h, q));
      continue;
    }
    if (prefer_lowrank(h, r, kept)) {
      TRY(lowrank_update(h, q, h->lst, r, -1));
      h->fac_valid[q] = false;
      launch_xy(make_args(h), h->st, h->dbl, q, q + 1, h->s);
      HIPCHK(h, hipGetLastError());
    } else {
      rebuild.push_back(q);
    }
  }
  TRY(rebuild_factors(h, rebuild));
  HIPCHK(h, hipMemsetAsync(h->gone, 0, sizeof(int) * h->Q, h->s));
  return SADMM_OK;
}

// Optimality re-check of eliminated pixels after convergence; *n_back = the
// number of violating pixels, which are reinstated unless check_only.
// Optimality re-check (solves that start from an initial selector):
// eliminated pixels with |g_qj| > kkt_tol * lambda, g_q = mu A_q^H (A_q x_q -
// y_q) + gamma x_q + beta u, are put back (history window +inf); *n_back =
// their number (only counted when check_only).
int kkt_reinstate(sadmm_t h, int* n_back, bool check_only = false) {
  *n_back = 0;
  std::vector<int> rebuild;
  hipStream_t s = h->s;
  const int N = h->N;
  if (!h->kg && hipMalloc((void**)&h->kg, 16 * (size_t)N) != hipSuccess) {
    h->kg = nullptr;
    return fail_msg(h, SADMM_E_NOMEM, "re-check buffer");
  }
  const double thr = h->p.kkt_tol * (h->p.lambda > 0 ? h->p.lambda : 1.0);
  for (int q = 0; q < h->Q; ++q) {
    if (h->nq[q] == N) continue;
    IterArgs a = make_args(h);
    // e = A_q x_q - y_q over all pixels (original measurement)
    scale_c128(h->y + 2 * (size_t)q * h->KMp, h->e, h->KMp, -1.0, s);
    launch_gather_fwd(a, h->st, h->dbl, q, nullptr, N, 1.0, h->e, h->gtmp, s);
    partition_flags(h->mask + (size_t)q * N, nullptr, N, nullptr, h->lst, h->counts, s);
    TRY(read_counts(h));
    const int ne = h->counts_h[1];
    if (ne == 0) continue;
    launch_kkt_grad(a, h->st, h->dbl, q, h->lst, ne, h->e, h->p.mu, h->p.gamma, h->kg, s);
    grad_flag(h->kg, ne, thr, h->flag, s);
    partition_flags(h->flag, h->lst, ne, h->lst2, nullptr, h->counts, s);
    TRY(read_counts(h));
    const int r = h->counts_h[0];
    if (r == 0) continue;
    if (check_only) { *n_back += r; continue; }
    if (h->p.prune_mode == 0)
      launch_gather_fwd(a, h->st, h->dbl, q, h->lst2, r, 1.0, h->yp + 2 * (size_t)q * h->KMp, h->gtmp, s);
    set_bytes_at(h->mask + (size_t)q * N, h->lst2, r, 1, s);
    set_ring_inf(h->D, h->dbl, h->p.Kp, h->Q, N, q, h->lst2, r, s);
    partition_flags(h->mask + (size_t)q * N, nullptr, N, h->J[q], nullptr, h->counts, s);
    TRY(read_counts(h));
    h->nq[q] = h->counts_h[0];
    TRY(compact_operator(h, q));
    TRY(push_descs(h));
    if (want_direct(h, h->nq[q])) {
      TRY(build_direct(h, q));
    } else if (h->direct[q]) {   // grown past the crossover
      TRY(to_woodbury(h, q));
    } else if (prefer_lowrank(h, r, h->nq[q])) {
      TRY(lowrank_update(h, q, h->lst2, r, +1));
      h->fac_valid[q] = false;
      launch_xy(make_args(h), h->st, h->dbl, q, q + 1, s);
      HIPCHK(h, hipGetLastError());
    } else {
      rebuild.push_back(q);
    }
    *n_back += r;
  }
  return rebuild_factors(h, rebuild);
}

double max_active_frac(sadmm_t h) {
  int m = 0;
  for (int q = 0; q < h->Q; ++q) m = std::max(m, h->nq[q]);
  return (double)m / h->N;
}

int validate(const sadmm_params* p) {
  if (!p) return SADMM_E_ARG;
  if (p->Q < 1 || p->K < 1 || p->M < 1 || p->N < 1) return SADMM_E_ARG;
  if (!(p->mu > 0) || !(p->beta > 0) || !(p->gamma >= 0) || !(p->lambda >= 0)) return SADMM_E_ARG;
  if (p->max_iter < 1 || p->check_every < 1) return SADMM_E_ARG;
  if (p->Kp < 1 || p->Kp > 64 || !(p->eps_p >= 0)) return SADMM_E_ARG;
  if (p->storage < SADMM_ST_FP64 || p->storage > SADMM_ST_MATRIX_FREE) return SADMM_E_ARG;
  if (p->gram < 0 || p->gram > 2) return SADMM_E_ARG;
  if (p->direct < 0 || p->direct > 1) return SADMM_E_ARG;
  if (p->refine_every < 0) return SADMM_E_ARG;
  if (p->nonneg < 0 || p->nonneg > 1) return SADMM_E_ARG;
  if (p->balance_every < 0) return SADMM_E_ARG;
  if (p->balance_every > 0 && !(p->balance_mu > 1.0 && p->balance_tau > 1.0)) return SADMM_E_ARG;
  if (p->refine_every > 0 && p->storage != SADMM_ST_FP16P && p->storage != SADMM_ST_BF16P)
    return SADMM_E_ARG;   // the correction is for 16-bit storage
  if (p->prune_mode < 0 || p->prune_mode > 1) return SADMM_E_ARG;
  if ((int64_t)p->K * p->M > 4096) return SADMM_E_SHAPE;   // W_q and LDS staging limits
  return SADMM_OK;
}

// ---- solve phases --------------------------------------------------------
// Prologue: measurements, state reset, selectors (caller mask, CNN),
// compaction, factor build, data term; uploads the iteration arguments.
// With rebuild_out, stops before the factor build and returns the sensors to
// rebuild (the caller builds them and then calls solve_prologue_finish).
// Buffers of the correction (allocated at the first solve that uses it) and
// a zero correction to start from.
int refine_setup(sadmm_t h) {
  for (int q = 0; q < h->Q; ++q)
    if (!h->rec[q])
      return fail_msg(h, SADMM_E_STATE,
                      "solve: refine_every needs the geometry of sensor %d (sadmm_set_operator_geometry)", q);
  const size_t QN = (size_t)h->Q * h->N;
  auto grab = [&](void** p, size_t bytes) -> int {
    if (*p) return SADMM_OK;
    if (hipMalloc(p, bytes) != hipSuccess) {
      *p = nullptr;
      return fail_msg(h, SADMM_E_NOMEM, "refinement buffers: %zu bytes", bytes);
    }
    return SADMM_OK;
  };
  TRY(grab((void**)&h->sens_mf_d, sizeof(SensorDesc) * h->Q));
  TRY(grab((void**)&h->gfix, 16 * QN));
  TRY(grab((void**)&h->gprev, 16 * QN));
  TRY(grab((void**)&h->dg, sizeof(double) * h->Q));
  if (!h->dg_h && hipHostMalloc((void**)&h->dg_h, sizeof(double) * h->Q) != hipSuccess) {
    h->dg_h = nullptr;
    return fail_msg(h, SADMM_E_NOMEM, "refinement buffers: pinned host copy");
  }
  TRY(grab(&h->g32, h->csz * QN));
  TRY(grab(&h->xfix, h->csz * QN));
  TRY(grab(&h->xprev, h->csz * QN));
  TRY(grab((void**)&h->re1, 16 * (size_t)h->Q * h->KMp));
  TRY(grab((void**)&h->re2, 16 * (size_t)h->Q * h->KMp));
  TRY(grab((void**)&h->rw, 16 * (size_t)h->Q * h->KMp));
  HIPCHK(h, hipMemsetAsync(h->gfix, 0, 16 * QN, h->s));
  HIPCHK(h, hipMemsetAsync(h->g32, 0, h->csz * QN, h->s));
  HIPCHK(h, hipMemsetAsync(h->xfix, 0, h->csz * QN, h->s));
  return SADMM_OK;
}

int solve_prologue_finish(sadmm_t h);
int solve_prologue(sadmm_t h, const void* y, int32_t dtype, int32_t on_device,
                   std::vector<int>* rebuild_out = nullptr) {
  if (!y || (dtype != SADMM_C128 && dtype != SADMM_C64)) return fail_msg(h, SADMM_E_ARG, "solve: bad y");
  for (int q = 0; q < h->Q; ++q)
    if (!h->op_set[q]) return fail_msg(h, SADMM_E_STATE, "solve: operator of sensor %d not set", q);
  if (h->p.refine_every > 0) TRY(refine_setup(h));
  if (h->p.beta != h->beta0) {   // a balanced solve left another beta: its factors do not fit
    h->p.beta = h->beta0;
    for (int q = 0; q < h->Q; ++q) h->fac_valid[q] = false;
  }
  hipStream_t s = h->s;
  h->info = sadmm_info{};
  h->solved = false;
  HIPCHK(h, hipEventRecord(h->ev0, s));
  const int Q = h->Q, N = h->N, KMp = h->KMp;
  // ---- measurements
  const size_t esz = dtype == SADMM_C128 ? 16 : 8;
  const void* ysrc = y;
  void* ystage = nullptr;
  if (!on_device) {
    if (hipMalloc(&ystage, esz * (size_t)Q * h->KM) != hipSuccess) return fail_msg(h, SADMM_E_NOMEM, "solve: y staging");
    HIPCHK(h, hipMemcpyAsync(ystage, y, esz * (size_t)Q * h->KM, hipMemcpyHostToDevice, s));
    ysrc = ystage;
  }
  load_measurements(ysrc, dtype == SADMM_C128, Q, h->KM, KMp, h->y, s);
  HIPCHK(h, hipMemcpyAsync(h->yp, h->y, 16 * (size_t)Q * KMp, hipMemcpyDeviceToDevice, s));
  // ---- state
  const size_t cN = h->csz * N;
  HIPCHK(h, hipMemsetAsync(h->X, 0, cN * Q, s));
  HIPCHK(h, hipMemsetAsync(h->dX, 0, cN * Q, s));
  HIPCHK(h, hipMemsetAsync(h->xbar, 0, cN, s));
  HIPCHK(h, hipMemsetAsync(h->z, 0, cN, s));
  HIPCHK(h, hipMemsetAsync(h->u, 0, cN, s));
  HIPCHK(h, hipMemsetAsync(h->D, 0, (h->dbl ? 8 : 4) * (size_t)h->p.Kp * Q * N, s));
  HIPCHK(h, hipMemsetAsync(h->gone, 0, sizeof(int) * Q, s));
  HIPCHK(h, hipMemsetAsync(h->hist, 0, sizeof(double) * 6 * (size_t)h->p.max_iter, s));
  Ctl c0{};
  c0.max_iter = h->p.max_iter;
  *h->ctl_h = c0;
  HIPCHK(h, hipMemcpyAsync(h->ctl, h->ctl_h, sizeof(Ctl), hipMemcpyHostToDevice, s));
  // ---- learned elimination (optional): matched filter -> CNN -> shared mask
  std::vector<uint8_t> cnn_keep;
  h->cnn_pruned = 0;
  if (h->cnn) {
    TRY(push_descs(h));
    int pe = prof_begin(h);
    launch_matched_filter(make_args(h), h->st, h->dbl, h->y, h->mf, s);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(s));
    const float* prob = nullptr;
    if (sadmm_cnn_prob_from_mf(h->cnn, h->mf, &prob) != SADMM_OK)
      return fail_msg(h, SADMM_E_HIP, "solve: CNN inference failed");
    std::vector<float> ph(N);
    HIPCHK(h, hipMemcpyAsync(ph.data(), prob, sizeof(float) * N, hipMemcpyDeviceToHost, sadmm_cnn_stream(h->cnn)));
    HIPCHK(h, hipStreamSynchronize(sadmm_cnn_stream(h->cnn)));
    prof_end(h, SADMM_KC_CNN, pe);
    cnn_keep.assign(N, 1);
    for (int n = 0; n < N; ++n)
      if (ph[n] >= h->cnn_thr) { cnn_keep[n] = 0; h->cnn_pruned += 1; }
  }
  // ---- selectors and compaction
  std::vector<int> rebuild;
  h->start_restricted = false;
  // host copies of the masks and index lists stay alive until the one stream
  // synchronisation after the loop (the uploads are asynchronous)
  std::vector<std::vector<uint8_t>> mh(Q);
  std::vector<std::vector<int>> Jq(Q);
  for (int q = 0; q < Q; ++q) {
    std::vector<int>& Jh = Jq[q];
    std::vector<uint8_t>& m = mh[q];
    m.assign(N, 1);
    if (!h->mask0[q].empty()) m = h->mask0[q];
    if (!cnn_keep.empty())
      for (int n = 0; n < N; ++n) m[n] = m[n] && cnn_keep[n];
    for (int n = 0; n < N; ++n)
      if (m[n]) Jh.push_back(n);
    h->nq[q] = (int)Jh.size();
    if (h->nq[q] < N) h->start_restricted = true;
    int rc = SADMM_OK;
    hipError_t e = hipMemcpyAsync(h->mask + (size_t)q * N, m.data(), N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !Jh.empty())
      e = hipMemcpyAsync(h->J[q], Jh.data(), sizeof(int) * Jh.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) rc = fail_msg(h, SADMM_E_HIP, "solve: mask upload: %s", hipGetErrorString(e));
    if (rc == SADMM_OK) rc = compact_operator(h, q);
    if (rc != SADMM_OK) {   // (uploads already queued read mh / Jq)
      hipStreamSynchronize(s);
      return rc;
    }
    // (built in solve_prologue_finish).  At the start only when F is also
    // smaller than W (N_q < KM): the Woodbury factors of a solve are built in
    // one batch, the direct inverses one sensor at a time.
    h->direct[q] = (want_direct(h, h->nq[q]) && h->nq[q] < h->KM) ? 1 : 0;
    if (!h->direct[q] && !h->shared_src &&
        (!h->p.reuse_factor || !h->fac_valid[q] || h->facJ[q] != Jh))
      rebuild.push_back(q);
    h->facJ[q] = Jh;
  }
  HIPCHK(h, hipStreamSynchronize(s));
  if (ystage) hipFree(ystage);
  TRY(push_descs(h));
  HIPCHK(h, hipEventRecord(h->evf0, s));
  if (rebuild_out) {
    *rebuild_out = rebuild;
    return SADMM_OK;
  }
  TRY(build_factors(h, rebuild));
  return solve_prologue_finish(h);
}

// Prologue, second part (factors built): data term, timing, arguments.
int solve_prologue_finish(sadmm_t h) {
  hipStream_t s = h->s;
  const int Q = h->Q;
  bool any_direct = false;
  for (int q = 0; q < Q; ++q) any_direct = any_direct || h->direct[q];
  if (!any_direct) {
    launch_xy(make_args(h), h->st, h->dbl, 0, Q, s);
  } else {
    for (int q = 0; q < Q; ++q) {
      if (h->direct[q]) TRY(build_direct(h, q, false));
      else launch_xy(make_args(h), h->st, h->dbl, q, q + 1, s);
    }
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->evf1, s));
  HIPCHK(h, hipEventSynchronize(h->evf1));
  prof_resolve(h);
  float fms = 0.f;
  hipEventElapsedTime(&fms, h->evf0, h->evf1);
  h->t_factor = fms;
  h->frac_pts.assign(1, {1, max_active_frac(h)});
  h->beta_pts.assign(1, {1, h->p.beta});
  h->kkt_rounds = 0;
  h->k_refined = 0;
  h->shift = 0.0;
  h->settled = false;
  h->k_jump = 0;
  h->retake_pts.clear();
  h->shift_pts.clear();
  h->status = 1;
  h->done = false;
  const IterArgs a = make_args(h);
  HIPCHK(h, hipMemcpyAsync(h->args_d, &a, sizeof(IterArgs), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return SADMM_OK;
}

// Correction of a 16-bit stored operator Ahat toward the accurate operator A
// (regenerated from the geometry's phase records, FP32 entries):
//   g = mu (A^H (y - A x) - Ahat^H (y' - Ahat x))   on the active pixels,
// with the x of the latest iteration.  The x-update then solves
// (mu Ahat^H Ahat + cI) x = mu Ahat^H y' + beta v + g, whose fixed point is
// the x-update of A itself.  A Woodbury sensor adds the precomputed
// xfix = (mu Ahat^H Ahat + cI)^{-1} g = (g - Ahat^H W Ahat g) / c, a direct
// sensor adds g to its right-hand side.  A x runs over every pixel, frozen
// ones included (y' holds their contribution through Ahat).
int refine_enqueue(sadmm_t h, hipStream_t s) {
  const size_t QK = (size_t)h->Q * h->KMp;
  const size_t QN = (size_t)h->Q * h->N;
  HIPCHK(h, hipMemcpyAsync(h->gprev, h->gfix, 16 * QN, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->xprev, h->xfix, h->csz * QN, hipMemcpyDeviceToDevice, s));
  const double mu = h->p.mu, cinv = 1.0 / (h->p.beta + h->p.gamma);
  const IterArgs a = make_args(h);
  IterArgs am = a;
  am.sens = h->sens_mf_d;
  int max_nq = 0;
  for (int q = 0; q < h->Q; ++q) max_nq = std::max(max_nq, h->nq[q]);
  // re1 = A x - y (every pixel), re2 = Ahat x - y' (active pixels)
  scale_c128(h->y, h->re1, (int)QK, -1.0, s);
  launch_refine_fwd(am, ST_MF, false, nullptr, 1.0, h->re1, s);
  scale_c128(h->yp, h->re2, (int)QK, -1.0, s);
  launch_refine_fwd(a, h->st, true, nullptr, 1.0, h->re2, s);
  // g = -mu A^H re1 + mu Ahat^H re2 on the active pixels
  launch_refine_grad(am, ST_MF, max_nq, h->re1, -mu, false, h->gfix, h->g32, s);
  launch_refine_grad(a, h->st, max_nq, h->re2, mu, true, h->gfix, h->g32, s);
  // xfix = (g - Ahat^H W (Ahat g)) / c   (Woodbury sensors)
  HIPCHK(h, hipMemsetAsync(h->re2, 0, 16 * QK, s));
  launch_refine_fwd(a, h->st, true, h->g32, 1.0, h->re2, s);
  launch_factor_vec(a, h->re2, h->rw, s);
  launch_refine_fix(a, h->st, max_nq, h->rw, h->gfix, cinv, h->xfix, s);
  // The move of the x-update under the new correction:
  // (mu Ahat^H Ahat + cI)^{-1} times the change of g, i.e. the change of xfix
  // for a Woodbury sensor and F applied to the change of g for a direct one.
  for (int q = 0; q < h->Q; ++q) {
    const size_t o = (size_t)q * h->N;
    if (h->direct[q])
      herm_apply_norm2(reinterpret_cast<const double*>(h->Fd[q]), h->fld[q], h->nq[q], h->J[q],
                       h->gfix + 2 * o, h->gprev + 2 * o, h->dg + q, s);
    else if (h->dbl)
      diff_norm2_c128(static_cast<const double*>(h->xfix) + 2 * o,
                      static_cast<const double*>(h->xprev) + 2 * o, h->N, h->dg + q, s);
    else
      diff_norm2_c64(static_cast<const float*>(h->xfix) + 2 * o,
                     static_cast<const float*>(h->xprev) + 2 * o, h->N, h->dg + q, s);
  }
  HIPCHK(h, hipMemcpyAsync(h->dg_h, h->dg, sizeof(double) * h->Q, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipGetLastError());
  return SADMM_OK;
}

// Iterations from the last scheduled correction to the next: the spacing
// doubles from 2 (corrections at 2, 4, 8, 16, ...) until it reaches
// refine_every.  A correction is taken at the current x, so its own error is
// proportional to the distance of x from the fixed point: early ones, while
// ADMM still moves x by more than that error, cost no convergence, and the
// fixed point is corrected as x approaches it instead of in jumps after x
// has settled on the uncorrected one.
int refine_gap(sadmm_t h) {
  return std::min(h->p.refine_every, std::max(2, h->k_refined));
}

// Completes a correction queued by refine_enqueue, once its stream has drained.
void refine_finish(sadmm_t h, int k) {
  double d2 = 0.0;
  for (int q = 0; q < h->Q; ++q) d2 += h->dg_h[q];
  h->shift = std::sqrt(d2);
  // settled: the move is within the primal tolerance, or within 1e-5 of the
  // iterate's norm (the scale in eps_pri), below which it is the FP32
  // rounding of the correction itself and no longer shrinks
  double tol = h->ctl_h->eps_pri;
  if (h->p.eps_rel > 0.0) {
    const double sqQN = std::sqrt((double)h->Q * h->N);
    tol = std::max(tol, 1e-5 * (h->ctl_h->eps_pri - sqQN * h->p.eps_abs) / h->p.eps_rel);
  }
  h->settled = h->shift <= tol;
  if (!h->settled) h->k_jump = k;
  h->shift_pts.push_back({k, h->shift});
  h->k_refined = k;
  h->args_dirty = true;      // SSC's window start moves with the correction
}

int refine(sadmm_t h, int k) {
  TRY(refine_enqueue(h, h->s));
  HIPCHK(h, hipStreamSynchronize(h->s));
  refine_finish(h, k);
  return SADMM_OK;
}

// Residual balancing (Boyd et al. 2011, Sec. 3.4.1), decided on the device at
// the last iteration: beta times or over balance_tau, the scaled dual divided
// by the same factor (beta u unchanged), every factor rebuilt for the new
// c = beta + gamma (the Woodbury ones in one batch), the arguments re-sent.
int apply_balance(sadmm_t h, int dir) {
  if (dir == 0) return SADMM_OK;
  const double f = dir > 0 ? h->p.balance_tau : 1.0 / h->p.balance_tau;
  scale_cplx(h->u, h->dbl, h->N, 1.0 / f, h->s);
  h->p.beta *= f;
  std::vector<int> wood;
  for (int q = 0; q < h->Q; ++q) {
    if (h->direct[q]) TRY(build_direct(h, q));
    else wood.push_back(q);
  }
  TRY(rebuild_factors(h, wood));
  for (int q = 0; q < h->Q; ++q) h->fac_valid[q] = false;
  h->args_dirty = true;
  return SADMM_OK;
}

// Handles the halt state of one scene after a status read.  Sets *active when
// the scene keeps iterating.
int handle_halt(sadmm_t h, const Ctl& c, bool* active) {
  *active = false;
  hipStream_t s = h->s;
  float fms = 0.f;
  if (c.halt & HALT_NAN) return fail_msg(h, SADMM_E_NUMERIC, "non-finite residual at iteration %d", c.k);
  if (!c.halt) { *active = true; return SADMM_OK; }
  if (c.halt & (HALT_PRUNE | HALT_BAL)) {
    HIPCHK(h, hipEventRecord(h->evf0, s));
    if (c.halt & HALT_PRUNE) {
      TRY(apply_prune(h));
      h->info.prune_events += 1;
      h->frac_pts.push_back({c.k, max_active_frac(h)});     // from the deciding iteration on
    }
    if (c.halt & HALT_BAL) {
      TRY(apply_balance(h, c.bal));
      h->beta_pts.push_back({c.k, h->p.beta});
    }
    if (h->p.refine_every > 0) TRY(refine(h, c.k));
    HIPCHK(h, hipEventRecord(h->evf1, s));
    HIPCHK(h, hipEventSynchronize(h->evf1));
    hipEventElapsedTime(&fms, h->evf0, h->evf1);
    h->t_factor += fms;
    const int nh = c.halt & ~(HALT_PRUNE | HALT_BAL);
    *h->halt_h = nh;
    HIPCHK(h, hipMemcpyAsync(&h->ctl->halt, h->halt_h, sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (nh == 0) { *active = true; return SADMM_OK; }
  }
  const int hb = c.halt & ~(HALT_PRUNE | HALT_BAL);
  if (hb & HALT_NMSE) { h->status = 2; h->done = true; return SADMM_OK; }
  if (hb & HALT_CONV) {
    bool any_frozen = false;
    for (int q = 0; q < h->Q; ++q) any_frozen = any_frozen || h->nq[q] < h->N;
    // the re-check judges solves that start from a selector (caller mask or
    // CNN): every elimination in them, the selector's and SSC's
    const bool judge = h->p.kkt && h->start_restricted && any_frozen;
    if (judge && h->kkt_rounds >= KKT_ROUNDS) {
      // round cap reached: certify without reinstating
      int bad = 0;
      TRY(kkt_reinstate(h, &bad, true));
      if (bad > 0) { h->status = 3; h->done = true; return SADMM_OK; }
    }
    if (judge && h->kkt_rounds < KKT_ROUNDS) {
      ++h->kkt_rounds;
      int back = 0;
      HIPCHK(h, hipEventRecord(h->evf0, s));
      TRY(kkt_reinstate(h, &back));
      HIPCHK(h, hipEventRecord(h->evf1, s));
      HIPCHK(h, hipEventSynchronize(h->evf1));
      hipEventElapsedTime(&fms, h->evf0, h->evf1);
      h->t_factor += fms;
      if (back > 0) {
        if (h->p.refine_every > 0) TRY(refine(h, c.k));
        h->info.reinstated += back;
        h->frac_pts.push_back({c.k + 1, max_active_frac(h)});
        if (c.k >= h->p.max_iter) { h->status = 1; h->done = true; return SADMM_OK; }
        *h->halt_h = 0;
        HIPCHK(h, hipMemcpyAsync(&h->ctl->halt, h->halt_h, sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(h, hipStreamSynchronize(s));
        *active = true;
        return SADMM_OK;
      }
    }
    if (h->p.refine_every > 0 && h->k_refined != c.k) {
      // The correction in use was taken at an earlier x.  Retake it at the
      // converged x; the solve stops only if the x-update moves by at most
      // the primal tolerance under the new one, else it goes on.  That move
      // is (mu Ahat^H Ahat + cI)^{-1} times the change of g: for a Woodbury
      // sensor the change of xfix itself, for a direct sensor F applied to
      // the change of g.  (The bound |dg| / c never meets the tolerance: the
      // inverse damps the part of dg in the range of Ahat^H, where the 16-bit
      // error and the FP32 rounding of A^H(y - A x) sit, by the operator's
      // large singular values.)
      if (c.k >= h->p.max_iter) { h->status = 1; h->done = true; return SADMM_OK; }
      TRY(refine(h, c.k));
      h->last_dg = h->shift;
      h->retake_pts.push_back({c.k, h->last_dg});
      if (!(h->last_dg <= c.eps_pri)) {
        *h->halt_h = 0;
        HIPCHK(h, hipMemcpyAsync(&h->ctl->halt, h->halt_h, sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(h, hipStreamSynchronize(s));
        *active = true;
        return SADMM_OK;
      }
    }
    h->status = 0;
    h->done = true;
    return SADMM_OK;
  }
  if (hb & HALT_MAXIT) { h->status = 1; h->done = true; }
  return SADMM_OK;
}

// Iteration loop over a batch of prepared handles (one launch per kernel for
// every scene; a hipGraph of one iteration is replayed between status reads).
int iterate(std::vector<sadmm_t>& hs, bool single, const SharedBatch* shared = nullptr) {
  sadmm_t h0 = hs[0];
  const int S = (int)hs.size();
  hipStream_t gs = h0->gs;
  // batch tables
  BatchDims d{};
  d.nscene = S;
  std::vector<int2> slots;
  for (int i = 0; i < S; ++i) {
    sadmm_t h = hs[i];
    for (int q = 0; q < h->Q; ++q) slots.push_back(make_int2(i, q));
    d.KMp_max = std::max(d.KMp_max, h->KMp);
    d.nchunk_max = std::max(d.nchunk_max, h->nchunk);
    d.N_max = std::max(d.N_max, h->N);
    d.nblk_max = std::max(d.nblk_max, h->nblk);
    d.fld_max = std::max(d.fld_max, direct_cap(h));   // covers every later switch
  }
  d.nslot = (int)slots.size();
  IterArgs* args_d = h0->args_d;
  int2* slots_d = h0->slots_d;
  Ctl** ctlp_d = nullptr;
  Ctl* ctl_all_d = nullptr;
  std::vector<Ctl> ctl_all(S);
  std::vector<IterArgs> av(S);          // host copies of the argument table
  std::vector<void*> tmp;
  auto cleanup = [&]() { for (void* p : tmp) hipFree(p); };
  if (!single) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(IterArgs) * S) != hipSuccess) return fail_msg(h0, SADMM_E_NOMEM, "batch tables");
    tmp.push_back(p); args_d = static_cast<IterArgs*>(p);
    if (hipMalloc(&p, sizeof(int2) * slots.size()) != hipSuccess) { cleanup(); return fail_msg(h0, SADMM_E_NOMEM, "batch tables"); }
    tmp.push_back(p); slots_d = static_cast<int2*>(p);
    if (hipMalloc(&p, sizeof(Ctl*) * S) != hipSuccess) { cleanup(); return fail_msg(h0, SADMM_E_NOMEM, "batch tables"); }
    tmp.push_back(p); ctlp_d = static_cast<Ctl**>(p);
    if (hipMalloc(&p, sizeof(Ctl) * S) != hipSuccess) { cleanup(); return fail_msg(h0, SADMM_E_NOMEM, "batch tables"); }
    tmp.push_back(p); ctl_all_d = static_cast<Ctl*>(p);
    std::vector<Ctl*> cp(S);
    for (int i = 0; i < S; ++i) { av[i] = make_args(hs[i]); cp[i] = hs[i]->ctl; }
    if (hipMemcpy(args_d, av.data(), sizeof(IterArgs) * S, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(slots_d, slots.data(), sizeof(int2) * slots.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctlp_d, cp.data(), sizeof(Ctl*) * S, hipMemcpyHostToDevice) != hipSuccess) {
      cleanup();
      return fail_msg(h0, SADMM_E_HIP, "batch tables: copy failed");
    }
  }
  const BatchView bv{args_d, slots_d};
  const bool staged = single && h0->prof_level >= 2;
  // graph of one iteration (captured once per handle, or per batch call)
  hipGraphExec_t ge = (single && !staged) ? h0->gexec : nullptr;
  hipGraph_t gr = nullptr;
  if (!staged && !ge) {
    bool ok = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      if (shared) launch_iteration_shared(bv, d, *shared, gs, nullptr);
      else launch_iteration_batch(bv, d, h0->st, gs, nullptr);
      ok = hipStreamEndCapture(gs, &gr) == hipSuccess && gr;
      ok = ok && hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0) == hipSuccess;
    }
    if (!ok) { ge = nullptr; (void)hipGetLastError(); }
    if (single && ge) { h0->gexec = ge; h0->graph = gr; gr = nullptr; }
  }
  const int check = h0->p.check_every;
  int rc = SADMM_OK;
  for (;;) {
    // status read where the earliest correction of a running scene is due
    // (scenes that halted in between run behind the others and correct at
    // the first status read at or after theirs)
    int nq_iter = check;
    for (const sadmm_t h : hs)
      if (!h->done && h->p.refine_every > 0)
        nq_iter = std::min(nq_iter, std::max(1, h->k_refined + refine_gap(h) - h->ctl_h->k));
    for (int i = 0; i < nq_iter; ++i) {
      if (ge) {
        if (hipGraphLaunch(ge, gs) != hipSuccess) { rc = fail_msg(h0, SADMM_E_HIP, "graph launch failed"); break; }
      } else if (staged) {
        sadmm_t h = h0;
        int ev[IT_NSTAGE];
        for (int k = 0; k < IT_NSTAGE; ++k) ev[k] = -1;
        if (h->evnext + 2 * IT_NSTAGE <= h->evpool.size()) {
          for (int k = 0; k < IT_NSTAGE; ++k) ev[k] = (int)(h->evnext + 2 * k);
          h->evnext += 2 * IT_NSTAGE;
        }
        {
          // algorithmic bytes of one iteration, per stage
          const double ob = op_bytes(h), cz = (double)h->csz;
          double nqs = 0;
          for (int q = 0; q < h->Q; ++q) nqs += h->nq[q];
          const double KM = h->KM, Q = h->Q, N = h->N;
          prof_work(h, SADMM_KC_FWD, nqs * KM * ob + nqs * 4 * cz + Q * KM * cz);
          prof_work(h, SADMM_KC_WPROD, Q * (KM * KM * 16.0 + 2 * KM * cz));
          prof_work(h, SADMM_KC_XUPD, nqs * KM * ob + Q * KM * cz + nqs * (7 * cz + cz / 2));
          prof_work(h, SADMM_KC_PIXEL, Q * N * 2 * cz + N * 6 * cz);
        }
        std::function<void(int, bool)> hook = [&](int stage, bool begin) {
          if (ev[0] < 0) return;
          hipEventRecord(h->evpool[ev[stage] + (begin ? 0 : 1)], gs);
          if (!begin) h->marks.push_back({SADMM_KC_FWD + stage, ev[stage], ev[stage] + 1});
        };
        if (shared) launch_iteration_shared(bv, d, *shared, gs, &hook);
        else launch_iteration_batch(bv, d, h0->st, gs, &hook);
      } else {
        if (shared) launch_iteration_shared(bv, d, *shared, gs, nullptr);
        else launch_iteration_batch(bv, d, h0->st, gs, nullptr);
      }
    }
    if (rc != SADMM_OK) break;
    if (hipGetLastError() != hipSuccess) { rc = fail_msg(h0, SADMM_E_HIP, "iteration launch failed"); break; }
    if (single) {
      if (hipMemcpyAsync(h0->ctl_h, h0->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, gs) != hipSuccess ||
          hipStreamSynchronize(gs) != hipSuccess) { rc = fail_msg(h0, SADMM_E_HIP, "status read failed"); break; }
      ctl_all[0] = *h0->ctl_h;
      prof_resolve(h0);
    } else {
      gather_ctl(ctlp_d, ctl_all_d, S, gs);
      if (hipMemcpyAsync(ctl_all.data(), ctl_all_d, sizeof(Ctl) * S, hipMemcpyDeviceToHost, gs) != hipSuccess ||
          hipStreamSynchronize(gs) != hipSuccess) { rc = fail_msg(h0, SADMM_E_HIP, "status read failed"); break; }
    }
    bool any = false;
    std::vector<int> due;                 // scenes whose scheduled correction is due
    for (int i = 0; i < S && rc == SADMM_OK; ++i) {
      sadmm_t h = hs[i];
      if (h->done) continue;
      *h->ctl_h = ctl_all[i];
      bool active = false;
      rc = handle_halt(h, ctl_all[i], &active);
      if (rc == SADMM_OK && active && h->p.refine_every > 0 &&
          ctl_all[i].k - h->k_refined >= refine_gap(h))
        due.push_back(i);
      if (rc != SADMM_OK && h != h0) h0->err = h->err;
      any = any || active;
    }
    // The due corrections of every scene queued together, one wait.  A
    // batch puts each scene's on that scene's own (idle) graph stream: the
    // kernels of one scene's correction are small, and the scenes' run side
    // by side instead of one after another.
    auto fix_stream = [&](sadmm_t h) { return single ? h->s : h->gs; };
    for (size_t j = 0; j < due.size() && rc == SADMM_OK; ++j) {
      rc = refine_enqueue(hs[due[j]], fix_stream(hs[due[j]]));
      if (rc != SADMM_OK && hs[due[j]] != h0) h0->err = hs[due[j]]->err;
    }
    if (rc == SADMM_OK && !due.empty()) {
      std::vector<hipStream_t> ss;
      for (int i : due)
        if (std::find(ss.begin(), ss.end(), fix_stream(hs[i])) == ss.end()) ss.push_back(fix_stream(hs[i]));
      for (hipStream_t st : ss)
        if (hipStreamSynchronize(st) != hipSuccess) rc = fail_msg(h0, SADMM_E_HIP, "correction failed");
      for (int i : due)
        if (rc == SADMM_OK) refine_finish(hs[i], ctl_all[i].k);
    }
    // changed iteration arguments, one wait
    bool uploaded = false;
    for (int i = 0; i < S && rc == SADMM_OK; ++i) {
      sadmm_t h = hs[i];
      if (!h->args_dirty) continue;
      av[i] = make_args(h);
      if (hipMemcpyAsync(args_d + i, &av[i], sizeof(IterArgs), hipMemcpyHostToDevice, gs) != hipSuccess)
        rc = fail_msg(h0, SADMM_E_HIP, "argument upload failed");
      h->args_dirty = false;
      uploaded = true;
    }
    if (rc == SADMM_OK && uploaded && hipStreamSynchronize(gs) != hipSuccess)
      rc = fail_msg(h0, SADMM_E_HIP, "argument upload failed");
    if (rc != SADMM_OK || !any) break;
  }
  if (!single) {
    if (ge) hipGraphExecDestroy(ge);
    if (gr) hipGraphDestroy(gr);
  }
  hipStreamSynchronize(gs);
  cleanup();
  return rc;
}

// Epilogue: timing, history, info.
int solve_epilogue(sadmm_t h, sadmm_info* info) {
  hipStream_t s = h->s;
  float fms = 0.f;
  HIPCHK(h, hipEventRecord(h->ev1, s));
  HIPCHK(h, hipEventSynchronize(h->ev1));
  hipEventElapsedTime(&fms, h->ev0, h->ev1);
  h->t_total = fms;
  h->t_iter = h->t_total - h->t_factor;
  HIPCHK(h, hipMemcpy(h->ctl_h, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  const Ctl c = *h->ctl_h;
  h->hist_count = c.k;
  h->hist_h.assign(9 * (size_t)h->p.max_iter, 0.0);
  HIPCHK(h, hipMemcpy(h->hist_h.data(), h->hist, sizeof(double) * 5 * h->p.max_iter, hipMemcpyDeviceToHost));
  for (int k = 1; k <= c.k; ++k) {
    double f = h->frac_pts[0].second;
    for (auto& pt : h->frac_pts)
      if (pt.first <= k) f = pt.second;
    h->hist_h[5 * (size_t)h->p.max_iter + k - 1] = f;
  }
  for (auto& pt : h->retake_pts)
    if (pt.first >= 1 && pt.first <= h->p.max_iter) h->hist_h[6 * (size_t)h->p.max_iter + pt.first - 1] = pt.second;
  for (auto& pt : h->shift_pts)
    if (pt.first >= 1 && pt.first <= h->p.max_iter) h->hist_h[8 * (size_t)h->p.max_iter + pt.first - 1] = pt.second;
  for (int k = 1; k <= c.k; ++k) {
    double b = h->beta_pts[0].second;
    for (auto& pt : h->beta_pts)
      if (pt.first <= k) b = pt.second;
    h->hist_h[7 * (size_t)h->p.max_iter + k - 1] = b;
  }
  h->info.iters = c.k;
  h->info.status = h->status;
  h->info.r = c.r; h->info.s = c.s; h->info.eps_pri = c.eps_pri; h->info.eps_dual = c.eps_dual;
  h->info.nmse = c.nmse;
  h->info.max_active_frac = max_active_frac(h);
  h->info.direct_sensors = 0;
  for (int q = 0; q < h->Q; ++q) h->info.direct_sensors += h->direct[q];
  h->solved = true;
  if (info) *info = h->info;
  return SADMM_OK;
}

}  // namespace


// ====================================================================== C ABI
extern "C" {

void sadmm_default_params(sadmm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->mu = 1.0; p->beta = 1.0; p->gamma = 1.0; p->lambda = 0.0;
  p->eps_abs = 0.0; p->eps_rel = 1e-4;
  p->max_iter = 200; p->stop = 1; p->check_every = 8;
  p->prune = 0; p->Kp = 5; p->eps_p = 1e-5; p->prune_mode = 0;
  p->kkt = 0; p->kkt_tol = 1e-2;
  p->balance_every = 0; p->balance_mu = 10.0; p->balance_tau = 2.0;
  p->storage = SADMM_ST_FP32;
  p->reuse_factor = 1;
  p->stream = nullptr;
}

static int create_impl(const sadmm_params* p, sadmm_t src, sadmm_t* out);

int sadmm_create(const sadmm_params* p, sadmm_t* out) { return create_impl(p, nullptr, out); }

int sadmm_create_shared(const sadmm_params* p, sadmm_t src, sadmm_t* out) {
  if (!out || !p || !src) return SADMM_E_ARG;
  *out = nullptr;
  auto bad = [&](const char* why) {
    g_create_err = std::string("create_shared: ") + why;
    return SADMM_E_ARG;
  };
  if (src->shared_src) return bad("the source borrows its operator itself");
  if (p->Q != src->Q || p->K != src->K || p->M != src->M || p->N != src->N || p->storage != src->p.storage)
    return bad("shape or storage differs from the source");
  if (p->mu != src->p.mu || p->beta != src->p.beta || p->gamma != src->p.gamma)
    return bad("mu, beta, gamma must equal the source's (the factor is shared)");
  if (p->prune || p->kkt || src->p.prune || src->p.kkt)
    return bad("shared operators need plain SADMM (prune = 0, kkt = 0) on both handles");
  for (int q = 0; q < src->Q; ++q)
    if (!src->mask0[q].empty()) return bad("the source has a pixel selector");
  return create_impl(p, src, out);
}

static int create_impl(const sadmm_params* p, sadmm_t src, sadmm_t* out) {
  if (!out) return SADMM_E_ARG;
  *out = nullptr;
  int rc = validate(p);
  if (rc != SADMM_OK) return rc;
  sadmm_t h = new sadmm_s();
  if (hipGetDevice(&h->dev) != hipSuccess) h->dev = 0;
  h->shared_src = src;
  if (src) src->n_sharers += 1;   // (given back by sadmm_destroy, also on a failed create)
  h->p = *p;
  h->beta0 = p->beta;
  h->Q = p->Q; h->K = p->K; h->M = p->M; h->N = p->N;
  h->KM = p->K * p->M;
  h->KMp = round_up(h->KM, 32);
  h->st = p->storage;
  h->dbl = (h->st == ST_FP64);
  h->csz = h->dbl ? 16 : 8;
  h->s = static_cast<hipStream_t>(p->stream);
  if (h->st == ST_FP64) { h->ldA = h->KMp; h->slot = 16; }
  else if (h->st == ST_FP32) { h->ldA = h->KMp; h->slot = 8; }
  else if (h->st == ST_MF) { h->ldA = MF_REC_BASE + MF_REC_PER_RX * (int64_t)h->M; h->slot = 8; }
  else { h->ldA = 2 * (int64_t)h->KMp; h->slot = 2; }
  // forward product: columns per work-group.  Long streams of stored FP32 /
  // FP64 or generated entries (1024 columns at N = 128^2: 6.2 TB/s against
  // 5.5 at 256), but at least 16 chunks per sensor; 16-bit planes at most
  // 256.  At c1 (N = 32^2, 256 rows) 64 columns took the forward from 14 to
  // 4 us.
  h->chunk_min = fwd_chunk_min(h->N);
  {
    const int cm = h->chunk_min;
    const int wide = (h->st == ST_FP16P || h->st == ST_BF16P) ? 256 : 1024;
    h->chunk = std::min(wide, std::max(cm, (h->N / 16) / cm * cm));
  }
  {
    const int tuned = tuned_chunk(h->st, h->KMp, h->N);
    if (tuned >= h->chunk_min) h->chunk = tuned;
  }
  h->nchunk = (h->N + h->chunk - 1) / h->chunk;
  h->nchunk_cap = (h->N + h->chunk_min - 1) / h->chunk_min;
  h->nblk = (h->N + 255) / 256;
  const int Q = h->Q, N = h->N, KMp = h->KMp;
  const size_t cN = h->csz * N;
  h->Afull.assign(Q, nullptr); h->Ahat_buf.assign(Q, nullptr);
  h->W64.assign(Q, nullptr); h->Wc.assign(Q, nullptr); h->W.assign(Q, nullptr);
  h->J.assign(Q, nullptr); h->Jnew.assign(Q, nullptr); h->xy.assign(Q, nullptr);
  h->nq.assign(Q, N); h->op_set.assign(Q, false); h->fac_valid.assign(Q, false);
  h->facJ.assign(Q, {}); h->mask0.assign(Q, {});
  h->hpdD.assign(Q, nullptr); h->hpdX.assign(Q, nullptr); h->hpdT.assign(Q, nullptr);
  h->direct.assign(Q, 0); h->Fd.assign(Q, nullptr); h->b0d.assign(Q, nullptr);
  h->rdir.assign(Q, nullptr); h->fld.assign(Q, 0);
  h->rec.assign(Q, nullptr);
  h->wtri.assign(Q, 0);
  h->sens_h.assign(Q, SensorDesc{});
  h->rmax = std::min(KMp, 1024);
  h->rpad_max = round_up(h->rmax, HPD_NB);
#define A_(expr) do { int r_ = (expr); if (r_ != SADMM_OK) { sadmm_destroy(h); return r_; } } while (0)
  for (int q = 0; q < Q; ++q) {
    if (src) {   // borrowed: operator, factor and its scratch
      h->Afull[q] = src->Afull[q];
      h->W64[q] = src->W64[q];
      h->hpdD[q] = src->hpdD[q];
      h->hpdX[q] = src->hpdX[q];
      h->hpdT[q] = src->hpdT[q];
      h->op_set[q] = true;
    } else {
      A_(dalloc(h, &h->Afull[q], (size_t)h->ldA * h->slot * N));
      A_(dalloc_t(h, &h->W64[q], sizeof(cd) * (size_t)KMp * KMp));
      A_(dalloc_t(h, &h->hpdD[q], sizeof(cd) * (size_t)HPD_NB * KMp));
      A_(dalloc_t(h, &h->hpdX[q], sizeof(cd) * (size_t)KMp * KMp));
      A_(dalloc_t(h, &h->hpdT[q], sizeof(cd) * ((size_t)KMp * KMp / 4 + 1)));
    }
    A_(dalloc_t(h, &h->J[q], sizeof(int) * N));
    A_(dalloc_t(h, &h->Jnew[q], sizeof(int) * N));
    A_(dalloc(h, &h->xy[q], cN));
  }
  A_(dalloc(h, &h->X, cN * Q));
  A_(dalloc(h, &h->dX, cN * Q));
  A_(dalloc(h, &h->xbar, cN));
  A_(dalloc(h, &h->z, cN));
  A_(dalloc(h, &h->u, cN));
  A_(dalloc(h, &h->xref, cN));
  A_(dalloc(h, &h->D, (h->dbl ? 8 : 4) * (size_t)p->Kp * Q * N));
  A_(dalloc(h, &h->tpart, h->csz * (size_t)Q * h->nchunk_cap * KMp));
  A_(dalloc(h, &h->gtmp, h->csz * (size_t)h->nchunk_cap * KMp));
  A_(dalloc(h, &h->t, h->csz * (size_t)Q * KMp));
  A_(dalloc(h, &h->w, h->csz * (size_t)Q * KMp));
  A_(dalloc_t(h, &h->y, 16 * (size_t)Q * KMp));
  A_(dalloc_t(h, &h->yp, 16 * (size_t)Q * KMp));
  A_(dalloc_t(h, &h->e, 16 * (size_t)KMp));
  A_(dalloc_t(h, &h->wy, 16 * (size_t)Q * KMp));
  A_(dalloc_t(h, &h->red, sizeof(double) * 8 * h->nblk));
  A_(dalloc_t(h, &h->hist, sizeof(double) * 6 * (size_t)p->max_iter));
  A_(dalloc_t(h, &h->mf, sizeof(double) * (size_t)Q * N));
  A_(dalloc_t(h, &h->mask, (size_t)Q * N));
  A_(dalloc_t(h, &h->keep, (size_t)Q * N));
  A_(dalloc_t(h, &h->flag, (size_t)N));
  A_(dalloc_t(h, &h->gone, sizeof(int) * Q));
  A_(dalloc_t(h, &h->fail, sizeof(int)));
  A_(dalloc_t(h, &h->counts, sizeof(int) * 2));
  A_(dalloc_t(h, &h->lst, sizeof(int) * N));
  A_(dalloc_t(h, &h->lst2, sizeof(int) * N));
  A_(dalloc_t(h, &h->ctl, sizeof(Ctl)));
  A_(dalloc_t(h, &h->args_d, sizeof(IterArgs)));
  A_(dalloc_t(h, &h->slots_d, sizeof(int2) * Q));
  A_(dalloc_t(h, &h->sens_d, sizeof(SensorDesc) * Q));
  A_(dalloc_t(h, &h->gemm_d, sizeof(GemmDesc) * std::max(Q, 4)));
  A_(dalloc_t(h, &h->hpd_d, sizeof(HpdDesc) * Q));
  A_(dalloc_t(h, &h->ws, 16 * (size_t)Q * KMp));
  A_(dalloc_t(h, &h->gi8_d, sizeof(GramI8Desc) * Q));
  {
    const std::vector<int2> order = tri_tile_order((KMp + 63) / 64);
    h->ntiles = (int)order.size();
    A_(dalloc_t(h, &h->tiles_d, sizeof(int2) * order.size()));
    A_(hipMemcpy(h->tiles_d, order.data(), sizeof(int2) * order.size(), hipMemcpyHostToDevice) == hipSuccess
           ? SADMM_OK : fail_msg(h, SADMM_E_HIP, "tile order upload"));
  }
  A_(dalloc_t(h, &h->Ar, sizeof(cd) * (size_t)KMp * h->rmax));
  A_(dalloc_t(h, &h->V, sizeof(cd) * (size_t)KMp * h->rmax));
  A_(dalloc_t(h, &h->Tm, sizeof(cd) * (size_t)KMp * h->rmax));
  A_(dalloc_t(h, &h->Cm, sizeof(cd) * (size_t)h->rpad_max * h->rpad_max));
  A_(dalloc_t(h, &h->Dg, sizeof(cd) * (size_t)HPD_NB * h->rpad_max));
  A_(dalloc_t(h, &h->Xg, sizeof(cd) * (size_t)h->rpad_max * h->rpad_max));
  A_(dalloc_t(h, &h->Tg, sizeof(cd) * ((size_t)h->rpad_max * h->rpad_max / 4 + 1)));
  A_(dalloc_t(h, &h->mm_d, sizeof(MmDesc) * std::max((size_t)Q * hpd_mm_count(KMp),
                                                     hpd_mm_count(h->rpad_max))));
  g_create_err.clear();
  if (hipHostMalloc((void**)&h->ctl_h, sizeof(Ctl)) != hipSuccess ||
      hipHostMalloc((void**)&h->counts_h, 2 * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&h->halt_h, sizeof(int)) != hipSuccess) {
    g_create_err = "pinned host allocation failed";
    sadmm_destroy(h);
    return SADMM_E_NOMEM;
  }
  {
    std::vector<int2> sl(Q);
    for (int q = 0; q < Q; ++q) sl[q] = make_int2(0, q);
    if (hipMemcpy(h->slots_d, sl.data(), sizeof(int2) * Q, hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreate(&h->gs) != hipSuccess) {
      sadmm_destroy(h);
      return SADMM_E_HIP;
    }
  }
  if (hipMemsetAsync(h->fail, 0, sizeof(int), h->s) != hipSuccess ||
      hipMemsetAsync(h->gone, 0, sizeof(int) * Q, h->s) != hipSuccess ||
      hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
      hipEventCreate(&h->evf0) != hipSuccess || hipEventCreate(&h->evf1) != hipSuccess ||
      hipStreamSynchronize(h->s) != hipSuccess) {
    sadmm_destroy(h);
    return SADMM_E_HIP;
  }
#undef A_
  if (src) {
    for (int q = 0; q < src->Q; ++q)   // borrowers read W itself
      if (ensure_w(src, q) != SADMM_OK) {
        sadmm_destroy(h);   // (gives back the share)
        return SADMM_E_HIP;
      }
  }
  *out = h;
  return SADMM_OK;
}

int sadmm_set_operator(sadmm_t h, int32_t q, const void* A, int32_t dtype, int64_t ld,
                       int32_t on_device) {
  if (!h) return SADMM_E_ARG;
  if (!A || q < 0 || q >= h->Q || (dtype != SADMM_C128 && dtype != SADMM_C64))
    return fail_msg(h, SADMM_E_ARG, "set_operator: bad argument");
  if (ld < h->KM) return fail_msg(h, SADMM_E_SHAPE, "set_operator: ld %lld < KM %d", (long long)ld, h->KM);
  if (h->shared_src) return fail_msg(h, SADMM_E_STATE, "set_operator: the operator is borrowed");
  if (h->st == ST_MF)
    return fail_msg(h, SADMM_E_STATE, "set_operator: a matrix-free handle takes sadmm_set_operator_geometry");
  const size_t esz = dtype == SADMM_C128 ? 16 : 8;
  const void* src = A;
  void* stage = nullptr;
  if (!on_device) {
    // stage through device memory in the caller's dtype, packed ld = KM
    if (hipMalloc(&stage, esz * (size_t)h->KM * h->N) != hipSuccess)
      return fail_msg(h, SADMM_E_NOMEM, "set_operator: staging allocation failed");
    hipError_t e = hipMemcpy2DAsync(stage, esz * h->KM, A, esz * ld, esz * h->KM, h->N,
                                    hipMemcpyHostToDevice, h->s);
    if (e != hipSuccess) {
      hipFree(stage);
      return fail_msg(h, SADMM_E_HIP, "set_operator: copy failed: %s", hipGetErrorString(e));
    }
    src = stage;
    ld = h->KM;
  }
  convert_operator(src, dtype == SADMM_C128, ld, h->KM, h->N, h->st, h->Afull[q], h->ldA, h->KMp, h->s);
  if (h->rec[q]) {   // the geometry no longer describes this operator
    hipStreamSynchronize(h->s);
    hipFree(h->rec[q]);
    h->rec[q] = nullptr;
  }
  hipError_t e = hipStreamSynchronize(h->s);
  if (stage) hipFree(stage);
  if (e != hipSuccess) return fail_msg(h, SADMM_E_HIP, "set_operator: %s", hipGetErrorString(e));
  TRY(cache_rowmax(h, q));
  h->op_set[q] = true;
  h->fac_valid[q] = false;
  return SADMM_OK;
}

int sadmm_set_operator_geometry(sadmm_t h, int32_t q, const double* tx_xy, const double* rx_xy,
                                const double* pix_xy, double f0, double bw) {
  if (!h) return SADMM_E_ARG;
  if (q < 0 || q >= h->Q || !tx_xy || !rx_xy || !pix_xy)
    return fail_msg(h, SADMM_E_ARG, "set_operator_geometry: bad argument");
  if (h->shared_src) return fail_msg(h, SADMM_E_STATE, "set_operator_geometry: the operator is borrowed");
  double* g = nullptr;
  const size_t nb = sizeof(double) * (2 + 2 * (size_t)h->M + 2 * (size_t)h->N);
  if (hipMalloc((void**)&g, nb) != hipSuccess)
    return fail_msg(h, SADMM_E_NOMEM, "set_operator_geometry: allocation failed");
  hipMemcpyAsync(g, tx_xy, 2 * sizeof(double), hipMemcpyHostToDevice, h->s);
  hipMemcpyAsync(g + 2, rx_xy, 2 * sizeof(double) * h->M, hipMemcpyHostToDevice, h->s);
  hipMemcpyAsync(g + 2 + 2 * h->M, pix_xy, 2 * sizeof(double) * h->N, hipMemcpyHostToDevice, h->s);
  if (h->st == ST_MF)
    mf_records(g, g + 2, g + 2 + 2 * h->M, h->M, h->K, h->N, f0, bw, static_cast<double*>(h->Afull[q]),
               h->ldA, h->s);
  else
    geometry_operator(g, g + 2, g + 2 + 2 * h->M, h->M, h->K, h->N, f0, bw, h->st, h->Afull[q], h->ldA,
                      h->KMp, h->s);
  if (h->st == ST_FP16P || h->st == ST_BF16P) {
    // phase records of the same geometry: the accurate operator of the correction
    const int64_t ldr = MF_REC_BASE + MF_REC_PER_RX * (int64_t)h->M;
    if (!h->rec[q] && hipMalloc((void**)&h->rec[q], sizeof(double) * ldr * h->N) != hipSuccess) {
      h->rec[q] = nullptr;
      hipStreamSynchronize(h->s);
      hipFree(g);
      return fail_msg(h, SADMM_E_NOMEM, "set_operator_geometry: record allocation failed");
    }
    mf_records(g, g + 2, g + 2 + 2 * h->M, h->M, h->K, h->N, f0, bw, h->rec[q], ldr, h->s);
  }
  hipError_t e = hipStreamSynchronize(h->s);
  hipFree(g);
  if (e != hipSuccess) return fail_msg(h, SADMM_E_HIP, "set_operator_geometry: %s", hipGetErrorString(e));
  TRY(cache_rowmax(h, q));
  h->op_set[q] = true;
  h->fac_valid[q] = false;
  return SADMM_OK;
}

int sadmm_set_active_mask(sadmm_t h, int32_t q, const uint8_t* mask) {
  if (!h) return SADMM_E_ARG;
  if (q < 0 || q >= h->Q) return fail_msg(h, SADMM_E_ARG, "set_active_mask: bad sensor");
  if (!mask) { h->mask0[q].clear(); return SADMM_OK; }
  if (h->shared_src || h->n_sharers > 0)
    return fail_msg(h, SADMM_E_STATE, "set_active_mask: the operator is shared (plain SADMM only)");
  h->mask0[q].assign(mask, mask + h->N);
  for (auto& v : h->mask0[q]) v = v ? 1 : 0;
  return SADMM_OK;
}

int sadmm_set_reference(sadmm_t h, const void* x_ref, int32_t dtype, int32_t on_device,
                        double nmse_target) {
  if (!h) return SADMM_E_ARG;
  if (!x_ref) { h->have_ref = false; h->nmse_target = 0; return SADMM_OK; }
  if (dtype != SADMM_C128 && dtype != SADMM_C64) return fail_msg(h, SADMM_E_ARG, "set_reference: dtype");
  const size_t esz = dtype == SADMM_C128 ? 16 : 8;
  std::vector<double> hostc(2 * (size_t)h->N);
  if (on_device) {
    if (hipMemcpy(hostc.data(), x_ref, esz * h->N, hipMemcpyDeviceToHost) != hipSuccess)
      return fail_msg(h, SADMM_E_HIP, "set_reference: copy failed");
    if (dtype == SADMM_C64) {
      std::vector<float> f(2 * (size_t)h->N);
      std::memcpy(f.data(), hostc.data(), esz * h->N);
      for (size_t i = 0; i < f.size(); ++i) hostc[i] = f[i];
    }
  } else if (dtype == SADMM_C128) {
    std::memcpy(hostc.data(), x_ref, esz * h->N);
  } else {
    const float* f = static_cast<const float*>(x_ref);
    for (size_t i = 0; i < 2 * (size_t)h->N; ++i) hostc[i] = f[i];
  }
  double n2 = 0.0;
  for (double v : hostc) n2 += v * v;
  if (!(n2 > 0)) return fail_msg(h, SADMM_E_ARG, "set_reference: zero reference");
  double* d = nullptr;
  if (hipMalloc((void**)&d, 16 * (size_t)h->N) != hipSuccess) return fail_msg(h, SADMM_E_NOMEM, "set_reference");
  hipMemcpyAsync(d, hostc.data(), 16 * (size_t)h->N, hipMemcpyHostToDevice, h->s);
  c128_to_compute(d, h->xref, h->dbl, h->N, h->s);
  hipError_t e = hipStreamSynchronize(h->s);
  hipFree(d);
  if (e != hipSuccess) return fail_msg(h, SADMM_E_HIP, "set_reference: %s", hipGetErrorString(e));
  h->xref_norm2 = n2;
  h->nmse_target = nmse_target;
  h->have_ref = true;
  return SADMM_OK;
}

// A handle that borrows an operator uses its source's factor: build it when
// it is not valid (the source's own solve would).
int ensure_source_factor(sadmm_t h) {
  sadmm_t src = h->shared_src;
  if (!src) return SADMM_OK;
  std::vector<int> qs;
  for (int q = 0; q < src->Q; ++q)
    if (!src->fac_valid[q]) qs.push_back(q);
  if (qs.empty()) return SADMM_OK;
  const int rc = build_factors(src, qs);
  if (rc != SADMM_OK) h->err = src->err;
  return rc;
}

int sadmm_solve(sadmm_t h, const void* y, int32_t dtype, int32_t on_device, sadmm_info* info) {
  if (!h) return SADMM_E_ARG;
  TRY(ensure_source_factor(h));
  TRY(solve_prologue(h, y, dtype, on_device));
  std::vector<sadmm_t> hs{h};
  TRY(iterate(hs, /*single=*/true));
  return solve_epilogue(h, info);
}

int sadmm_autotune(sadmm_t h, const void* y, int32_t dtype, int32_t on_device, int32_t iters, int32_t* chunk) {
  if (!h || !chunk) return SADMM_E_ARG;
  if (iters == 0) { *chunk = h->chunk; return SADMM_OK; }
  if (iters < 2) return fail_msg(h, SADMM_E_ARG, "autotune: iters >= 2 (or 0 to query)");
  if (h->shared_src || h->n_sharers) return fail_msg(h, SADMM_E_ARG, "autotune: not for shared operators");
  const sadmm_params saved = h->p;
  // plain iterations of the handle's problem, factor built once and reused
  h->p.max_iter = std::min(iters, saved.max_iter);
  h->p.stop = 0; h->p.prune = 0; h->p.kkt = 0; h->p.refine_every = 0; h->p.balance_every = 0;
  h->p.reuse_factor = 1;
  auto drop_graph = [&]() {
    if (h->gexec) hipGraphExecDestroy(h->gexec);
    if (h->graph) hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
  };
  int best = h->chunk, rc = SADMM_OK;
  double best_ms = 1e300;
  for (int c : FWD_CHUNKS) {
    if (c < h->chunk_min) continue;
    if (c > h->chunk_min && c >= h->N) break;         // one chunk already covers the image
    h->chunk = c;
    h->nchunk = (h->N + c - 1) / c;
    drop_graph();
    sadmm_info inf{};
    // untimed pass: captures this width's graph (and builds the factor once)
    rc = sadmm_solve(h, y, dtype, on_device, &inf);
    if (rc != SADMM_OK) break;
    rc = sadmm_solve(h, y, dtype, on_device, &inf);
    if (rc != SADMM_OK) break;
    const double ms = h->t_iter / std::max(1, inf.iters);
    if (ms < best_ms) { best_ms = ms; best = c; }
  }
  h->p = saved;
  h->chunk = best;
  h->nchunk = (h->N + best - 1) / best;
  drop_graph();
  h->solved = false;
  if (rc != SADMM_OK) return rc;
  set_tuned_chunk(h->st, h->KMp, h->N, best);
  *chunk = best;
  return SADMM_OK;
}

int sadmm_solve_batch(sadmm_t* hs, int32_t S, const void* const* ys, int32_t dtype, int32_t on_device,
                      sadmm_info* infos) {
  if (!hs || S < 1 || !ys) return SADMM_E_ARG;
  for (int i = 0; i < S; ++i) {
    if (!hs[i]) return SADMM_E_ARG;
    if (hs[i]->st != hs[0]->st)
      return fail_msg(hs[0], SADMM_E_ARG, "solve_batch: every handle must use the same storage");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail_msg(hs[0], SADMM_E_ARG, "solve_batch: handle repeated");
  }
  // scenes borrowing an operator whose source is not in the batch: the
  // source's factor must be valid before the data terms
  for (int i = 0; i < S; ++i) {
    const sadmm_t src = hs[i]->shared_src;
    if (!src) continue;
    bool in_batch = false;
    for (int j = 0; j < S; ++j) in_batch = in_batch || hs[j] == src;
    if (!in_batch) TRY(ensure_source_factor(hs[i]));
  }
  // inputs of every scene, then the factors of every (scene, sensor) in one
  // build per group of equal order and Gram path, then the data terms
  std::vector<std::vector<int>> rebuild(S);
  for (int i = 0; i < S; ++i) TRY(solve_prologue(hs[i], ys[i], dtype, on_device, &rebuild[i]));
  std::vector<bool> built(S, false);
  for (int i = 0; i < S; ++i) {
    if (built[i]) continue;
    std::vector<FacItem> items;
    for (int j = i; j < S; ++j) {
      if (built[j] || hs[j]->KMp != hs[i]->KMp || integer_gram(hs[j]) != integer_gram(hs[i])) continue;
      built[j] = true;
      for (int q : rebuild[j]) items.push_back({hs[j], q});
    }
    const int rc = build_factors_items(hs[i], items);
    if (rc != SADMM_OK) {
      for (int j = 0; j < S; ++j)
        if (hs[j] != hs[i]) hs[j]->err = hs[i]->err;
      return rc;
    }
  }
  for (int i = 0; i < S; ++i) TRY(solve_prologue_finish(hs[i]));
  std::vector<sadmm_t> v(hs, hs + S);
  // every scene on one FP32 operator: multi-right-hand-side products
  const sadmm_t root = hs[0]->shared_src ? hs[0]->shared_src : hs[0];
  bool shared = S >= 2 && S <= 64 && root->st == ST_FP32;
  for (int i = 0; i < S && shared; ++i)
    shared = (hs[i]->shared_src ? hs[i]->shared_src : hs[i]) == root && !hs[i]->p.prune;
  if (shared) {
    const int Q = root->Q, N = root->N, KMp = root->KMp;
    SharedBatch sb{};
    sb.S = S;
    sb.nch = (N + MRHS_CHUNK - 1) / MRHS_CHUNK;
    std::vector<void*> tmp;
    auto cleanup = [&]() { for (void* p : tmp) hipFree(p); };
    auto grab = [&](size_t bytes) -> void* {
      void* p = nullptr;
      if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
      tmp.push_back(p);
      return p;
    };
    sb.Vb = static_cast<float*>(grab(8 * (size_t)Q * N * S));
    sb.Tp = static_cast<float*>(grab(8 * (size_t)sb.nch * Q * KMp * S));
    sb.T64 = static_cast<cd*>(grab(16 * (size_t)Q * S * KMp));
    sb.Wt64 = static_cast<cd*>(grab(16 * (size_t)Q * S * KMp));
    sb.Wt32 = static_cast<float*>(grab(8 * (size_t)Q * S * KMp));
    MmDesc* wd = static_cast<MmDesc*>(grab(sizeof(MmDesc) * Q));
    if (!sb.Vb || !sb.Tp || !sb.T64 || !sb.Wt64 || !sb.Wt32 || !wd) {
      cleanup();
      return fail_msg(hs[0], SADMM_E_NOMEM, "solve_batch: shared-operator buffers");
    }
    std::vector<MmDesc> w(Q);
    for (int q = 0; q < Q; ++q)
      w[q] = MmDesc{root->W64[q], sb.T64 + (int64_t)q * S * KMp, sb.Wt64 + (int64_t)q * S * KMp,
                    KMp, S, KMp, KMp, KMp, KMp, 1.0, 0.0, 0.0};
    if (hipMemcpy(wd, w.data(), sizeof(MmDesc) * Q, hipMemcpyHostToDevice) != hipSuccess) {
      cleanup();
      return fail_msg(hs[0], SADMM_E_HIP, "solve_batch: descriptor upload");
    }
    sb.wdesc = wd;
    const int rc = iterate(v, false, &sb);
    hipStreamSynchronize(hs[0]->gs);
    cleanup();
    TRY(rc);
  } else {
    TRY(iterate(v, S == 1));
  }
  for (int i = 0; i < S; ++i) TRY(solve_epilogue(hs[i], infos ? &infos[i] : nullptr));
  return SADMM_OK;
}

int sadmm_get_image(sadmm_t h, void* xG, int32_t dtype, int32_t on_device) {
  if (!h) return SADMM_E_ARG;
  if (!xG || (dtype != SADMM_C128 && dtype != SADMM_C64)) return fail_msg(h, SADMM_E_ARG, "get_image: bad argument");
  if (!h->solved) return fail_msg(h, SADMM_E_STATE, "get_image: no solve yet");
  const size_t esz = dtype == SADMM_C128 ? 16 : 8;
  void* d = xG;
  if (!on_device) HIPCHK(h, hipMalloc(&d, esz * h->N));
  if (dtype == SADMM_C128) compute_to_c128(h->z, h->dbl, static_cast<double*>(d), h->N, h->s);
  else compute_to_c64(h->z, h->dbl, static_cast<float*>(d), h->N, h->s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(xG, d, esz * h->N, hipMemcpyDeviceToHost, h->s);
  if (e == hipSuccess) e = hipStreamSynchronize(h->s);
  if (!on_device) hipFree(d);
  if (e != hipSuccess) return fail_msg(h, SADMM_E_HIP, "get_image: %s", hipGetErrorString(e));
  return SADMM_OK;
}

int sadmm_get_sensor_image(sadmm_t h, int32_t q, void* xq, int32_t dtype, int32_t on_device) {
  if (!h) return SADMM_E_ARG;
  if (!xq || q < 0 || q >= h->Q || (dtype != SADMM_C128 && dtype != SADMM_C64))
    return fail_msg(h, SADMM_E_ARG, "get_sensor_image: bad argument");
  if (!h->solved) return fail_msg(h, SADMM_E_STATE, "get_sensor_image: no solve yet");
  const size_t esz = dtype == SADMM_C128 ? 16 : 8;
  void* d = xq;
  if (!on_device) HIPCHK(h, hipMalloc(&d, esz * h->N));
  const void* src = static_cast<const char*>(h->X) + h->csz * (size_t)q * h->N;
  if (dtype == SADMM_C128) compute_to_c128(src, h->dbl, static_cast<double*>(d), h->N, h->s);
  else compute_to_c64(src, h->dbl, static_cast<float*>(d), h->N, h->s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(xq, d, esz * h->N, hipMemcpyDeviceToHost, h->s);
  if (e == hipSuccess) e = hipStreamSynchronize(h->s);
  if (!on_device) hipFree(d);
  if (e != hipSuccess) return fail_msg(h, SADMM_E_HIP, "get_sensor_image: %s", hipGetErrorString(e));
  return SADMM_OK;
}

int sadmm_get_dual(sadmm_t h, void* u, int32_t dtype, int32_t on_device) {
  if (!h) return SADMM_E_ARG;
  if (!u || (dtype != SADMM_C128 && dtype != SADMM_C64)) return fail_msg(h, SADMM_E_ARG, "get_dual: bad argument");
  if (!h->solved) return fail_msg(h, SADMM_E_STATE, "get_dual: no solve yet");
  const size_t esz = dtype == SADMM_C128 ? 16 : 8;
  void* d = u;
  if (!on_device) HIPCHK(h, hipMalloc(&d, esz * h->N));
  if (dtype == SADMM_C128) compute_to_c128(h->u, h->dbl, static_cast<double*>(d), h->N, h->s);
  else compute_to_c64(h->u, h->dbl, static_cast<float*>(d), h->N, h->s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(u, d, esz * h->N, hipMemcpyDeviceToHost, h->s);
  if (e == hipSuccess) e = hipStreamSynchronize(h->s);
  if (!on_device) hipFree(d);
  if (e != hipSuccess) return fail_msg(h, SADMM_E_HIP, "get_dual: %s", hipGetErrorString(e));
  return SADMM_OK;
}

int sadmm_get_factor(sadmm_t h, int32_t q, void* W, int32_t* n) {
  if (!h) return SADMM_E_ARG;
  if (!W || !n || q < 0 || q >= h->Q) return fail_msg(h, SADMM_E_ARG, "get_factor: bad argument");
  if (!h->fac_valid[q] && !h->solved) return fail_msg(h, SADMM_E_STATE, "get_factor: no factor");
  if (h->direct[q]) {   // not kept in the direct form; built for the current active set
    TRY(build_factors(h, std::vector<int>{q}));
    h->fac_valid[q] = false;   // (the reuse check compares against the starting set)
  }
  TRY(ensure_w(h, q));
  *n = h->KM;
  HIPCHK(h, hipMemcpy2DAsync(W, 16 * (size_t)h->KM, h->W64[q], 16 * (size_t)h->KMp, 16 * (size_t)h->KM,
                             h->KM, hipMemcpyDeviceToHost, h->s));
  HIPCHK(h, hipStreamSynchronize(h->s));
  return SADMM_OK;
}

int sadmm_get_active_mask(sadmm_t h, int32_t q, uint8_t* mask) {
  if (!h) return SADMM_E_ARG;
  if (!mask || q < 0 || q >= h->Q) return fail_msg(h, SADMM_E_ARG, "get_active_mask: bad argument");
  HIPCHK(h, hipMemcpyAsync(mask, h->mask + (size_t)q * h->N, h->N, hipMemcpyDeviceToHost, h->s));
  HIPCHK(h, hipStreamSynchronize(h->s));
  return SADMM_OK;
}

int sadmm_get_active_indices(sadmm_t h, int32_t q, int32_t* idx, int32_t* count) {
  if (!h) return SADMM_E_ARG;
  if (!idx || !count || q < 0 || q >= h->Q) return fail_msg(h, SADMM_E_ARG, "get_active_indices: bad argument");
  *count = h->nq[q];
  if (h->nq[q] > 0)
    HIPCHK(h, hipMemcpyAsync(idx, h->J[q], sizeof(int) * h->nq[q], hipMemcpyDeviceToHost, h->s));
  HIPCHK(h, hipStreamSynchronize(h->s));
  return SADMM_OK;
}

int sadmm_get_history(sadmm_t h, int32_t which, double* out, int32_t cap, int32_t* count) {
  if (!h) return SADMM_E_ARG;
  if (!out || !count || which < 0 || which > 8 || cap < 0) return fail_msg(h, SADMM_E_ARG, "get_history: bad argument");
  if (!h->solved) return fail_msg(h, SADMM_E_STATE, "get_history: no solve yet");
  const int n = std::min(cap, h->hist_count);
  std::memcpy(out, h->hist_h.data() + (size_t)which * h->p.max_iter, sizeof(double) * n);
  *count = h->hist_count;
  return SADMM_OK;
}

int sadmm_matched_filter(sadmm_t h, const void* y, int32_t dtype, int32_t on_device, double* out) {
  if (!h) return SADMM_E_ARG;
  if (!y || !out || (dtype != SADMM_C128 && dtype != SADMM_C64)) return fail_msg(h, SADMM_E_ARG, "matched_filter: bad argument");
  for (int q = 0; q < h->Q; ++q)
    if (!h->op_set[q]) return fail_msg(h, SADMM_E_STATE, "matched_filter: operator %d not set", q);
  const size_t esz = dtype == SADMM_C128 ? 16 : 8;
  const void* ysrc = y;
  void* ystage = nullptr;
  if (!on_device) {
    HIPCHK(h, hipMalloc(&ystage, esz * (size_t)h->Q * h->KM));
    HIPCHK(h, hipMemcpyAsync(ystage, y, esz * (size_t)h->Q * h->KM, hipMemcpyHostToDevice, h->s));
    ysrc = ystage;
  }
  load_measurements(ysrc, dtype == SADMM_C128, h->Q, h->KM, h->KMp, h->yp, h->s);
  // full-operator descriptors for the matched filter
  for (int q = 0; q < h->Q; ++q) h->nq[q] = h->N;
  TRY(push_descs(h));
  launch_matched_filter(make_args(h), h->st, h->dbl, h->yp, h->mf, h->s);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(out, h->mf, sizeof(double) * (size_t)h->Q * h->N, hipMemcpyDeviceToHost, h->s));
  HIPCHK(h, hipStreamSynchronize(h->s));
  if (ystage) hipFree(ystage);
  h->solved = false;
  return SADMM_OK;
}

int sadmm_back_projection(sadmm_t h, const void* y, int32_t dtype, int32_t on_device, double* out) {
  if (!h) return SADMM_E_ARG;
  if (!y || !out || (dtype != SADMM_C128 && dtype != SADMM_C64))
    return fail_msg(h, SADMM_E_ARG, "back_projection: bad argument");
  for (int q = 0; q < h->Q; ++q)
    if (!h->op_set[q]) return fail_msg(h, SADMM_E_STATE, "back_projection: operator %d not set", q);
  const size_t esz = dtype == SADMM_C128 ? 16 : 8;
  const void* ysrc = y;
  void* ystage = nullptr;
  double* c = nullptr;
  auto release = [&]() {
    if (ystage) hipFree(ystage);
    if (c) hipFree(c);
  };
  if (hipMalloc((void**)&c, 16 * (size_t)h->Q * h->N) != hipSuccess) {
    c = nullptr;
    return fail_msg(h, SADMM_E_NOMEM, "back_projection: %zu bytes", 16 * (size_t)h->Q * h->N);
  }
  if (!on_device) {
    if (hipMalloc(&ystage, esz * (size_t)h->Q * h->KM) != hipSuccess) {
      ystage = nullptr;
      release();
      return fail_msg(h, SADMM_E_NOMEM, "back_projection: staging");
    }
    if (hipMemcpyAsync(ystage, y, esz * (size_t)h->Q * h->KM, hipMemcpyHostToDevice, h->s) != hipSuccess) {
      release();
      return fail_msg(h, SADMM_E_HIP, "back_projection: copy");
    }
    ysrc = ystage;
  }
  load_measurements(ysrc, dtype == SADMM_C128, h->Q, h->KM, h->KMp, h->yp, h->s);
  for (int q = 0; q < h->Q; ++q) h->nq[q] = h->N;
  int rc = push_descs(h);
  if (rc == SADMM_OK) {
    launch_matched_filter(make_args(h), h->st, h->dbl, h->yp, c, h->s, true);
    bp_sum(c, h->Q, h->N, h->mf, h->s);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(out, h->mf, sizeof(double) * (size_t)h->N, hipMemcpyDeviceToHost, h->s) != hipSuccess ||
        hipStreamSynchronize(h->s) != hipSuccess)
      rc = fail_msg(h, SADMM_E_HIP, "back_projection: launch failed");
  }
  release();
  h->solved = false;
  return rc;
}

int sadmm_stack_real(const void* src, int32_t dtype, int64_t rows, int64_t cols, int64_t ld, void* dst,
                     void* stream) {
  if (!src || !dst || rows < 1 || cols < 1 || ld < rows || (dtype != SADMM_C128 && dtype != SADMM_C64))
    return SADMM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  stack_real(src, dtype == SADMM_C128, rows, cols, ld, static_cast<double*>(dst), s);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SADMM_E_HIP;
  return SADMM_OK;
}

int sadmm_render_db(const void* img, int32_t is_complex, int64_t n, double range_db, int32_t on_device,
                    uint8_t* levels, void* stream) {
  if (!img || !levels || n < 1 || !(range_db > 0.0) || (is_complex != 0 && is_complex != 1))
    return SADMM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t ib = (is_complex ? 16 : 8) * (size_t)n;
  double thr[255];
  for (int L = 1; L <= 255; ++L) thr[L - 1] = std::pow(10.0, (L / 255.0 - 1.0) * range_db / 20.0);
  void* dimg = nullptr;
  double* dthr = nullptr;   // 255 thresholds + the maximum
  uint8_t* dout = nullptr;
  int rc = SADMM_OK;
  if (hipMalloc((void**)&dthr, sizeof(double) * 256) != hipSuccess) return SADMM_E_NOMEM;
  if (!on_device) {
    if (hipMalloc(&dimg, ib) != hipSuccess || hipMalloc((void**)&dout, (size_t)n) != hipSuccess) rc = SADMM_E_NOMEM;
    else if (hipMemcpyAsync(dimg, img, ib, hipMemcpyHostToDevice, s) != hipSuccess) rc = SADMM_E_HIP;
  }
  if (rc == SADMM_OK && hipMemcpyAsync(dthr, thr, sizeof(thr), hipMemcpyHostToDevice, s) != hipSuccess)
    rc = SADMM_E_HIP;
  if (rc == SADMM_OK) {
    const double* x = static_cast<const double*>(on_device ? img : dimg);
    uint8_t* o = on_device ? levels : dout;
    render_levels(x, is_complex != 0, n, dthr, dthr + 255, o, s);
    if (hipGetLastError() != hipSuccess) rc = SADMM_E_HIP;
    if (rc == SADMM_OK && !on_device &&
        hipMemcpyAsync(levels, dout, (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = SADMM_E_HIP;
    if (rc == SADMM_OK && hipStreamSynchronize(s) != hipSuccess) rc = SADMM_E_HIP;
  }
  if (dimg) hipFree(dimg);
  if (dout) hipFree(dout);
  hipFree(dthr);
  return rc;
}

int sadmm_set_pruning_cnn(sadmm_t h, sadmm_cnn_t cnn, double threshold) {
  if (!h) return SADMM_E_ARG;
  if (!cnn) { h->cnn = nullptr; return SADMM_OK; }
  int cq = 0, ch = 0, cw = 0;
  sadmm_cnn_shape(cnn, &cq, &ch, &cw);
  if (cq != h->Q || (int64_t)ch * cw != h->N)
    return fail_msg(h, SADMM_E_SHAPE, "set_pruning_cnn: CNN shape does not match Q x N");
  if (!(threshold > 0.0 && threshold <= 1.0)) return fail_msg(h, SADMM_E_ARG, "set_pruning_cnn: threshold");
  if (!h->p.kkt)
    return fail_msg(h, SADMM_E_ARG, "set_pruning_cnn: learned eliminations need the KKT re-check (kkt = 1)");
  h->cnn = cnn;
  h->cnn_thr = threshold;
  return SADMM_OK;
}

int sadmm_set_profiling(sadmm_t h, int32_t on) {
  if (!h) return SADMM_E_ARG;
  if (on < 0 || on > 2) return fail_msg(h, SADMM_E_ARG, "set_profiling: level 0, 1 or 2");
  h->prof = on != 0;
  h->prof_level = on;
  if (h->prof && h->evpool.empty()) {
    h->evpool.resize(8192);
    for (auto& e : h->evpool)
      if (hipEventCreate(&e) != hipSuccess) return fail_msg(h, SADMM_E_HIP, "set_profiling: event creation");
  }
  for (int i = 0; i < SADMM_KC_COUNT; ++i) { h->kt_ms[i] = 0.0; h->kt_n[i] = 0; h->kt_work[i] = 0.0; }
  h->marks.clear();
  h->evnext = 0;
  return SADMM_OK;
}

int sadmm_get_kernel_stats(sadmm_t h, int32_t kclass, int32_t* launches, double* total_ms,
                           double* work) {
  if (!h) return SADMM_E_ARG;
  if (kclass < 0 || kclass >= SADMM_KC_COUNT || !launches || !total_ms || !work)
    return fail_msg(h, SADMM_E_ARG, "get_kernel_stats: bad argument");
  *launches = h->kt_n[kclass];
  *total_ms = h->kt_ms[kclass];
  *work = h->kt_work[kclass];
  return SADMM_OK;
}

int sadmm_get_timing(sadmm_t h, int32_t which, double* ms) {
  if (!h) return SADMM_E_ARG;
  if (!ms || which < 0 || which > 2) return fail_msg(h, SADMM_E_ARG, "get_timing: bad argument");
  *ms = which == 0 ? h->t_total : (which == 1 ? h->t_factor : h->t_iter);
  return SADMM_OK;
}

void sadmm_destroy(sadmm_t h) {
  if (!h) return;
  if (h->shared_src) h->shared_src->n_sharers -= 1;
  if (h->s) hipStreamSynchronize(h->s);
  else hipDeviceSynchronize();
  for (void* p : h->allocs) hipFree(p);
  for (int q = 0; q < (int)h->Fd.size(); ++q) {
    if (h->Fd[q]) hipFree(h->Fd[q]);
    if (h->b0d[q]) hipFree(h->b0d[q]);
    if (h->rdir[q]) hipFree(h->rdir[q]);
  }
  for (void* p : {(void*)h->A64, (void*)h->dirD, (void*)h->dirX, (void*)h->dirT, (void*)h->dir_desc})
    if (p) hipFree(p);
  if (h->kg) hipFree(h->kg);
  for (double* p : h->rec)
    if (p) hipFree(p);
  for (unsigned long long* p : h->rmaxc)
    if (p) hipFree(p);
  for (void* p : {(void*)h->sens_mf_d, (void*)h->gfix, h->g32, h->xfix, (void*)h->re1, (void*)h->re2,
                  (void*)h->rw, (void*)h->gprev, (void*)h->dg, h->xprev})
    if (p) hipFree(p);
  if (h->ctl_h) hipHostFree(h->ctl_h);
  if (h->dg_h) hipHostFree(h->dg_h);
  if (h->counts_h) hipHostFree(h->counts_h);
  if (h->halt_h) hipHostFree(h->halt_h);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  if (h->evf0) hipEventDestroy(h->evf0);
  if (h->evf1) hipEventDestroy(h->evf1);
  for (auto& e : h->evpool) hipEventDestroy(e);
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  if (h->graph) hipGraphDestroy(h->graph);
  if (h->gs) { hipStreamSynchronize(h->gs); hipStreamDestroy(h->gs); }
  delete h;
}

const char* sadmm_last_error(sadmm_t h) { return h ? h->err.c_str() : g_create_err.c_str(); }

}  // extern "C"
